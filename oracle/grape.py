"""GRAPE objective and exact gradient, FP64, dense or block-reduced (Eqs. (1)-(4); App. B).

Slice convention (Eq. (3)): u[j, k] is the control sample of slice j
(the midpoint value of Eq. (3)), j = 0..N-1 applied first to last:
    H_j = H0 + sum_k u[j,k] H_k,   U_j = exp(-i dt H_j),   psi_{j+1} = U_j psi_j.
Objective (Eq. (4)): o = <psi_f|psi_N>; F = |o|^2 / (||psi_N||^2 ||psi_f||^2), which
equals |o|^2 for normalised states because every U_j is unitary.
Costates: lambda_N = psi_f, lambda_j = U_j^dagger lambda_{j+1}; then
o = <lambda_{j+1}| U_j |psi_j> for every j.
Gradient: dF/du[j,k] = 2 Re(conj(o) <lambda_{j+1}| dU_j/du_k |psi_j>) / (||psi_N||^2 ||psi_f||^2),
with the exact derivative of the matrix exponential written through the eigen-
decomposition H_j = V diag(e) V^dagger (Daleckii-Krein):
    dU_j/du_k = V [ (V^dagger H_k V) o Gamma ] V^dagger,
    Gamma_ab = -i dt exp(-i dt (e_a + e_b)/2) sinc(dt (e_a - e_b)/2),   sinc(0) = 1.
Eq. (B2) of the paper keeps only the first-order term -i dt H_k U_j; that form
is available as ``first_order_gradient`` and is the dt -> 0 limit of the above.

A "system" is a list of blocks; block b has H0 (m x m), Hk (list of m x m) and
state panels psi0[b], psif[b] of shape (m, d_b) (one column per copy).  The
dense computation is the one-block system of the full 2^n space.
"""
from __future__ import annotations

import numpy as np


def slice_hamiltonian(H0, Hk, uj):
    H = np.array(H0, dtype=complex, copy=True)
    for k, Hkk in enumerate(Hk):
        H = H + uj[k] * Hkk
    return H


def eig_slice(H0, Hk, uj):
    H = slice_hamiltonian(H0, Hk, uj)
    H = 0.5 * (H + H.conj().T)
    e, V = np.linalg.eigh(H)
    return e, V


def propagator(H0, Hk, uj, dt):
    e, V = eig_slice(H0, Hk, uj)
    return (V * np.exp(-1j * dt * e)) @ V.conj().T


def gamma_matrix(e, dt):
    ea = e[:, None]
    eb = e[None, :]
    return -1j * dt * np.exp(-1j * dt * (ea + eb) / 2.0) * np.sinc(dt * (ea - eb) / (2.0 * np.pi))


def derivative_contractions(e, V, Hk, lam, psi, dt):
    """[<lam| dU/du_k |psi>] over k, summed over the panel's columns."""
    lt = V.conj().T @ lam
    pt = V.conj().T @ psi
    Gm = gamma_matrix(e, dt)
    out = []
    for Hkk in Hk:
        D = (V.conj().T @ Hkk @ V) * Gm
        out.append(np.sum(lt.conj() * (D @ pt)))
    return np.array(out)


def fidelity_grad(blocks, u, dt, psi0, psif, keep_states=False):
    """F, |o|^2, o, ||psi_N||^2 and the exact gradient (N, K) for a block system."""
    u = np.asarray(u, dtype=float)
    N, K = u.shape
    nb = len(blocks)
    states = []
    psiN = []
    eig_cache = []
    cache_ok = sum(b["H0"].shape[0] ** 2 for b in blocks) * N * 16 < 2 * 1024 ** 3
    for b in range(nb):
        H0, Hk = blocks[b]["H0"], blocks[b]["Hk"]
        psi = np.array(psi0[b], dtype=complex)
        traj = [psi] if keep_states else None
        cache = []
        for j in range(N):
            e, V = eig_slice(H0, Hk, u[j])
            if cache_ok:
                cache.append((e, V))
            psi = (V * np.exp(-1j * dt * e)) @ (V.conj().T @ psi)
            if keep_states:
                traj.append(psi)
        psiN.append(psi)
        states.append(traj)
        eig_cache.append(cache)
    o = sum(np.sum(np.conj(psif[b]) * psiN[b]) for b in range(nb))
    nN = sum(float(np.sum(np.abs(psiN[b]) ** 2)) for b in range(nb))
    nf = sum(float(np.sum(np.abs(psif[b]) ** 2)) for b in range(nb))
    g = np.zeros((N, K), dtype=complex)
    # backward sweep: lambda_{j+1} is held while slice j is differentiated, then stepped back
    for b in range(nb):
        H0, Hk = blocks[b]["H0"], blocks[b]["Hk"]
        lam = np.array(psif[b], dtype=complex)
        # psi_j is needed again: re-run the forward states unless stored
        if keep_states:
            traj = states[b]
        else:
            traj = [np.array(psi0[b], dtype=complex)]
            for j in range(N):
                e, V = eig_cache[b][j] if cache_ok else eig_slice(H0, Hk, u[j])
                traj.append((V * np.exp(-1j * dt * e)) @ (V.conj().T @ traj[-1]))
        for j in range(N - 1, -1, -1):
            e, V = eig_cache[b][j] if cache_ok else eig_slice(H0, Hk, u[j])
            g[j] += derivative_contractions(e, V, Hk, lam, traj[j], dt)
            lam = (V * np.exp(1j * dt * e)) @ (V.conj().T @ lam)
    norm = nN * nf
    grad = 2.0 * np.real(np.conj(o) * g) / norm
    res = {"F": abs(o) ** 2 / norm, "F_raw": abs(o) ** 2, "o": o, "normN2": nN, "normf2": nf,
           "grad": grad, "psiN": psiN}
    if keep_states:
        res["states"] = states
    return res


def sweeps(blocks, u, dt, psi0, psif):
    """Forward states psi_j (j = 0..N) and costates lambda_j (j = 0..N) per block."""
    u = np.asarray(u, dtype=float)
    N = u.shape[0]
    fw, bw = [], []
    for b, blk in enumerate(blocks):
        Us = [propagator(blk["H0"], blk["Hk"], u[j], dt) for j in range(N)]
        ps = [np.array(psi0[b], dtype=complex)]
        for j in range(N):
            ps.append(Us[j] @ ps[-1])
        ls = [None] * (N + 1)
        ls[N] = np.array(psif[b], dtype=complex)
        for j in range(N - 1, -1, -1):
            ls[j] = Us[j].conj().T @ ls[j + 1]
        fw.append(ps)
        bw.append(ls)
    return fw, bw


def first_order_gradient(blocks, u, dt, psi0, psif):
    """Gradient with the first-order derivative of Eq. (B2): dU_j/du_k ~ -i dt H_k U_j."""
    fw, bw = sweeps(blocks, u, dt, psi0, psif)
    N, K = np.asarray(u).shape
    o = sum(np.sum(np.conj(psif[b]) * fw[b][N]) for b in range(len(blocks)))
    nN = sum(float(np.sum(np.abs(fw[b][N]) ** 2)) for b in range(len(blocks)))
    nf = sum(float(np.sum(np.abs(psif[b]) ** 2)) for b in range(len(blocks)))
    g = np.zeros((N, K), dtype=complex)
    for b, blk in enumerate(blocks):
        for j in range(N):
            for k, Hkk in enumerate(blk["Hk"]):
                g[j, k] += np.sum(np.conj(bw[b][j + 1]) * (-1j * dt) * (Hkk @ fw[b][j + 1]))
    return 2.0 * np.real(np.conj(o) * g) / (nN * nf)


# ----------------------------------------------------------------------------- systems
def dense_system(n, h0_terms, hk_terms):
    from . import pauli
    H0 = pauli.hamiltonian(n, h0_terms).toarray()
    Hk = [pauli.hamiltonian(n, t).toarray() for t in hk_terms]
    return [{"label": "dense", "m": 2 ** n, "d": 1, "H0": H0, "Hk": Hk}]


def block_system(n, h0_terms, hk_terms, group="dihedral", stride=1, route="convention"):
    """Blocks A_theta^dagger H A_theta in block order, with the isometries that define them."""
    from . import basis, counts, pauli
    if group == "symmetric":
        H0b = basis.sn_blocks(n, h0_terms)
        Hkb = [basis.sn_blocks(n, t) for t in hk_terms]
        out = []
        for i, (twoJ, H0) in enumerate(H0b):
            out.append({"label": f"J{twoJ}/2", "m": twoJ + 1, "d": 1, "H0": H0,
                        "Hk": [Hkb[k][i][1] for k in range(len(hk_terms))]})
        return out
    reflection = group == "dihedral"
    L = n // stride
    H0 = pauli.hamiltonian(n, h0_terms)
    Hk = [pauli.hamiltonian(n, t) for t in hk_terms]
    out = []
    for lab in counts.irrep_labels(L, reflection):
        if route == "convention":
            Vs, reps = basis.convention_basis(n, lab, stride, reflection)
        else:
            Vs, reps = basis.projector_basis(n, lab, stride, reflection), None
        m = Vs[0].shape[1]
        if m == 0:
            continue
        out.append({"label": lab, "m": m, "d": len(Vs), "V": Vs, "reps": reps,
                    "H0": basis.project(H0, Vs[0]),
                    "Hk": [basis.project(h, Vs[0]) for h in Hk]})
    return out


def panels_from_dense(blocks, psi):
    return [np.stack([V.conj().T @ psi for V in blk["V"]], axis=1) for blk in blocks]


def dense_from_panels(blocks, panels):
    out = 0
    for blk, P in zip(blocks, panels):
        for c, V in enumerate(blk["V"]):
            out = out + V @ P[:, c]
    return out
