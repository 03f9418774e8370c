"""Pins for the FP64 GRAPE oracle: propagators (Eq. (3)), objective (Eq. (4)), exact
gradient and its first-order form (Eq. (B2)), against routes that share no arithmetic."""
import numpy as np
import pytest
from scipy.linalg import expm

import qoc_workloads as W
from oracle import closed_form, fd, grape


def _plain_states(blocks, rng):
    mA1 = blocks[0]["m"]
    pf = W.gaussian_panel(rng, mA1)
    psif = [pf[:, None]] + [np.zeros((b["m"], b["d"]), complex) for b in blocks[1:]]
    psi0 = [np.eye(mA1, dtype=complex)[:, [0]]] + [np.zeros((b["m"], b["d"]), complex) for b in blocks[1:]]
    return psi0, psif


def _all_states(blocks, rng):
    sizes = [b["m"] * b["d"] for b in blocks]
    vf = W.gaussian_panel(rng, sum(sizes))
    v0 = W.gaussian_panel(rng, sum(sizes))
    out0, outf, off = [], [], 0
    for b, s in zip(blocks, sizes):
        outf.append(vf[off:off + s].reshape(b["d"], b["m"]).T)
        out0.append(v0[off:off + s].reshape(b["d"], b["m"]).T)
        off += s
    return out0, outf


@pytest.fixture(scope="module")
def config1_results():
    w = W.config1()
    rng = w.notes["rng"]
    blocks = grape.block_system(6, w.h0, w.hk)
    psi0, psif = _plain_states(blocks, rng)
    dense = grape.dense_system(6, w.h0, w.hk)
    d0 = grape.dense_from_panels(blocks, psi0)
    df = grape.dense_from_panels(blocks, psif)
    rb = grape.fidelity_grad(blocks, w.u, w.dt, psi0, psif)
    rd = grape.fidelity_grad(dense, w.u, w.dt, [d0[:, None]], [df[:, None]])
    return w, blocks, psi0, psif, df, rb, rd


def test_unitarity():
    w = W.config1(N=5)
    for blk in grape.block_system(6, w.h0, w.hk) + grape.dense_system(6, w.h0, w.hk):
        for j in range(5):
            U = grape.propagator(blk["H0"], blk["Hk"], w.u[j], w.dt)
            assert np.abs(U.conj().T @ U - np.eye(U.shape[0])).max() < 1e-13


def test_propagator_matches_library_expm():
    w = W.config1(N=3)
    blk = grape.dense_system(6, w.h0, w.hk)[0]
    for j in range(3):
        H = blk["H0"] + sum(w.u[j, k] * blk["Hk"][k] for k in range(2))
        assert np.abs(grape.propagator(blk["H0"], blk["Hk"], w.u[j], w.dt) - expm(-1j * w.dt * H)).max() < 1e-13


def test_config1_dense_vs_block(config1_results):
    w, blocks, psi0, psif, df, rb, rd = config1_results
    assert abs(rb["F"] - rd["F"]) < 1e-13
    assert np.abs(rb["grad"] - rd["grad"]).max() < 1e-14
    assert 0.0 < rb["F"] < 1.0


def test_config1_su2_closed_form(config1_results):
    """Independent route: product of 2x2 rotations times the coupling phase."""
    w, blocks, psi0, psif, df, rb, rd = config1_results
    rc = closed_form.fidelity_grad(6, 0.5, 1.0, [("x", 1.0), ("y", 1.0)], w.u, w.dt, df)
    assert abs(rc["F"] - rd["F"]) < 1e-13
    assert np.abs(rc["grad"] - rd["grad"]).max() < 1e-14


def test_fd_matches_exact_gradient(config1_results):
    w, blocks, psi0, psif, df, rb, rd = config1_results
    ent = [(0, 0), (17, 1), (99, 0), (150, 1), (199, 1)]
    g_fd = fd.fd_gradient(blocks, w.u, w.dt, psi0, psif, ent, h=1e-4)
    g = np.array([rb["grad"][j, k] for j, k in ent])
    assert np.abs(g_fd - g).max() < 1e-10


def test_overlap_invariant_along_sweep():
    w = W.config1(N=20)
    blocks = grape.block_system(6, w.h0, w.hk)
    psi0, psif = _all_states(blocks, np.random.default_rng(5))
    fw, bw = grape.sweeps(blocks, w.u, w.dt, psi0, psif)
    ovs = [sum(np.sum(np.conj(bw[b][j]) * fw[b][j]) for b in range(len(blocks))) for j in range(21)]
    assert np.abs(np.array(ovs) - ovs[-1]).max() < 1e-14


def test_zero_controls_single_exponential():
    """u = 0: the product of slices is exp(-i N dt H0), one exponential of the whole pulse."""
    w = W.config1(N=30)
    u = np.zeros_like(w.u)
    blocks = grape.block_system(6, w.h0, w.hk)
    psi0, psif = _all_states(blocks, np.random.default_rng(1))
    r = grape.fidelity_grad(blocks, u, w.dt, psi0, psif)
    o = 0
    for b, blk in enumerate(blocks):
        o += np.sum(np.conj(psif[b]) * (expm(-1j * 30 * w.dt * blk["H0"]) @ psi0[b]))
    assert abs(r["F"] - abs(o) ** 2) < 1e-13


def test_single_slice_frechet():
    """N = 1: the gradient is the directional derivative of one exponential, checked with
    scipy's Frechet derivative of expm (Al-Mohy-Higham)."""
    from scipy.linalg import expm_frechet
    w = W.config1(N=1)
    blk = grape.dense_system(6, w.h0, w.hk)[0]
    rng = np.random.default_rng(3)
    p0 = W.gaussian_panel(rng, 64)[:, None]
    pf = W.gaussian_panel(rng, 64)[:, None]
    r = grape.fidelity_grad([blk], w.u, w.dt, [p0], [pf])
    X = -1j * w.dt * (blk["H0"] + sum(w.u[0, k] * blk["Hk"][k] for k in range(2)))
    U = expm(X)
    o = np.vdot(pf, U @ p0)
    for k in range(2):
        L = expm_frechet(X, -1j * w.dt * blk["Hk"][k], compute_expm=False)
        g = 2 * np.real(np.conj(o) * np.vdot(pf, L @ p0))
        assert abs(g - r["grad"][0, k]) < 1e-13


def test_uncoupled_ring_is_product_of_rotations():
    """J = 0: the closed form with no coupling phase equals the dense computation."""
    n = 4
    w = W.config1(N=25)
    h0 = [W.one_body(0.5, "z")]
    dense = grape.dense_system(n, h0, w.hk)
    rng = np.random.default_rng(2)
    pf = W.gaussian_panel(rng, 2 ** n)
    p0 = np.zeros(2 ** n, complex)
    p0[0] = 1
    rd = grape.fidelity_grad(dense, w.u, w.dt, [p0[:, None]], [pf[:, None]])
    rc = closed_form.fidelity_grad(n, 0.5, 0.0, [("x", 1.0), ("y", 1.0)], w.u, w.dt, pf)
    assert abs(rd["F"] - rc["F"]) < 1e-13
    assert np.abs(rd["grad"] - rc["grad"]).max() < 1e-14


def test_first_order_limit():
    """Eq. (B2): as dt -> 0 the exact gradient approaches the first-order form, with
    an error that shrinks linearly in dt."""
    errs = []
    for dt in (0.02, 0.01, 0.005):
        w = W.config1(N=12)
        blocks = grape.block_system(6, w.h0, w.hk)
        psi0, psif = _all_states(blocks, np.random.default_rng(4))
        ge = grape.fidelity_grad(blocks, w.u, dt, psi0, psif)["grad"]
        ga = grape.first_order_gradient(blocks, w.u, dt, psi0, psif)
        errs.append(np.abs(ge - ga).max() / np.abs(ge).max())
    assert errs[0] > errs[1] > errs[2]
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4


@pytest.mark.parametrize("stride,K", [(1, 2), (2, 4)])
def test_all_blocks_dense_vs_block_nondegenerate(stride, K):
    """Every block carries state; staggered controls (stride 2) leave only the two-site group."""
    n = 6
    w = W.config4(N=15, n=n) if stride == 2 else W.config1(N=15)
    h0 = W.heisenberg_ring_terms(0.9, 0.5) + [W.ring_pair(0.3, "zz", 2)]
    hk = w.hk[:K]
    blocks = grape.block_system(n, h0, hk, "dihedral", stride)
    psi0, psif = _all_states(blocks, np.random.default_rng(7))
    d0 = grape.dense_from_panels(blocks, psi0)
    df = grape.dense_from_panels(blocks, psif)
    rb = grape.fidelity_grad(blocks, w.u, w.dt, psi0, psif)
    rd = grape.fidelity_grad(grape.dense_system(n, h0, hk), w.u, w.dt, [d0[:, None]], [df[:, None]])
    assert abs(rb["F"] - rd["F"]) < 1e-13
    assert np.abs(rb["grad"] - rd["grad"]).max() < 1e-14


def test_symmetric_blocks_vs_dense():
    n = 5
    h0 = [W.one_body(1.0, "z"), W.all_pairs(0.1, "xx"), W.all_pairs(0.05, "yy")]
    hk = [[W.one_body(1.0, "x")], [W.one_body(1.0, "y")]]
    rng = np.random.default_rng(11)
    u = rng.uniform(-1, 1, (20, 2))
    blocks = grape.block_system(n, h0, hk, "symmetric")
    dense = grape.dense_system(n, h0, hk)
    # top block only: psi0 = |J,J> = all-up, psi_f a random Dicke superposition
    pf = W.gaussian_panel(rng, n + 1)
    psi0 = [np.eye(n + 1, dtype=complex)[:, [0]]] + [np.zeros((b["m"], 1), complex) for b in blocks[1:]]
    psif = [pf[:, None]] + [np.zeros((b["m"], 1), complex) for b in blocks[1:]]
    from math import comb
    D = np.zeros((2 ** n, n + 1))
    for x in range(2 ** n):
        w_ = bin(x).count("1")
        D[x, w_] = 1 / np.sqrt(comb(n, w_))
    rb = grape.fidelity_grad(blocks, u, 0.05, psi0, psif)
    rd = grape.fidelity_grad(dense, u, 0.05, [D[:, [0]].astype(complex)], [(D @ pf)[:, None]])
    assert abs(rb["F"] - rd["F"]) < 1e-13
    assert np.abs(rb["grad"] - rd["grad"]).max() < 1e-14
