#!/usr/bin/env python3
"""GRAPE slices*blocks/s (objective + exact gradient) on one MI355X.

Workload (synthetic, seeded): 12-qubit Heisenberg ring H0 = 0.5 sum sz + J sum (xx+yy+zz)
with J ~ U[0.5, 1.5], two global controls u_x sum sx, u_y sum sy with u ~ U[-2, 2],
N = 1000 slices of dt = 0.02, block-reduced under D_12 (9 distinct irreducible blocks,
128..346 wide; E blocks carry two copies); psi0 and psi_f are independent normalised
complex Gaussians over every block, so every block carries work.

One step = one full hot-path call: all slice propagators (complex64 MFMA, FP64 norms),
forward sweep, objective (FP64), backward sweep and exact gradient (FP64 accumulation).
value = (slices x distinct blocks) per second of the timed steps.  The FP64 (complex128)
path is timed beside it.  The roofline entry covers the dominant kernel, the propagator
GEMM: algorithmic flops 8 m^3 per complex m x m product (4 m^2 (m + 1) for the Hermitian
powers of the generator, whose upper triangle is a mirror image), with the products each
slice needs for its (degree, squarings) choice, over its summed launch time measured with
HIP events on the launch stream during the timed steps.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MFMA_PEAK = {"c64": 157.3, "c128": 78.6}  # dense FP32 / FP64 matrix TFLOP/s, MI355X

# HBM-side bytes of k_expm_step<float> on this workload, from two rocprofv3 --pmc runs per
# tile variant (FETCH_SIZE, then WRITE_SIZE; mean KiB per dispatch over the 6 dispatches of
# the timed step of `bench.py --steps 1 --warmup 1 --fp64-steps 0 --no-cpu-baseline
# --copy-calibration 256 --gemm-variant32 V --sym-candidates 0 --ring14-slices 0
# --batch-problems 0 --dense-slices 0 --paper-comparison 0 --optimizer 0 --gate 0 --lts 0`
# for the two variants the autotuner picks between here), each scaled by what the same
# counter reads for the 256 MiB calibration copy (FETCH_SIZE reads half of the bytes
# copied: x2.0; WRITE_SIZE all of them: x1.0).  Valid only for the kernel sources they
# were taken with (sha1 of mfma_tile.h + grape.hip).
TRAFFIC = {"sources_sha1": "085f90a56709576932e5fc8ab3b7cb87e9b5e984", "fetch_scale": 2.0, "write_scale": 1.0,
           "kib": {"fp32 64x128": (9226842.5, 3146659.8), "fp32 128x64": (8436696.0, 3534275.5)}}


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in ("mfma_tile.h", "grape.hip"):
        with open(os.path.join(ROOT, "paper_2309_05884_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--cpu-slices", type=int, default=128,
                    help="oracle sample size on all host cores (slices, all blocks)")
    ap.add_argument("--cpu-slices-1t", type=int, default=16, help="oracle sample size on one host thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sym-candidates", type=int, default=1024,
                    help="S_128 candidate pulses timed in one batched plan (0: skip; 1024 = the full workload)")
    ap.add_argument("--ring14-slices", type=int, default=4000,
                    help="slices of the 14-qubit staggered-control ring timed (0: skip; 4000 = the full pulse)")
    ap.add_argument("--batch-problems", type=int, default=256,
                    help="problems of the 256-ring batched workload timed in one plan (0: skip; 256 = all, "
                         "about 3 minutes per step)")
    ap.add_argument("--dense-slices", type=int, default=16,
                    help="slices of the same pulse timed on the dense 4096-dim space (0: skip)")
    ap.add_argument("--paper-comparison", type=int, default=14, metavar="NMAX",
                    help="also time the transfer all-up -> all-down for n = 3..NMAX qubits on the dense "
                         "space (n <= 12), the first D_n block and (no coupling) the first S_n block "
                         "(0: skip)")
    ap.add_argument("--gate", type=int, default=1,
                    help="also time the unitary of the whole pulse and the gate fidelity (1) or skip (0)")
    ap.add_argument("--lts", type=int, default=1,
                    help="also run the Trotterised per-qubit-control legs (1) or skip them (0)")
    ap.add_argument("--optimizer", type=int, default=1,
                    help="also run the L-BFGS GRAPE optimiser legs (1) or skip them (0)")
    ap.add_argument("--gemm-variant32", type=int, default=-1, metavar="V",
                    help="run the headline FP32 plan in tile variant V instead of the autotuner's choice (for "
                         "hardware-counter runs of one variant; -1: autotune)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of this many MiB (a known-size kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def build_problem(q, W, torch):
    w = W.config2(seed=0, variant="all")
    rng = w.notes["rng"]
    B = q.Basis(12, "dihedral", 1)
    S = q.System(B, w.h0, w.hk)
    vf = W.gaussian_panel(rng, B.dim)
    v0 = W.gaussian_panel(rng, B.dim)
    dev = dict(u=torch.tensor(w.u, device="cuda"), psi0=torch.tensor(v0, device="cuda"),
               psif=torch.tensor(vf, device="cuda"))
    return w, B, S, v0, vf, dev


def timed_steps(q, torch, plan, dev, steps, warmup):
    for _ in range(warmup):
        q.fidelity_grad(plan, dev["u"], dev["psi0"], dev["psif"])
    torch.cuda.synchronize()
    q.profile_begin(steps * 4096)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        out, grad = q.fidelity_grad(plan, dev["u"], dev["psi0"], dev["psif"], check=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = q.profile_end()
    q.check_flags(out)
    return e0.elapsed_time(e1) / steps, wall, prof, out, grad


def _product_flops(m, qs, ss, r, pow_free=0):
    """Algorithmic flops of the propagator products of one block over its slices.  A
    general complex m x m product is 8 m^3; the powers Y^2..Y^r of the skew-Hermitian
    generator are (skew-)Hermitian, so only their lower triangle with the diagonal,
    4 m^2 (m + 1), is work.  Degree-12 scheme (q = 0): 2 power products, then 2 + s general
    ones; Paterson-Stockmeyer degree q r: r - 1 powers, then q - 1 + s general.  The
    pow_free powers the generator forms from the operator products (Y^2, Y^3) are no
    products."""
    herm = 4.0 * m * m * (m + 1)
    full = 8.0 * m ** 3
    npow = np.maximum(np.where(qs == 0, 2, r - 1) - pow_free, 0)
    ngen = np.where(qs == 0, 2 + ss, (qs - 1) + ss)
    return float((npow * herm + ngen * full).sum())


def gemm_flops(q, plan, dev, sizes):
    """Algorithmic flops of the propagator GEMMs of one call (see _product_flops)."""
    qs, ss, _ = q.slice_stats(plan, dev["u"])
    r, pf = plan.info["taylor_step"], plan.info["powers_from_generator"]
    tot = sum(_product_flops(m, qs[b], ss[b], r, pf) for b, m in enumerate(sizes))
    return tot, qs, ss


def gemm_flops_jobs(q, plan, u_flat, job_sizes):
    """gemm_flops for any plan: job_sizes lists m per (problem, block) job in plan order."""
    qs, ss, _ = q.slice_stats(plan, u_flat)
    r, pf = plan.info["taylor_step"], plan.info["powers_from_generator"]
    tot = 0.0
    for b, m in enumerate(job_sizes):
        valid = qs[b] >= 0
        tot += _product_flops(m, qs[b][valid], ss[b][valid], r, pf)
    return tot


def executed_flops_jobs(q, plan, u_flat, job_sizes, job_problem=None):
    """(algorithmic, executed) propagator GEMM flops of one fidelity+gradient call: the
    executed count adds the slices recomputed in the backward sweep of a segmented plan or
    problem group (a job recomputes every segment of its group before its own last one).
    job_problem: the problem of each job (batched plans)."""
    qs, ss, _ = q.slice_stats(plan, u_flat)
    r, pf = plan.info["taylor_step"], plan.info["powers_from_generator"]
    groups = plan.groups()
    alg = ex = 0.0
    for b, m in enumerate(job_sizes):
        p = 0 if job_problem is None else job_problem[b]
        L = [sl for (p0, sl, _) in groups if p0 <= p][-1]
        valid = np.where(qs[b] >= 0)[0]
        if valid.size == 0:
            continue
        f = _product_flops(m, qs[b][valid], ss[b][valid], r, pf)
        nj = int(valid.size)
        last_start = ((nj - 1) // L) * L
        alg += f
        ex += f + (_product_flops(m, qs[b][:last_start], ss[b][:last_start], r, pf) if last_start > 0 else 0.0)
    return alg, ex


def golden_values(name):
    """(scalars, gradient) stored by tests/golden/make_golden.py (FP64 oracle), or None."""
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    vals, grad = {}, []
    for line in open(path):
        if line.startswith("#"):
            continue
        k, *v = line.split()
        # values are Python float reprs (older files: numpy scalar reprs)
        num = [float(x.replace("np.float64(", "").rstrip(")")) for x in v]
        if k == "g":
            grad.append(num)
        else:
            vals[k] = num[0]
    return vals, np.array(grad)


def parity(name, F, grad):
    """|dF| and gradient error of one result against the stored oracle values `name`."""
    gv = golden_values(name)
    if gv is None:
        return None
    vals, gref = gv
    g = np.asarray(grad)
    gmax = float(np.abs(gref).max())
    dg = float(np.abs(g - gref).max())
    return {"oracle": name, "dF": abs(float(F) - vals["F"]), "max_grad_err": dg,
            "grad_err_rel_to_max": dg / gmax if gmax > 0 else None}


def one_step(torch, run):
    """Milliseconds of one call of run(), HIP events on the current stream."""
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    res = run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), res


def profiled_leg(q, torch, plan, run, steps, warmup, u_flat, job_sizes, units, precision="c64", job_problem=None,
                 launches_per_step=8192):
    """Time `steps` calls of run() after `warmup`, with the library's per-kernel events;
    returns throughput and the propagator GEMM's fraction of the MFMA peak.  The plan's
    workspace is allocated before the timed region (set-up, not part of a step)."""
    plan.workspace()
    torch.cuda.synchronize()
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    q.profile_begin(steps * launches_per_step)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    prof = q.profile_end()
    ms = e0.elapsed_time(e1) / steps
    flops, ex_flops = executed_flops_jobs(q, plan, u_flat, job_sizes, job_problem)
    gemm_ms, gemm_n = prof["propagator_gemm"]
    tf = flops * steps / (gemm_ms * 1e-3) / 1e12
    tfx = ex_flops * steps / (gemm_ms * 1e-3) / 1e12
    return {"ms_per_step": ms, "value": units / (ms * 1e-3), "unit": "slices*blocks/s",
            "gemm_tflops": tf, "gemm_frac": tf / MFMA_PEAK[precision],
            "gemm_tflops_with_recompute": tfx, "gemm_frac_with_recompute": tfx / MFMA_PEAK[precision],
            "gemm_ms_per_step": gemm_ms / steps, "gemm_launches_per_step": gemm_n / steps,
            "gemm_variant": plan.variant_name, "steps": steps, "warmup": warmup, "segments": plan.info["segments"],
            "segment_slices": plan.info["segment"], "problem_groups": plan.info["problem_groups"],
            "groups_segmented": sum(1 for g in plan.groups() if g[2] > 1), "workspace_gb": plan.workspace_bytes / 1e9,
            "kernel_ms_per_step": {k: v[0] / steps for k, v in prof.items() if v[1]}}


def paper_comparison(q, torch, W, nmax, N=100, dt=0.05, dense_max=12, steps=2):
    """Milliseconds per fidelity+gradient step of the transfer all-up -> all-down (the
    runtime comparison of the paper's Sec. II B, Fig. 3a/b): on the dense 2^n space (n <= dense_max),
    on the first D_n block alone, and, without coupling, on the first S_n block alone.
    Eq. (5) with B_z = 1 and c_cpl = 0 (no coupling) or 1 (nearest neighbours), and Eq. (7)
    with B_z = 1 and c^(d) = 1/d for d = 1 .. floor(n/2) (full coupling, D_n only); global
    controls of Eq. (6); N slices of dt; a resonant circular pi pulse (u_x, u_y) =
    (pi / T)(cos t, sin t) at the slice midpoints t, T = N dt, which flips each free qubit,
    plus seeded U[-0.05, 0.05] noise on both controls, so that F is far from 0 (about 0.995
    at n = 14 without coupling); complex64 plans."""
    def timed(B, h0, hk, u, blocks, psi, key, e):
        """Eager step time under e[key + "_ms"]; for blocks of a few hundred or less, where
        launch latency dominates, also the replay time of the step captured in a HIP graph
        under e[key + "_graph_ms"].  Returns F."""
        S = q.System(B, h0, hk)
        P = q.Plan(S, "c64", N, dt, 1.0, blocks=blocks)
        out, _ = q.fidelity_grad(P, u, psi[0], psi[1], check=False)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            out, _ = q.fidelity_grad(P, u, psi[0], psi[1], check=False)
        e1.record()
        torch.cuda.synchronize()
        q.check_flags(out)
        e[key + "_ms"] = e0.elapsed_time(e1) / steps
        F = out[0].item()
        if e[key + "_m"] <= 512:
            cap = q.CapturedStep(P, u, psi[0], psi[1])
            reps = 20
            cap.replay()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                gout, _ = cap.replay()
            e1.record()
            torch.cuda.synchronize()
            q.check_flags(gout)
            e[key + "_graph_ms"] = e0.elapsed_time(e1) / reps
            assert abs(gout[0].item() - F) <= 1e-6, (key, gout[0].item(), F)
        return F

    def unit(n, i, length):
        v = torch.zeros(length, dtype=torch.complex128, device="cuda")
        v[i] = 1.0
        return v

    res = {"N": N, "dt": dt, "precision": "complex64", "no_coupling": [], "nn_coupling": [],
           "full_coupling": []}
    hk = W.global_controls(0.5)
    t_mid = (np.arange(N) + 0.5) * dt
    for case, h0_of in (("no_coupling", lambda n: [W.one_body(0.5, "z")]),
                        ("nn_coupling", lambda n: W.ising_ring_terms(1.0, 1.0)),
                        ("full_coupling", lambda n: W.full_coupling_terms(
                            n, 1.0, [1.0 / dd for dd in range(1, n // 2 + 1)]))):
        for n in range(3, nmax + 1):
            rng = np.random.default_rng(1000 + n)
            u_np = rng.uniform(-0.05, 0.05, (N, 2))
            u_np[:, 0] += np.pi / (N * dt) * np.cos(t_mid)
            u_np[:, 1] += np.pi / (N * dt) * np.sin(t_mid)
            u = torch.tensor(u_np, device="cuda")
            h0 = h0_of(n)
            e = {"n": n}
            Fs = []
            if n <= dense_max:
                Bd = q.Basis(n, "cyclic", n)
                e["dense_m"] = 2 ** n
                Fs.append(timed(Bd, h0, hk, u, None, (unit(n, 0, 2 ** n), unit(n, 2 ** n - 1, 2 ** n)),
                                "dense", e))
            Bs = q.Basis(n, "dihedral", 1)
            up, dn = unit(n, 0, 2 ** n), unit(n, 2 ** n - 1, 2 ** n)
            m0 = Bs.sizes[0]
            pu, pd = Bs.to_blocks(up)[:m0].contiguous(), Bs.to_blocks(dn)[:m0].contiguous()
            e["dn_a1_m"] = m0
            Fs.append(timed(Bs, h0, hk, u, [0], (pu, pd), "dn_a1", e))
            if case == "no_coupling":
                Bj = q.Basis(n, "symmetric")
                e["sn_m"] = n + 1
                Fs.append(timed(Bj, h0, hk, u, [0], (unit(n, 0, n + 1), unit(n, n, n + 1)), "sn", e))
            e["F"] = Fs[-1]
            e["max_dF"] = max(Fs) - min(Fs)
            if "dense_ms" in e:
                e["speedup_dn"] = e["dense_ms"] / e["dn_a1_ms"]
                if "sn_ms" in e:
                    e["speedup_sn"] = e["dense_ms"] / e["sn_ms"]
            res[case].append(e)
            print(f"[bench] comparison {case} n={n}: {e}", file=sys.stderr, flush=True)
    return res


def gate_leg(q, torch, P, dev, B, w, reps=3):
    """The unitary of the whole pulse for every block of the ring-12 workload
    (qoc_gate_propagate: the slice propagators, then their time-ordered product as a tree
    of batched complex GEMMs) and the gate fidelity of Sec. III B between the unitaries
    of two nearby pulses.  The product tree's algorithmic flops are (N - 1) 8 m^3 per
    block (complex products)."""
    u = dev["u"]
    u2 = (u + 0.01 * torch.sin(torch.arange(u.numel(), device="cuda", dtype=torch.float64)).view_as(u)).contiguous()
    K = q.gate_propagate(P, u)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        K = q.gate_propagate(P, u)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    q.profile_begin(reps * 8192)
    for _ in range(reps):
        q.gate_propagate(P, u)
    prof = q.profile_end()
    chain_ms = prof["gate_chain"][0] / reps
    flops = sum(8.0 * m ** 3 for m in B.sizes) * (w.N - 1)
    K2 = q.gate_propagate(P, u2)
    f_self = q.gate_fidelity(P, K, K).cpu().numpy()
    f_pair = q.gate_fidelity(P, K, K2).cpu().numpy()
    res = {"workload": "ring12_heisenberg_D12_gate", "slices": w.N, "blocks": list(B.sizes),
           "precision": "complex64 MFMA", "ms": ms, "propagator_ms": prof["propagator_gemm"][0] / reps,
           "chain_ms": chain_ms, "chain_launches": prof["gate_chain"][1] // reps,
           "chain_tflops": flops / (chain_ms * 1e-3) / 1e12,
           "chain_frac_of_fp32_peak": flops / (chain_ms * 1e-3) / 157.3e12,
           "F_self": float(f_self[0]), "F_nearby_pulse": float(f_pair[0]), "D": float(f_pair[3]),
           "unitarity_drift": float(f_self[4] / f_self[3] - 1.0)}
    print(f"[bench] gate {res}", file=sys.stderr, flush=True)
    return res


def lts_leg(q, torch, nmax=13, dt=0.05, Bz=1.0, c_cpl=1.0, dense_max=12, fid_n=11, fid_N=2000):
    """The Trotterised per-qubit-control propagator of Sec. III B (Eqs. (8)-(11)) on the
    Ising ring with B_z = 1, c_cpl = 1, tau = 0.05 and seeded U[-1, 1] per-qubit pulses:
    (a) the runtime per time step of the unitary, K^LTS by qoc_lts_apply (FP64, all 2^n
    columns) against the untrotterised dense propagator (the dense plan with 2n per-qubit
    controls, complex64 MFMA, qoc_gate_propagate), n = 3..nmax (dense up to dense_max), the
    comparison of Fig. 5b; (b) the gate fidelity of K^LTS against the dense unitary for
    fid_n qubits after fid_N steps (Fig. 5a; the dense reference holds every propagator of
    the pulse, which bounds fid_N)."""
    def per_qubit_system(n):
        B = q.Basis(n, "cyclic", n)
        h0 = [{"kind": "one_body", "coeff": 0.5 * Bz, "op": "z", "sites": "all", "stagger": False},
              {"kind": "ring_pair", "coeff": 0.25 * c_cpl, "op": "zz", "distance": 1}]
        hk = []
        for i in range(1, n + 1):
            for a in "XY":
                st = ["I"] * n
                st[i - 1] = a
                hk.append([{"kind": "pauli", "coeff": 0.5, "string": "".join(st)}])
        return B, q.System(B, h0, hk)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, r

    res = {"Bz": Bz, "c_cpl": c_cpl, "dt": dt, "per_step": []}
    for n in range(3, nmax + 1):
        rng = np.random.default_rng(700 + n)
        Nl = 200
        u = torch.tensor(rng.uniform(-1, 1, (Nl, 2 * n)), device="cuda")
        ms_l, _ = timed(lambda: q.lts_apply(n, Bz, c_cpl, u, dt), 2)
        # FP64 vector work per step: 2^n columns x n qubits x 2^(n-1) amplitude pairs, each a
        # 2 x 2 complex product (28 flops) and two phase products (12 flops)
        tflops = (2 ** n) * n * 2 ** (n - 1) * 40.0 / (ms_l / Nl * 1e-3) / 1e12
        e = {"n": n, "lts_ms_per_step": ms_l / Nl, "lts_fp64_tflops": tflops, "lts_frac_of_fp64_vector_peak": tflops / 78.6}
        if n <= dense_max:
            Nd = 20 if n <= 10 else 8
            B, S = per_qubit_system(n)
            P = q.Plan(S, "c64", Nd, dt, 1.0)
            ud = u[:Nd].contiguous()
            ms_d, _ = timed(lambda: q.gate_propagate(P, ud), 2)
            e["dense_ms_per_step"] = ms_d / Nd
            e["speedup"] = e["dense_ms_per_step"] / e["lts_ms_per_step"]
            del P, S, B
            torch.cuda.empty_cache()
        res["per_step"].append(e)
        print(f"[bench] lts {e}", file=sys.stderr, flush=True)
    # gate fidelity of the Trotterised unitary after fid_N steps
    rng = np.random.default_rng(711)
    u = torch.tensor(rng.uniform(-1, 1, (fid_N, 2 * fid_n)), device="cuda")
    B, S = per_qubit_system(fid_n)
    P = q.Plan(S, "c64", fid_N, dt, 1.0)
    steps = fid_N
    if P.info["segments"] > 1:  # less free memory than the whole pulse needs: the part that fits
        steps = P.info["segment"]
        del P
        P = q.Plan(S, "c64", steps, dt, 1.0)
        u = u[:steps].contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Kd = q.gate_propagate(P, u)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Kl = q.lts_apply(fid_n, Bz, c_cpl, u, dt)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    f = q.gate_fidelity(P, [Kl], Kd).cpu().numpy()
    res["fidelity"] = {"n": fid_n, "steps": steps, "F": float(f[0]), "F_paper_form": float(f[1] ** 2 + f[2] ** 2) / f[3] ** 2,
                       "dense_complex64_s": t1 - t0, "lts_fp64_s": t2 - t1}
    print(f"[bench] lts fidelity {res['fidelity']}", file=sys.stderr, flush=True)
    del P, S, B, Kd, Kl
    torch.cuda.empty_cache()
    # objective and exact gradient: Pg candidate pulses through the Trotterised propagator
    # (one work-group each) against the dense exact path of one pulse
    n, Ng, Pg = fid_n, fid_N, 64
    rng = np.random.default_rng(712)
    ug = torch.tensor(rng.uniform(-1, 1, (Pg, Ng, 2 * n)), device="cuda")
    p0 = torch.zeros((Pg, 2 ** n), dtype=torch.complex128, device="cuda")
    p0[:, 0] = 1.0
    pf = torch.zeros((Pg, 2 ** n), dtype=torch.complex128, device="cuda")
    pf[:, -1] = 1.0
    ms_g, _ = timed(lambda: q.lts_fidelity_grad(n, Bz, c_cpl, ug, dt, p0, pf), 2)
    Nd = 20
    B, S = per_qubit_system(n)
    P = q.Plan(S, "c64", Nd, dt, 1.0)
    ud = ug[0, :Nd].contiguous()
    ms_d, _ = timed(lambda: q.fidelity_grad(P, ud, p0[0], pf[0], check=False), 2)
    res["gradient"] = {"n": n, "slices": Ng, "candidates": Pg, "lts_ms": ms_g,
                       "lts_us_per_slice_per_candidate": ms_g * 1e3 / (Ng * Pg),
                       "dense_exact_ms_per_slice": ms_d / Nd, "dense_slices": Nd, "dense_precision": "complex64 MFMA"}
    print(f"[bench] lts gradient {res['gradient']}", file=sys.stderr, flush=True)
    del P, S, B
    torch.cuda.empty_cache()
    return res


def optimizer_leg(q, torch, W, N=100, dt=0.05):
    """GRAPE optimisation (qoc_optimize_lbfgs) of the transfer all-up -> all-down in the first
    D_n block, nearest-neighbour (Eq. (5), c_cpl = 1) against full coupling (Eq. (7),
    c^(d) = 1/d), n = 4..6 qubits (the convergence comparison of Fig. 4e), complex128,
    seeded U[-0.1, 0.1] start, F target 0.999; and one larger run (12 qubits, first block of
    224, 500 slices, complex64) that measures the optimiser's own overhead per evaluation
    against a plain objective+gradient call."""
    hk = W.global_controls(0.5)

    def first_block(n, h0, prec, Nn, u_bound):
        B = q.Basis(n, "dihedral", 1)
        S = q.System(B, h0, hk)
        P = q.Plan(S, prec, Nn, dt, u_bound, blocks=[0])
        up = torch.zeros(2 ** n, dtype=torch.complex128, device="cuda")
        dn = torch.zeros(2 ** n, dtype=torch.complex128, device="cuda")
        up[0] = 1.0
        dn[-1] = 1.0
        m0 = B.sizes[0]
        return P, B.to_blocks(up)[:m0].contiguous(), B.to_blocks(dn)[:m0].contiguous()

    def run(P, u0, pu, pd, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = q.optimize_lbfgs(P, u0, pu, pd, **kw)
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    out = {"N": N, "dt": dt, "precision": "complex128", "f_target": 0.999, "runs": []}
    for n in (4, 5, 6):
        for case, h0 in (("nn_coupling", W.ising_ring_terms(1.0, 1.0)),
                         ("full_coupling", W.full_coupling_terms(n, 1.0, [1.0 / d for d in range(1, n // 2 + 1)]))):
            P, pu, pd = first_block(n, h0, "c128", N, 4.0)
            rng = np.random.default_rng(500 + n)
            u0 = torch.tensor(rng.uniform(-0.1, 0.1, (N, 2)), device="cuda")
            r, ms = run(P, u0, pu, pd, max_iter=1000, memory=10, step0=0.2, f_target=0.999)
            e = {"n": n, "case": case, "m": int(pu.numel()), "F0": float(r["hist"][0]), "F": r["F"],
                 "iterations": r["iterations"], "evaluations": r["evaluations"], "reason": r["reason"],
                 "ms": ms}
            out["runs"].append(e)
            print(f"[bench] optimizer {e}", file=sys.stderr, flush=True)
    # overhead of the optimiser around its evaluations, on a larger block
    n, Nn = 12, 500
    P, pu, pd = first_block(n, W.ising_ring_terms(1.0, 1.0), "c64", Nn, 4.0)
    rng = np.random.default_rng(512)
    u0 = torch.tensor(rng.uniform(-0.1, 0.1, (Nn, 2)), device="cuda")
    q.optimize_lbfgs(P, u0, pu, pd, max_iter=2)  # warm-up
    r, ms = run(P, u0, pu, pd, max_iter=40, memory=10, step0=0.2, f_target=0.99)
    ws = P.workspace()
    q.fidelity_grad(P, u0, pu, pd, workspace=ws, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        q.fidelity_grad(P, u0, pu, pd, workspace=ws, check=False)
    torch.cuda.synchronize()
    eval_ms = (time.perf_counter() - t0) * 1e3 / 5
    big = {"n": n, "m": int(pu.numel()), "N": Nn, "precision": "complex64", "F0": float(r["hist"][0]),
           "F": r["F"], "iterations": r["iterations"], "evaluations": r["evaluations"], "reason": r["reason"],
           "ms": ms, "ms_per_evaluation": ms / r["evaluations"], "plain_evaluation_ms": eval_ms,
           "overhead_frac": 1.0 - r["evaluations"] * eval_ms / ms}
    out["large"] = big
    print(f"[bench] optimizer large {big}", file=sys.stderr, flush=True)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, v0, vf, nslices, nslices_1t):
    """The FP64 oracle (eigendecomposition propagators, Daleckii-Krein gradient) on the host,
    on the first slices of the same workload (all blocks): on every BLAS thread, and on one."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import grape as og
    ob = og.block_system(12, w.h0, w.hk)

    def panels(v):
        out, off = [], 0
        for b in ob:
            s = b["m"] * b["d"]
            out.append(v[off:off + s].reshape(b["d"], b["m"]).T)
            off += s
        return out

    t0 = time.perf_counter()
    og.fidelity_grad(ob, w.u[:nslices], w.dt, panels(v0), panels(vf))
    el = time.perf_counter() - t0
    threads = max([i["num_threads"] for i in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        og.fidelity_grad(ob, w.u[:nslices_1t], w.dt, panels(v0), panels(vf))
        el1 = time.perf_counter() - t0
    return {"value": nslices * len(ob) / el, "unit": "slices*blocks/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"first {nslices} of {w.N} slices, all {len(ob)} blocks, FP64 eigendecomposition "
                      f"propagators and Daleckii-Krein gradient ({el:.1f} s on {threads} BLAS threads)",
            "single_thread": {"value": nslices_1t * len(ob) / el1, "unit": "slices*blocks/s", "cores": 1,
                              "sample": f"first {nslices_1t} slices, all blocks ({el1:.1f} s)"}}


def _fp64_subset(q, torch, make_plan, run, reps=1):
    """ms per step of the same work in complex64 and complex128 (one warm-up each)."""
    res = {}
    for prec in ("c64", "c128"):
        P = make_plan(prec)
        run(P)
        ms, _ = one_step(torch, lambda: run(P))
        for _ in range(reps - 1):
            ms = min(ms, one_step(torch, lambda: run(P))[0])
        res[prec] = ms
        del P
        torch.cuda.empty_cache()
    return {"c64_ms": res["c64"], "c128_ms": res["c128"], "speedup": res["c128"] / res["c64"]}


def sym_leg(q, torch, W, C):
    """All-to-all S_128 register: C candidate pulses (500 slices of 0.01 each, 65 blocks of
    129..1 states) in one batched plan, complex64, every block of every candidate carrying
    state.  One timed step (the kernels are warmed up and the tile variant chosen by the
    autotuner on a 32-candidate plan of the same blocks).  Parity: candidates 0, 5 and C - 1
    against stored oracle values when C = 1024 (the full workload).  FP32 vs FP64: the
    first 16 candidates in both precisions."""
    ws = W.config5(seed=0, C=C)
    uc = ws.notes["u_candidates"]
    rs = ws.notes["rng"]
    Bs = q.Basis(128, "symmetric")
    Ss = q.System(Bs, ws.h0, ws.hk)
    states = []
    for _ in range(C):  # psi_f then psi0 per candidate, after the pulses
        vf = W.gaussian_panel(rs, Bs.dim)
        v0 = W.gaussian_panel(rs, Bs.dim)
        states.append((v0, vf))
    us = [torch.tensor(x, device="cuda") for x in uc]
    p0 = [torch.tensor(st[0], device="cuda") for st in states]
    pf = [torch.tensor(st[1], device="cuda") for st in states]
    sub = min(32, C)
    Pt = q.Plan.batched([Ss] * sub, "c64", [ws.N] * sub, [ws.dt] * sub, 1.0)
    chosen, tune_ms = Pt.autotune(torch.cat([x.reshape(-1) for x in us[:sub]]))
    q.fidelity_grad_batched(Pt, us[:sub], p0[:sub], pf[:sub], check=False)
    del Pt
    torch.cuda.empty_cache()
    Ps = q.Plan.batched([Ss] * C, "c64", [ws.N] * C, [ws.dt] * C, 1.0)
    Ps.set_variant(chosen)
    uflat = torch.cat([x.reshape(-1) for x in us])
    res = {}

    def run():
        res["out"], res["grads"] = q.fidelity_grad_batched(Ps, us, p0, pf, check=False)

    nb = len(Bs.sizes)
    sym = profiled_leg(q, torch, Ps, run, 1, 0, uflat, list(Bs.sizes) * C, C * nb * ws.N,
                       job_problem=[c for c in range(C) for _ in range(nb)], launches_per_step=1 << 17)
    out = res["out"]
    for c in range(C):
        q.check_flags(out[c])
    sym.update({"workload": "allpairs128_S128_candidates", "full_size": C == 1024, "candidates": C,
                "slices": ws.N, "blocks": len(Bs.sizes), "autotune_ms": tune_ms})
    if C == 1024:
        sym["parity"] = [parity(f"sym128_C1024_cand{c}_N{ws.N}.txt", out[c, 0].item(), res["grads"][c].cpu().numpy())
                         for c in (0, 5, C - 1)]
    del Ps, res
    torch.cuda.empty_cache()
    k = min(16, C)
    sym["fp32_vs_fp64"] = _fp64_subset(
        q, torch, lambda prec: q.Plan.batched([Ss] * k, prec, [ws.N] * k, [ws.dt] * k, 1.0),
        lambda P: q.fidelity_grad_batched(P, us[:k], p0[:k], pf[:k], check=False))
    sym["fp32_vs_fp64"]["subset"] = f"first {k} candidates"
    print(f"[bench] S_128 x {C}: {sym}", file=sys.stderr, flush=True)
    return sym


def ring14_leg(q, torch, W, N):
    """The 14-qubit ring with staggered controls under the two-site group (blocks 1300,
    1044, 3 x 2340; 4 controls; slices of 0.01): the first N slices of its 4000-slice pulse
    (N = 4000: the full workload), all blocks, complex64, the default workspace budget
    (propagators recomputed segment by segment in the backward sweep).  One timed step after
    the kernels are warmed up and the tile variant chosen on the 64-slice prefix plan.
    Parity and FP32 vs FP64: the 64-slice prefix in both precisions against stored oracle
    values (the oracle takes about 35 s per slice of this workload)."""
    w4 = W.config4(seed=0, variant="all")
    r4 = w4.notes["rng"]
    B4 = q.Basis(14, "dihedral", 2)
    S4 = q.System(B4, w4.h0, w4.hk)
    f4 = torch.tensor(W.gaussian_panel(r4, B4.dim), device="cuda")
    z4 = torch.tensor(W.gaussian_panel(r4, B4.dim), device="cuda")
    u_all = torch.tensor(w4.u, device="cuda")
    # prefix: parity in both precisions, FP32 vs FP64 timing, autotune
    Np = min(64, N)
    gname = f"ring14_T2R_allblocks_N{Np}.txt"
    if golden_values(gname) is None:
        Np = min(8, N)
        gname = f"ring14_T2R_allblocks_N{Np}.txt"
    up = u_all[:Np].contiguous()
    prefix = {"slices": Np}
    chosen = 0
    for prec in ("c64", "c128"):
        P = q.Plan(S4, prec, Np, w4.dt, 2.0)
        if prec == "c64":
            chosen, prefix["autotune_ms"] = P.autotune(up)
        q.fidelity_grad(P, up, z4, f4)
        ms, (o, g) = one_step(torch, lambda: q.fidelity_grad(P, up, z4, f4))
        q.check_flags(o)
        prefix[prec + "_ms"] = ms
        prefix["parity_" + prec] = parity(gname, o[0].item(), g.cpu().numpy())
        del P
        torch.cuda.empty_cache()
    prefix["speedup"] = prefix["c128_ms"] / prefix["c64_ms"]
    u4 = u_all[:N].contiguous()
    P4 = q.Plan(S4, "c64", N, w4.dt, 2.0)
    P4.set_variant(chosen)
    res = {}

    def run():
        res["out"], res["grad"] = q.fidelity_grad(P4, u4, z4, f4, check=False)

    ring14 = profiled_leg(q, torch, P4, run, 1, 0, u4, list(B4.sizes), len(B4.sizes) * N)
    q.check_flags(res["out"])
    ring14.update({"workload": "ring14_stagger_T2R_allblocks", "full_size": N == 4000, "slices": N,
                   "blocks": list(B4.sizes), "F": res["out"][0].item(), "prefix": prefix})
    print(f"[bench] ring14: {ring14}", file=sys.stderr, flush=True)
    del P4, res
    torch.cuda.empty_cache()
    return ring14


def batch_leg(q, torch, W, Pn):
    """The first Pn problems of the 256-ring batched workload (n in {8, 10, 12, 14}, 200-2000
    slices of 0.02, J ~ U[0.5, 1.5], all blocks carrying state) in one complex64 plan with
    the default workspace budget; Pn = 256 is the full workload.  One timed step after the
    kernels are warmed up and the tile variant chosen on a plan of the first 4 problems.
    Parity: every problem with stored oracle values; FP32 vs FP64: the first 4 problems in
    both precisions."""
    wl, rb = W.config3_list(seed=0)
    wl = wl[:Pn]
    states = []
    for x in wl:  # psi_f then psi0 per problem, in list order
        vf = W.gaussian_panel(rb, 2 ** x.n)
        v0 = W.gaussian_panel(rb, 2 ** x.n)
        states.append((v0, vf))
    bases = {n: q.Basis(n) for n in sorted({x.n for x in wl})}
    systems = [q.System(bases[x.n], x.h0, x.hk) for x in wl]
    ub = [torch.tensor(x.u, device="cuda") for x in wl]
    p0 = [torch.tensor(st[0], device="cuda") for st in states]
    pf = [torch.tensor(st[1], device="cuda") for st in states]
    k = min(4, Pn)

    def subset_plan(prec):
        return q.Plan.batched(systems[:k], prec, [x.N for x in wl[:k]], [x.dt for x in wl[:k]], 1.0)

    Pt = subset_plan("c64")
    chosen, tune_ms = Pt.autotune(torch.cat([x.reshape(-1) for x in ub[:k]]))
    del Pt
    torch.cuda.empty_cache()
    fp = _fp64_subset(q, torch, subset_plan, lambda P: q.fidelity_grad_batched(P, ub[:k], p0[:k], pf[:k], check=False))
    fp["subset"] = f"first {k} problems"
    print(f"[bench] batch: planning {len(wl)} problems", file=sys.stderr, flush=True)
    Pb = q.Plan.batched(systems, "c64", [x.N for x in wl], [x.dt for x in wl], 1.0)
    Pb.set_variant(chosen)
    uflat = torch.cat([x.reshape(-1) for x in ub])
    sizes = [m for x in wl for m in bases[x.n].sizes]
    units_b = sum(len(bases[x.n].sizes) * x.N for x in wl)
    res = {}

    def run():
        res["out"], res["grads"] = q.fidelity_grad_batched(Pb, ub, p0, pf, check=False)

    jp = [p for p, x in enumerate(wl) for _ in bases[x.n].sizes]
    print(f"[bench] batch plan: {Pb.info['problem_groups']} problem groups, workspace {Pb.workspace_bytes / 2**30:.1f} GiB",
          file=sys.stderr, flush=True)
    q.set_progress(True)  # a line per finished problem group: a full-size step runs for minutes
    batch = profiled_leg(q, torch, Pb, run, 1, 0, uflat, sizes, units_b, job_problem=jp, launches_per_step=1 << 18)
    q.set_progress(False)
    out = res["out"]
    for p in range(len(wl)):
        q.check_flags(out[p])
    par = []
    for p, x in enumerate(wl):
        r = parity(f"batch256_p{p}_n{x.n}_N{x.N}.txt", out[p, 0].item(), res["grads"][p].cpu().numpy())
        if r is not None:
            r["problem"] = p
            par.append(r)
    batch.update({"workload": "batch_rings", "full_size": Pn == 256, "problems": len(wl),
                  "n": [x.n for x in wl], "slices": [x.N for x in wl], "block_slices": units_b,
                  "autotune_ms": tune_ms, "parity": par, "fp32_vs_fp64": fp})
    print(f"[bench] batch: {batch}", file=sys.stderr, flush=True)
    del Pb, res, systems, bases
    torch.cuda.empty_cache()
    return batch


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (each GPU would take its own "
              "share of blocks or problems); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2309_05884_amd as q
    import qoc_workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration << 18  # float32 elements
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {n * 4} bytes read, {n * 4} bytes written", file=sys.stderr, flush=True)
        del src, dst
    measured_peak = {"c64": q.measure_mfma_peak("c64"), "c128": q.measure_mfma_peak("c128")}
    print(f"[bench] measured MFMA rate (TFLOP/s): {measured_peak}", file=sys.stderr, flush=True)
    w, B, S, v0, vf, dev = build_problem(q, W, torch)
    nblocks = len(B.sizes)
    units = w.N * nblocks
    print(f"[bench] blocks {B.sizes} copies {B.copies}", file=sys.stderr, flush=True)

    P32 = q.Plan(S, "c64", w.N, w.dt, 2.0)
    if args.gemm_variant32 >= 0:
        P32.set_variant(args.gemm_variant32)
        tune32 = (args.gemm_variant32, [])
    else:
        tune32 = P32.autotune(dev["u"])
    print(f"[bench] c64 plan {P32.info} workspace {P32.workspace_bytes / 2**30:.1f} GiB; GEMM variant "
          f"{P32.variant_name} (autotune ms {tune32[1]})", file=sys.stderr, flush=True)
    ms32, wall32, prof32, out32, grad32 = timed_steps(q, torch, P32, dev, args.steps, args.warmup)
    flops32, qs32, ss32 = gemm_flops(q, P32, dev, B.sizes)
    var32 = P32.variant_name
    print(f"[bench] c64 {ms32:.2f} ms/step  profile {prof32}", file=sys.stderr, flush=True)
    gate = gate_leg(q, torch, P32, dev, B, w) if args.gate else None
    del P32
    torch.cuda.empty_cache()

    dense = None
    if args.dense_slices > 0:
        # the same hot path on the dense 2^12 space (trivial group: one 4096-wide block)
        Bd = q.Basis(12, "cyclic", 12)
        Sd = q.System(Bd, w.h0, w.hk)
        Nd = args.dense_slices
        Pd = q.Plan(Sd, "c64", Nd, w.dt, 2.0)
        ud = dev["u"][:Nd].contiguous()
        d0, df = B.from_blocks(dev["psi0"]), B.from_blocks(dev["psif"])
        q.fidelity_grad(Pd, ud, d0, df)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        od, gd = q.fidelity_grad(Pd, ud, d0, df)
        e1.record()
        torch.cuda.synchronize()
        msd = e0.elapsed_time(e1)
        dense = {"n": 12, "dim": 4096, "slices": Nd, "ms": msd, "ms_per_slice": msd / Nd,
                 "blocks_ms_per_slice": ms32 / w.N, "symmetry_speedup": (msd / Nd) / (ms32 / w.N),
                 "precision": "complex64 MFMA, same kernels, trivial group"}
        print(f"[bench] dense 4096: {msd:.1f} ms for {Nd} slices", file=sys.stderr, flush=True)
        del Pd, Sd, Bd
        torch.cuda.empty_cache()

    def leg(name, fn, *a):
        t0 = time.time()
        r = fn(*a)
        print(f"[bench] {name} leg: {time.time() - t0:.1f} s wall", file=sys.stderr, flush=True)
        return r

    sym = leg("S_128 candidates", sym_leg, q, torch, W, args.sym_candidates) if args.sym_candidates > 0 else None
    comparison = None
    if args.paper_comparison > 0:
        comparison = leg("paper comparison", paper_comparison, q, torch, W, args.paper_comparison)
        torch.cuda.empty_cache()
    optimizer = leg("optimizer", optimizer_leg, q, torch, W) if args.optimizer else None
    lts = leg("Trotterised", lts_leg, q, torch) if args.lts else None

    ring14 = leg("ring-14", ring14_leg, q, torch, W, args.ring14_slices) if args.ring14_slices > 0 else None
    batch = leg("ring batch", batch_leg, q, torch, W, args.batch_problems) if args.batch_problems > 0 else None

    gemm_ms, gemm_n = prof32["propagator_gemm"]
    achieved = flops32 * args.steps / (gemm_ms * 1e-3) / 1e12
    fp64 = cmp = par64 = None
    par32 = parity("ring12_D12_allblocks_N1000.txt", out32[0].item(), grad32.cpu().numpy())
    if args.fp64_steps > 0:
        P64 = q.Plan(S, "c128", w.N, w.dt, 2.0)
        tune64 = P64.autotune(dev["u"])
        ms64, wall64, prof64, out64, grad64 = timed_steps(q, torch, P64, dev, args.fp64_steps, 1)
        flops64, _, _ = gemm_flops(q, P64, dev, B.sizes)
        print(f"[bench] c128 {ms64:.2f} ms/step  profile {prof64}", file=sys.stderr, flush=True)
        var64 = P64.variant_name
        del P64
        gemm64_ms, _ = prof64["propagator_gemm"]
        achieved64 = flops64 * args.fp64_steps / (gemm64_ms * 1e-3) / 1e12
        g64 = grad64.cpu()
        fp64 = {"value": units / (ms64 * 1e-3), "ms_per_step": ms64, "steps": args.fp64_steps,
                "gemm_tflops": achieved64, "gemm_frac": achieved64 / MFMA_PEAK["c128"],
                "gemm_variant": var64, "autotune_ms": tune64[1]}
        cmp = {"speedup": ms64 / ms32, "dF": abs(out32[0].item() - out64[0].item()),
               "grad_rel_err": float((grad32.cpu() - g64).abs().max() / g64.abs().max()), "F64": out64[0].item()}
        par64 = parity("ring12_D12_allblocks_N1000.txt", out64[0].item(), g64.numpy())

    traffic = None
    if kernel_sources_sha1() == TRAFFIC["sources_sha1"] and var32 in TRAFFIC["kib"]:
        fetch_kib, write_kib = TRAFFIC["kib"][var32]
        traffic = 1024.0 * (fetch_kib * TRAFFIC["fetch_scale"] + write_kib * TRAFFIC["write_scale"])
    line = {
        "metric": "GRAPE slices*blocks/sec (fidelity+gradient), FP32-batched vs FP64, |dF|<=1e-6",
        "value": units / (ms32 * 1e-3),
        "unit": "slices*blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ring12_heisenberg_D12_allblocks", "n": 12, "group": "D12", "slices": w.N,
                   "dt": w.dt, "controls": 2, "blocks": B.sizes, "copies": B.copies, "J": round(w.J, 6),
                   "precision": "complex64 MFMA products; FP64 norms, objective and gradient accumulation"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_PEAK["c64"], "unit": "TFLOP/s",
                     "frac": achieved / MFMA_PEAK["c64"], "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM side)",
                     "kernel": "k_expm_step<float>", "gemm_variant": var32, "autotune_ms": tune32[1],
                     "launches": gemm_n,
                     "alg_flops_per_launch": flops32 * args.steps / gemm_n,
                     "avg_launch_ms": gemm_ms / gemm_n, "kernel_ms_per_step": gemm_ms / args.steps,
                     "executed_mfma_frac": 0.75 * achieved / MFMA_PEAK["c64"],
                     "measured_peak": measured_peak["c64"],
                     "measured_peak_note": "v_mfma_f32_16x16x4f32 chains on register operands over a full grid "
                                           "(qoc_measure_mfma_peak); FP64: %.1f TFLOP/s" % measured_peak["c128"],
                     "executed_frac_of_measured_peak": 0.75 * achieved / measured_peak["c64"],
                     "note": "algorithmic flops 8 m^3 per complex m x m product, 4 m^2 (m + 1) for the "
                             "(skew-)Hermitian powers of the generator (lower triangle; the upper is mirrored); "
                             "the kernel forms each with three real MFMA products (Gauss): 3/4 of them executed"},
        "parity": {"c64": par32, "c128": par64,
                   "bounds": "c64: |dF| <= 1e-6; c128: |dF| and max grad error <= 1e-12 (FP64 oracle)"},
        "fp64": fp64,
        "fp32_vs_fp64": cmp,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof32.items()},
        "dense_comparison": dense,
        "batched_sym128": sym,
        "ring14_stagger": ring14,
        "batched_rings": batch,
    }
    if comparison is not None:
        line["paper_comparison"] = comparison
    if optimizer is not None:
        line["optimizer"] = optimizer
    if gate is not None:
        line["gate"] = gate
    if lts is not None:
        line["lts"] = lts
    if not args.no_cpu_baseline:
        print("[bench] oracle sample on the host ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, v0, vf, args.cpu_slices, args.cpu_slices_1t)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
