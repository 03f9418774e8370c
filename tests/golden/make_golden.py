"""Write oracle-computed expected values for full-size parity tests.

Calls only the FP64 CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_golden.py ring12       # 12-qubit ring, D12, all blocks, N=1000
    python tests/golden/make_golden.py ring14       # 14-qubit ring, two-site group, first 8 slices
    python tests/golden/make_golden.py sym128       # S_128, 8 candidates, candidates 0 and 5
    python tests/golden/make_golden.py sym128 1024  # S_128, 1024 candidates, candidates 0, 5, 1023
    python tests/golden/make_golden.py ring14 64    # 14-qubit ring, first 64 slices
    python tests/golden/make_golden.py batch 0 1 2 4   # problems of the 256-ring batch
The output files hold F, o, ||psi_N||^2 and the full gradient, one value per line.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import qoc_workloads as W  # noqa: E402
from oracle import grape as og  # noqa: E402


def panels(blocks, v):
    out, off = [], 0
    for b in blocks:
        s = b["m"] * b["d"]
        out.append(v[off:off + s].reshape(b["d"], b["m"]).T)
        off += s
    return out


def _write(path, header, r, N):
    with open(path, "w") as fh:
        fh.write(header + "\n")
        fh.write(f"F {float(r['F'])!r}\nF_raw {float(r['F_raw'])!r}\no_re {float(r['o'].real)!r}\n")
        fh.write(f"o_im {float(r['o'].imag)!r}\nnormN2 {float(r['normN2'])!r}\n")
        for j in range(N):
            fh.write("g " + " ".join(repr(float(v)) for v in r["grad"][j]) + "\n")


def ring12():
    """The benchmark workload: psi_f then psi0 drawn after u from the same generator."""
    w = W.config2(seed=0, variant="all")
    rng = w.notes["rng"]
    ob = og.block_system(12, w.h0, w.hk)
    D = sum(b["m"] * b["d"] for b in ob)
    vf = W.gaussian_panel(rng, D)
    v0 = W.gaussian_panel(rng, D)
    t = time.time()
    r = og.fidelity_grad(ob, w.u, w.dt, panels(ob, v0), panels(ob, vf))
    path = os.path.join(HERE, "ring12_D12_allblocks_N1000.txt")
    with open(path, "w") as fh:
        fh.write("# oracle (FP64, eigendecomposition + Daleckii-Krein) for qoc_workloads.config2(seed=0, "
                 "variant='all'), psi_f then psi0 Gaussian panels; written by make_golden.py\n")
        fh.write(f"F {float(r['F'])!r}\nF_raw {float(r['F_raw'])!r}\no_re {float(r['o'].real)!r}\n")
        fh.write(f"o_im {float(r['o'].imag)!r}\nnormN2 {float(r['normN2'])!r}\n")
        for j in range(w.N):
            fh.write("g " + " ".join(repr(float(v)) for v in r["grad"][j]) + "\n")
    print(path, f"{time.time() - t:.1f} s", r["F"])


def ring14(nslices=8):
    """The 14-qubit staggered-control workload under the two-site group (blocks 1300, 1044,
    3 x 2340): the first `nslices` slices of its 4000-slice pulse, all blocks carrying state
    (psi_f then psi0 drawn after u)."""
    w = W.config4(seed=0, variant="all")
    rng = w.notes["rng"]
    t = time.time()
    ob = og.block_system(14, w.h0, w.hk, "dihedral", 2)
    D = sum(b["m"] * b["d"] for b in ob)
    vf = W.gaussian_panel(rng, D)
    v0 = W.gaussian_panel(rng, D)
    r = og.fidelity_grad(ob, w.u[:nslices], w.dt, panels(ob, v0), panels(ob, vf), keep_states=True)
    path = os.path.join(HERE, f"ring14_T2R_allblocks_N{nslices}.txt")
    with open(path, "w") as fh:
        fh.write("# oracle (FP64, eigendecomposition + Daleckii-Krein) for qoc_workloads.config4(seed=0, "
                 f"variant='all'), first {nslices} slices, psi_f then psi0 Gaussian panels; written by "
                 "make_golden.py\n")
        fh.write(f"F {float(r['F'])!r}\nF_raw {float(r['F_raw'])!r}\no_re {float(r['o'].real)!r}\n")
        fh.write(f"o_im {float(r['o'].imag)!r}\nnormN2 {float(r['normN2'])!r}\n")
        for j in range(nslices):
            fh.write("g " + " ".join(repr(float(v)) for v in r["grad"][j]) + "\n")
    print(path, f"{time.time() - t:.1f} s", r["F"])


def sym128(C=8, which=None):
    """The all-to-all S_128 workload with C candidate pulses (500 slices each); states are
    drawn after the pulses, psi_f then psi0 per candidate.  Candidates `which` are written."""
    w = W.config5(seed=0, C=C)
    rng = w.notes["rng"]
    uc = w.notes["u_candidates"]
    if which is None:
        which = (0, 5) if C == 8 else (0, 5, C - 1)
    t = time.time()
    ob = og.block_system(128, w.h0, w.hk, "symmetric")
    D = sum(b["m"] * b["d"] for b in ob)
    states = []
    for _ in range(C):
        vf = W.gaussian_panel(rng, D)
        v0 = W.gaussian_panel(rng, D)
        states.append((v0, vf))
    for c in which:
        r = og.fidelity_grad(ob, uc[c], w.dt, panels(ob, states[c][0]), panels(ob, states[c][1]))
        path = os.path.join(HERE, f"sym128_C{C}_cand{c}_N{w.N}.txt")
        with open(path, "w") as fh:
            fh.write(f"# oracle (FP64, eigendecomposition + Daleckii-Krein) for qoc_workloads.config5(seed=0, C={C}), "
                     f"candidate {c}, states psi_f then psi0 per candidate drawn after the pulses; written by "
                     "make_golden.py\n")
            fh.write(f"F {float(r['F'])!r}\nF_raw {float(r['F_raw'])!r}\no_re {float(r['o'].real)!r}\n")
            fh.write(f"o_im {float(r['o'].imag)!r}\nnormN2 {float(r['normN2'])!r}\n")
            for j in range(w.N):
                fh.write("g " + " ".join(repr(float(v)) for v in r["grad"][j]) + "\n")
        print(path, f"{time.time() - t:.1f} s", r["F"], flush=True)


def batch(problems):
    """Problems of the 256-ring batched workload (qoc_workloads.config3_list(seed=0)):
    after the list is drawn, each problem in list order draws psi_f then psi0 (2^n
    amplitudes each, Gaussian panels over every block) from the list's generator, so a
    problem's states do not depend on how many problems follow it."""
    ws, rng = W.config3_list(seed=0)
    states = []
    for w in ws[:max(problems) + 1]:
        vf = W.gaussian_panel(rng, 2 ** w.n)
        v0 = W.gaussian_panel(rng, 2 ** w.n)
        states.append((v0, vf))
    for p in problems:
        w = ws[p]
        t = time.time()
        ob = og.block_system(w.n, w.h0, w.hk, "dihedral", w.stride)
        v0, vf = states[p]
        r = og.fidelity_grad(ob, w.u, w.dt, panels(ob, v0), panels(ob, vf), keep_states=True)
        path = os.path.join(HERE, f"batch256_p{p}_n{w.n}_N{w.N}.txt")
        _write(path, f"# oracle (FP64, eigendecomposition + Daleckii-Krein) for problem {p} of "
                     f"qoc_workloads.config3_list(seed=0) (n={w.n}, N={w.N}, J={w.J!r}), "
                     "states psi_f then psi0 per problem in list order; written by make_golden.py", r, w.N)
        print(path, f"{time.time() - t:.1f} s", r["F"], flush=True)


if __name__ == "__main__":
    cmd, rest = sys.argv[1], [int(a) for a in sys.argv[2:]]
    if cmd == "batch":
        batch(rest)
    elif cmd in ("ring14", "sym128"):
        {"ring14": ring14, "sym128": sym128}[cmd](*rest)
    else:
        {"ring12": ring12}[cmd]()
