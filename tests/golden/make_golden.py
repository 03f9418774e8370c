"""Write oracle-computed expected values for full-size parity tests.

Calls only the FP64 CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_golden.py ring12       # 12-qubit ring, D12, all blocks, N=1000
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
        fh.write(f"F {r['F']!r}\nF_raw {r['F_raw']!r}\no_re {r['o'].real!r}\no_im {r['o'].imag!r}\n")
        fh.write(f"normN2 {r['normN2']!r}\n")
        for j in range(w.N):
            fh.write("g " + " ".join(repr(float(v)) for v in r["grad"][j]) + "\n")
    print(path, f"{time.time() - t:.1f} s", r["F"])


if __name__ == "__main__":
    {"ring12": ring12}[sys.argv[1]]()
