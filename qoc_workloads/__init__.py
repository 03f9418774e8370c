"""Seeded synthetic workloads for symmetry-reduced GRAPE.

This module is shared by the CPU oracle and the HIP path.  It holds plain
data only: Hamiltonians as lists of Pauli-sum term descriptors, control
samples, and random state panels drawn from a seeded generator.  It does no
projection, exponentiation or contraction; block sizes needed to shape the
state panels are passed in by the caller.

Term descriptors (dicts), with qubits numbered 1..n as in the paper
(Sec. II A, Kronecker order, qubit 1 leftmost):

* ``{"kind": "one_body", "coeff": c, "op": a, "sites": "all"|"even"|"odd",
  "stagger": bool}``  ->  c * sum_i w_i sigma_a^(i), with w_i = (-1)^i when
  staggered, summed over the selected qubits i.
* ``{"kind": "ring_pair", "coeff": c, "op": "ab", "distance": d}``  ->
  c * sum_{i=1..n} sigma_a^(i) sigma_b^(i+d), indices mod n (Eq. (5), Eq. (7)).
* ``{"kind": "all_pairs", "coeff": c, "op": "ab"}``  ->
  c * sum_{i<j} sigma_a^(i) sigma_b^(j).
* ``{"kind": "pauli", "coeff": c, "string": "XIZ..."}`` -> c * one Pauli
  string, character q of the string acting on qubit q+1.

Random draws follow one protocol: ``numpy.random.default_rng(seed)``; draw
J (when random), then u as ``uniform(lo, hi, (N, K))``, then the real and
imaginary parts of psi_f, then psi0 when it is random.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Workload", "heisenberg_ring_terms", "ising_ring_terms", "full_coupling_terms",
    "global_controls", "config1", "config2", "config4", "config5", "config3_list",
    "gaussian_panel", "draw_controls",
]


def one_body(coeff, op, sites="all", stagger=False):
    return {"kind": "one_body", "coeff": float(coeff), "op": op, "sites": sites,
            "stagger": bool(stagger)}


def ring_pair(coeff, op, distance=1):
    return {"kind": "ring_pair", "coeff": float(coeff), "op": op, "distance": int(distance)}


def all_pairs(coeff, op):
    return {"kind": "all_pairs", "coeff": float(coeff), "op": op}


def heisenberg_ring_terms(J: float, field_z: float = 0.5):
    """H0 = field_z * sum sigma_z + J * sum_<i,i+1> (xx + yy + zz) on a ring."""
    return [one_body(field_z, "z"), ring_pair(J, "xx"), ring_pair(J, "yy"), ring_pair(J, "zz")]


def ising_ring_terms(Bz: float, c_cpl: float):
    """Eq. (5): H0 = Bz/2 sum sigma_z + c_cpl/4 sum sigma_z sigma_z (nearest neighbours)."""
    return [one_body(0.5 * Bz, "z"), ring_pair(0.25 * c_cpl, "zz", 1)]


def full_coupling_terms(n: int, Bz: float, couplings):
    """Eq. (7): Bz/2 sum sigma_z + sum_d c^(d)/4 sum_i sigma_z^(i) sigma_z^(i+d), d = 1..floor(n/2)."""
    terms = [one_body(0.5 * Bz, "z")]
    for d, c in enumerate(couplings, start=1):
        if d > n // 2:
            raise ValueError("coupling distance beyond floor(n/2)")
        terms.append(ring_pair(0.25 * c, "zz", d))
    return terms


def global_controls(scale: float = 1.0):
    """Global x and y fields: H_1 = scale*sum sigma_x, H_2 = scale*sum sigma_y (Eq. (6) with scale 1/2)."""
    return [[one_body(scale, "x")], [one_body(scale, "y")]]


@dataclass
class Workload:
    name: str
    n: int
    group: str                 # "dihedral" | "cyclic" | "symmetric"
    stride: int
    h0: list
    hk: List[list]
    N: int
    dt: float
    u: np.ndarray              # (N, K) float64
    J: Optional[float] = None
    variant: str = "plain"     # "plain": psi0 = all-up, psi_f in the first block; "all": every block
    seed: int = 0
    notes: dict = field(default_factory=dict)

    @property
    def K(self):
        return len(self.hk)


def draw_controls(rng, N, K, lo, hi):
    return rng.uniform(lo, hi, (N, K))


def gaussian_panel(rng, length: int) -> np.ndarray:
    """A normalised complex Gaussian vector: real parts drawn first, then imaginary parts."""
    re = rng.standard_normal(length)
    im = rng.standard_normal(length)
    v = re + 1j * im
    return v / np.linalg.norm(v)


def config1(seed=0, N=200):
    """n=6 Heisenberg ring, J=1, controls sum sx, sum sy, N=200, dt=0.05, u ~ U[-1,1]."""
    rng = np.random.default_rng(seed)
    u = draw_controls(rng, N, 2, -1.0, 1.0)
    w = Workload("ring6_heisenberg", 6, "dihedral", 1, heisenberg_ring_terms(1.0),
                 global_controls(), N, 0.05, u, J=1.0, seed=seed)
    w.notes["rng"] = rng
    return w


def config2(seed=0, N=1000, n=12, variant="plain"):
    """n=12 Heisenberg ring, J ~ U[0.5,1.5], N=1000, dt=0.02, 2 controls ~ U[-2,2]."""
    rng = np.random.default_rng(seed)
    J = float(rng.uniform(0.5, 1.5))
    u = draw_controls(rng, N, 2, -2.0, 2.0)
    w = Workload(f"ring{n}_heisenberg", n, "dihedral", 1, heisenberg_ring_terms(J),
                 global_controls(), N, 0.02, u, J=J, variant=variant, seed=seed)
    w.notes["rng"] = rng
    return w


def config4(seed=0, N=4000, n=14, variant="plain"):
    """n=14 Heisenberg ring (J=1) with four controls: sum sx, sum sy, staggered sum sz,
    sum of sx on even qubits; N=4000, dt=0.01, u ~ U[-1,1].  The staggered and
    even-site controls keep only the subgroup generated by the two-site rotation
    and the site-centred reflection, so the group stride is 2."""
    rng = np.random.default_rng(seed)
    u = draw_controls(rng, N, 4, -1.0, 1.0)
    hk = [[one_body(1.0, "x")], [one_body(1.0, "y")], [one_body(1.0, "z", stagger=True)],
          [one_body(1.0, "x", sites="even")]]
    w = Workload(f"ring{n}_stagger", n, "dihedral", 2, heisenberg_ring_terms(1.0), hk, N, 0.01,
                 u, J=1.0, variant=variant, seed=seed)
    w.notes["rng"] = rng
    return w


def config5(seed=0, n=128, C=1024, N=500, dt=0.01, omega=1.0, Jc=1.0, cxyz=(1.0, 0.5, 0.0)):
    """All-to-all register under S_n: H0 = omega sum sz + (J/n)(cx Sx^2 + cy Sy^2 + cz Sz^2),
    with S_a = (1/2) sum sigma_a, so S_a^2 = (1/2) sum_{i<j} sigma_a sigma_a + n/4.
    Controls 2 S_x, 2 S_y; C candidate pulses of N slices, u ~ U[-1,1] per candidate."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, (C, N, 2))
    h0 = [one_body(omega, "z")]
    for c, a in zip(cxyz, "xyz"):
        if c != 0.0:
            # (J/n) c S_a^2 = (J c / n) * ((1/2) sum_{i<j} s_a s_a + n/4); the constant is a global phase.
            h0.append(all_pairs(0.5 * Jc * c / n, a + a))
    w = Workload(f"allpairs{n}", n, "symmetric", 1, h0, global_controls(), N, dt, u[0], J=Jc,
                 seed=seed)
    w.notes["u_candidates"] = u
    w.notes["rng"] = rng
    return w


def config3_list(seed=0, count=256):
    """256 independent ring problems: n from {8,10,12,14}, N in [200,2000], J ~ U[0.5,1.5],
    dt=0.02, 2 global controls ~ U[-1,1]; every block carries state (variant "all")."""
    rng = np.random.default_rng(seed)
    ns = rng.choice([8, 10, 12, 14], count)
    Ns = rng.integers(200, 2001, count)
    out = []
    for p in range(count):
        J = float(rng.uniform(0.5, 1.5))
        u = draw_controls(rng, int(Ns[p]), 2, -1.0, 1.0)
        w = Workload(f"batch{p}_ring{int(ns[p])}", int(ns[p]), "dihedral", 1,
                     heisenberg_ring_terms(J), global_controls(), int(Ns[p]), 0.02, u, J=J,
                     variant="all", seed=seed)
        out.append(w)
    return out, rng
