"""Device slice propagators (Eq. (3)) against eigendecomposition propagators of the oracle."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import grape as og
from tests._common import oracle_blocks

pytestmark = pytest.mark.gpu


def _run(lib, n, h0, hk, u, dt, prec, group="dihedral", stride=1, u_bound=None):
    import torch
    B = lib.Basis(n, group, stride)
    S = lib.System(B, h0, hk)
    P = lib.Plan(S, prec, u.shape[0], dt, float(np.abs(u).max()) if u_bound is None else u_bound)
    Us = lib.propagate(P, torch.tensor(u, device="cuda"))
    return B, P, [U.cpu().numpy() for U in Us]


@pytest.mark.parametrize("prec,tol", [("c128", 1e-12), ("c64", 3e-6)])
@pytest.mark.parametrize("dt", [0.05, 0.4])
def test_propagators_config1_blocks(lib, prec, tol, dt):
    print(f"propagate prec={prec} dt={dt}", flush=True)
    w = W.config1(N=6)
    B, P, Us = _run(lib, 6, w.h0, w.hk, w.u, dt, prec)
    ob = oracle_blocks(6, w.h0, w.hk)
    for b, blk in enumerate(ob):
        for j in range(6):
            Uo = og.propagator(blk["H0"], blk["Hk"], w.u[j], dt)
            assert np.abs(Us[b][j] - Uo).max() < tol, (blk["label"], j)
            m = blk["m"]
            assert np.abs(Us[b][j].conj().T @ Us[b][j] - np.eye(m)).max() < 4 * tol


@pytest.mark.parametrize("prec,tol", [("c128", 2e-12), ("c64", 2e-5)])
def test_propagators_ragged_tiles(lib, prec, tol):
    """n = 10 blocks of 30..105 rows: several 64-wide tiles with ragged edges."""
    print(f"propagate ragged prec={prec}", flush=True)
    rng = np.random.default_rng(3)
    n = 10
    h0 = W.full_coupling_terms(n, 1.1, [0.4, 0.3, 0.2, 0.1, 0.05])
    hk = [[W.one_body(0.5, "x")], [W.one_body(0.5, "y")]]
    u = rng.uniform(-2, 2, (3, 2))
    B, P, Us = _run(lib, n, h0, hk, u, 0.1, prec)
    ob = oracle_blocks(n, h0, hk)
    for b, blk in enumerate(ob):
        for j in range(3):
            Uo = og.propagator(blk["H0"], blk["Hk"], u[j], 0.1)
            assert np.abs(Us[b][j] - Uo).max() < tol, (blk["label"], j)


def test_squarings_engage_for_large_norm(lib):
    """A large dt forces scaling and squaring; the result still matches."""
    w = W.config1(N=2)
    B, P, Us = _run(lib, 6, w.h0, w.hk, w.u, 3.0, "c128")
    assert P.info["max_squarings"] >= 3
    ob = oracle_blocks(6, w.h0, w.hk)
    for b, blk in enumerate(ob):
        Uo = og.propagator(blk["H0"], blk["Hk"], w.u[1], 3.0)
        assert np.abs(Us[b][1] - Uo).max() < 1e-11


@pytest.mark.parametrize("prec,tol", [("c128", 2e-12), ("c64", 3e-6)])
def test_both_taylor_evaluations_match(lib, prec, tol):
    """Norms from 1e-3 to ~4 make an FP32 plan pick Paterson-Stockmeyer degrees (q >= 1) and
    the four-product degree-12 evaluation (q = 0), with and without squarings (FP64 plans
    use Paterson-Stockmeyer only); every propagator matches the oracle's
    eigendecomposition."""
    import torch
    print(f"both Taylor evaluations {prec}", flush=True)
    w = W.config1(N=4)
    ob = oracle_blocks(6, w.h0, w.hk)
    seen = set()
    for dt in (0.0005, 0.005, 0.03, 0.08, 0.15, 0.3, 0.6, 1.2):
        B, P, Us = _run(lib, 6, w.h0, w.hk, w.u, dt, prec)
        qs, ss, _ = lib.slice_stats(P, torch.tensor(w.u, device="cuda"))
        for b, blk in enumerate(ob):
            for j in range(4):
                seen.add((int(qs[b, j]) == 0, int(ss[b, j]) > 0))
                Uo = og.propagator(blk["H0"], blk["Hk"], w.u[j], dt)
                assert np.abs(Us[b][j] - Uo).max() < tol, (dt, blk["label"], j, int(qs[b, j]), int(ss[b, j]))
    print(f"  (degree-12 scheme, squarings) combinations seen: {sorted(seen)}", flush=True)
    if prec == "c64":
        assert (True, False) in seen and (True, True) in seen and (False, False) in seen
    else:
        assert not any(t12 for t12, _ in seen) and (False, True) in seen and (False, False) in seen
