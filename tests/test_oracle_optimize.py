"""Pins for the oracle's L-BFGS ascent (oracle/optimize.py): the two-loop recursion against
the explicit BFGS inverse-Hessian update, convergence to the maximiser of a concave
quadratic, the first-step scaling, the line search's handling of invalid trials, and the
GRAPE objective wrapper's norm-bound rule."""
import numpy as np
import pytest

import qoc_workloads as W
from oracle import grape
from oracle import optimize as opt


def _spd(rng, n, cond):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.geomspace(1.0, cond, n)) @ Q.T


@pytest.mark.parametrize("npairs", [1, 3, 7])
def test_two_loop_equals_explicit_bfgs_update(npairs):
    """The two-loop recursion evaluates H g for the matrix built by the BFGS inverse update
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, applied oldest pair first from
    H0 = gamma I (gamma from the newest pair)."""
    rng = np.random.default_rng(40 + npairs)
    n = 9
    A = _spd(rng, n, 30.0)
    pairs = []
    for _ in range(npairs):
        s = rng.standard_normal(n)
        pairs.append((s, A @ s))  # s.y > 0
    g = rng.standard_normal(n)
    s_new, y_new = pairs[-1]
    H = (s_new @ y_new) / (y_new @ y_new) * np.eye(n)
    for s, y in pairs:
        rho = 1.0 / (s @ y)
        L = np.eye(n) - rho * np.outer(s, y)
        H = L @ H @ L.T + rho * np.outer(s, s)
    ref = H @ g
    got = opt.two_loop(g, pairs)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # the estimate satisfies the newest secant equation H y = s
    assert np.abs(opt.two_loop(y_new, pairs) - s_new).max() <= 1e-10 * np.abs(s_new).max()


def test_concave_quadratic_reaches_the_maximiser():
    rng = np.random.default_rng(7)
    n = 8
    A = _spd(rng, n, 100.0)
    ustar = rng.standard_normal(n)

    def fun(u):
        e = u - ustar
        return 1.0 - 0.5 * e @ A @ e, -(A @ e), True

    r = opt.lbfgs_ascent(fun, np.zeros(n), memory=10, step0=0.5, max_iter=200, f_target=2.0, gtol=1e-11)
    assert r["reason"] == opt.GTOL
    assert np.abs(r["u"] - ustar).max() <= 1e-9
    assert np.all(np.diff(r["hist"]) >= 0.0)  # Armijo: every accepted step raises F
    assert len(r["hist"]) <= 60


def test_first_step_moves_the_largest_control_by_step0():
    rng = np.random.default_rng(3)
    n = 5
    A = _spd(rng, n, 4.0)
    ustar = 10.0 * rng.standard_normal(n)

    def fun(u):
        e = u - ustar
        return -0.5 * e @ A @ e, -(A @ e), True

    u0 = np.zeros(n)
    r = opt.lbfgs_ascent(fun, u0, step0=0.01, max_iter=1, f_target=np.inf)
    assert r["evals"] == 2  # the first trial (alpha = 1) is accepted for a small step
    assert abs(np.abs(r["u"] - u0).max() - 0.01) <= 1e-15
    g0 = A @ ustar
    assert np.allclose(r["u"], 0.01 * g0 / np.abs(g0).max(), rtol=0, atol=1e-15)


def test_line_search_backtracks_over_invalid_trials_and_reports_failure():
    # F grows without bound along +u, but trials with any |u| > 1 are invalid
    def fun(u):
        if np.abs(u).max() > 1.0:
            return -np.inf, np.zeros_like(u), False
        return float(u.sum()), np.ones_like(u), True

    r = opt.lbfgs_ascent(fun, np.zeros(3), step0=0.8, max_iter=50, max_backtrack=10, f_target=np.inf)
    assert np.abs(r["u"]).max() <= 1.0
    assert r["reason"] == opt.LINE_SEARCH_FAILED
    assert np.all(np.diff(r["hist"]) > 0.0)
    with pytest.raises(ValueError):
        opt.lbfgs_ascent(fun, 2.0 * np.ones(3))


def test_stop_reasons_target_and_iterations():
    def fun(u):
        return float(1.0 - (u[0] - 1.0) ** 2), np.array([-2.0 * (u[0] - 1.0)]), True

    r = opt.lbfgs_ascent(fun, np.zeros(1), step0=0.5, f_target=0.5)
    assert r["reason"] == opt.TARGET and r["F"] >= 0.5
    r = opt.lbfgs_ascent(fun, np.zeros(1), step0=0.001, max_iter=2, f_target=2.0)
    assert r["reason"] == opt.MAX_ITER and len(r["hist"]) == 3


def test_grape_objective_norm_bound_rule():
    """A trial is valid exactly when every slice's dt ||H_j||_1 stays within
    dt (||H0||_1 + u_bound sum_k ||H_k||_1)."""
    n, N, dt = 4, 6, 0.05
    blocks = grape.block_system(n, W.ising_ring_terms(1.0, 1.0), W.global_controls(0.5))
    b0 = [blocks[0]]
    m = b0[0]["m"]
    p0 = [np.eye(m, dtype=complex)[:, [0]]]
    pf = [np.eye(m, dtype=complex)[:, [m - 1]]]
    fun = opt.grape_objective(b0, dt, p0, pf, (N, 2), u_bound=1.0)
    u = np.full((N, 2), 1.0)
    assert fun(u.reshape(-1))[2]  # |u| = u_bound: within the triangle bound
    n1 = lambda A: np.abs(A).sum(axis=0).max()
    # one control far above u_bound breaks the bound when the other is zero
    u[2] = (1.0 + n1(b0[0]["Hk"][1]) / n1(b0[0]["Hk"][0])) * 1.5, 0.0
    assert not fun(u.reshape(-1))[2]


def test_grape_ascent_transfers_all_up_to_all_down():
    """L-BFGS on the exact gradient raises the transfer F monotonically; with enough time
    and no coupling the transfer is complete (a global pi pulse exists)."""
    n, N, dt = 3, 40, 0.05
    blocks = grape.block_system(n, [W.one_body(0.5, "z")], W.global_controls(0.5))
    b0 = [blocks[0]]
    m = b0[0]["m"]
    up = np.zeros(2 ** n, complex)
    up[0] = 1.0
    dn = np.zeros(2 ** n, complex)
    dn[-1] = 1.0
    p0 = grape.panels_from_dense(blocks, up)[:1]
    pf = grape.panels_from_dense(blocks, dn)[:1]
    assert np.abs(p0[0]).sum() == 1.0 and np.abs(pf[0]).sum() == 1.0 and m == 4
    rng = np.random.default_rng(11)
    u0 = rng.uniform(-0.5, 0.5, (N, 2)).reshape(-1)
    fun = opt.grape_objective(b0, dt, p0, pf, (N, 2))
    r = opt.lbfgs_ascent(fun, u0, step0=0.5, max_iter=80, f_target=0.9999)
    assert r["reason"] == opt.TARGET and r["F"] >= 0.9999
    assert np.all(np.diff(r["hist"]) >= 0.0)
