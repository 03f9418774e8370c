"""GRAPE pulse optimisation by limited-memory BFGS ascent, FP64 (test infrastructure only).

GRAPE (Sec. I; App. B) raises the objective F of Eq. (4) by gradient steps on every
slice sample u[j, k]; the paper's update rule sits in its Supplementary Material, which
is not available, so the rule here is the standard limited-memory BFGS method (Nocedal,
Math. Comp. 35, 1980; Liu & Nocedal, Math. Prog. 45, 1989) with a backtracking Armijo
line search, applied to F as a function of the flattened controls:

* direction d = H g, H the L-BFGS inverse-Hessian estimate of f = -F built from the
  last M accepted pairs s = u_new - u_old, y = g_old - g_new (g = dF/du), starting from
  H0 = gamma I, gamma = s.y / y.y of the newest pair, evaluated by the two-loop recursion;
  with no stored pair, d = (step0 / max_i |g_i|) g, so the first trial moves the largest
  control by step0;
* a pair is kept only when s.y > 1e-10 sqrt(s.s y.y) (curvature condition), which keeps H
  positive definite; the oldest pair is dropped beyond M;
* if g.d <= 0 the memory is cleared and the first-step direction is used;
* line search: alpha = 1, 1/2, 1/4, ... (at most max_backtrack halvings after the first
  trial); a trial is accepted when it is valid (finite, within the plan's norm bound) and
  F(u + alpha d) >= F(u) + c1 alpha g.d;
* stop when F >= f_target (reason 0), max |g| <= gtol (1), after max_iter accepted steps
  (2), or when no trial of a line search is accepted (3).

``lbfgs_ascent`` takes the objective as a callable, so the pins can drive it with closed
forms; ``grape_objective`` wraps the FP64 GRAPE oracle of ``grape``.
"""
from __future__ import annotations

import numpy as np

from . import grape

TARGET, GTOL, MAX_ITER, LINE_SEARCH_FAILED = 0, 1, 2, 3
CURVATURE_EPS = 1e-10


def two_loop(g, pairs):
    """H g for the L-BFGS inverse-Hessian estimate of the stored pairs (oldest first),
    H0 = gamma I with gamma from the newest pair (Nocedal & Wright, Numerical
    Optimization, Algorithm 7.4)."""
    q = np.array(g, dtype=float, copy=True)
    alphas = []
    for s, y in reversed(pairs):
        rho = 1.0 / np.dot(s, y)
        a = rho * np.dot(s, q)
        q = q - a * y
        alphas.append(a)
    s_new, y_new = pairs[-1]
    r = (np.dot(s_new, y_new) / np.dot(y_new, y_new)) * q
    for (s, y), a in zip(pairs, reversed(alphas)):
        rho = 1.0 / np.dot(s, y)
        b = rho * np.dot(y, r)
        r = r + (a - b) * s
    return r


def first_direction(g, step0):
    gmax = np.max(np.abs(g))
    return (step0 / gmax) * g


def lbfgs_ascent(fun, u0, memory=10, step0=0.1, c1=1e-4, max_backtrack=20, max_iter=100,
                 f_target=1.0, gtol=0.0):
    """Maximise fun over u.  fun(u) -> (F, grad, valid).  Returns a dict with the final
    u, F and gradient, the history of F at u0 and after every accepted step, the number of
    objective evaluations and the stop reason."""
    u = np.array(u0, dtype=float, copy=True)
    F, g, ok = fun(u)
    if not ok:
        raise ValueError("the starting point is not a valid evaluation")
    hist, evals, pairs = [F], 1, []
    reason = MAX_ITER
    for _ in range(max_iter):
        if F >= f_target:
            reason = TARGET
            break
        if np.max(np.abs(g)) <= gtol:
            reason = GTOL
            break
        d = two_loop(g, pairs) if pairs else first_direction(g, step0)
        gd = np.dot(g, d)
        if gd <= 0.0:
            pairs = []
            d = first_direction(g, step0)
            gd = np.dot(g, d)
        alpha, accepted = 1.0, False
        for _b in range(max_backtrack + 1):
            ut = u + alpha * d
            Ft, gt, okt = fun(ut)
            evals += 1
            if okt and np.isfinite(Ft) and Ft >= F + c1 * alpha * gd:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            reason = LINE_SEARCH_FAILED
            break
        s, y = ut - u, g - gt
        sy, ss, yy = np.dot(s, y), np.dot(s, s), np.dot(y, y)
        if sy > CURVATURE_EPS * np.sqrt(ss * yy):
            pairs.append((s, y))
            if len(pairs) > memory:
                pairs.pop(0)
        u, F, g = ut, Ft, gt
        hist.append(F)
    else:
        reason = MAX_ITER
    if reason == MAX_ITER and F >= f_target:
        reason = TARGET
    return {"u": u, "F": F, "grad": g, "hist": np.array(hist), "evals": evals, "reason": reason}


def _norm1(A):
    return float(np.max(np.sum(np.abs(A), axis=0)))


def grape_objective(blocks, dt, psi0, psif, shape, u_bound=None):
    """fun(u_flat) for lbfgs_ascent: F and dF/du of the block system (Eq. (4); App. B),
    the controls reshaped to (N, K).  With u_bound, a trial is invalid when some slice's
    dt ||H0 + sum_k u[j,k] H_k||_1 exceeds the largest over the blocks of
    dt (||H0||_1 + u_bound sum_k ||H_k||_1), the norm bound an execution plan derives from
    u_bound (triangle inequality on the blocks' exact 1-norms)."""
    nb = None
    if u_bound is not None:
        nb = max(dt * (_norm1(b["H0"]) + u_bound * sum(_norm1(H) for H in b["Hk"])) for b in blocks)

    def fun(uf):
        u = uf.reshape(shape)
        if nb is not None:
            for b in blocks:
                for j in range(shape[0]):
                    if dt * _norm1(grape.slice_hamiltonian(b["H0"], b["Hk"], u[j])) > nb * (1 + 1e-12):
                        return -np.inf, np.zeros_like(uf), False
        r = grape.fidelity_grad(blocks, u, dt, psi0, psif)
        return r["F"], np.asarray(r["grad"]).reshape(-1), bool(np.isfinite(r["F"]))
    return fun
