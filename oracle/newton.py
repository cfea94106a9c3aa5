"""Algorithm 1 of the paper: damped Newton with eps-continuation and relaxed
backtracking line search (oracle; test infrastructure only).

Readings taken where the paper leaves room:
  * the loop also continues while eps_k > eps_min, so a continued solve always
    ends at the target smoothing;
  * backtracking halves alpha while NOT (||F(x + alpha d)|| <= sigma ||F(x)||), so
    a NaN trial is rejected like a too-large one; below alpha_min the solve stops
    with status LINESEARCH_FAIL and keeps the last accepted iterate;
  * norms are Euclidean norms of the discrete vectors; a NaN residual never
    counts as converged (the loop test is written as NOT (||F|| <= threshold)).
"""
import dataclasses

import numpy as np
import scipy.sparse.linalg as spla

CONVERGED, NOT_CONVERGED, LINESEARCH_FAIL = 0, 1, 2


@dataclasses.dataclass
class NewtonInfo:
    status: int
    iterations: int
    backtracks: int
    residual: float
    residual0: float
    eps: float


def newton_continuation(residual, jacobian, x0, eps0, eps_min, gamma, sigma,
                        tol, kmax, alpha_min, linsolve=None, on_step=None, tol_rel=None):
    """Algorithm 1.

    residual(x, eps) -> F_eps(x);  jacobian(x, eps) -> sparse F'_eps(x).
    The loop runs while (||F_{eps_k}(x^k)|| > max(tol, tol_rel ||F_{eps_0}(x^0)||) or
    eps_k > eps_min) and k <= kmax (tol_rel = tol unless given: the algorithm uses one
    tolerance for both branches; a tolerance in the units of F and a relative one may
    differ when F is scaled): solve F'_{eps_k}(x^k) d = -F_{eps_k}(x^k),
    backtrack alpha = 1, 1/2, ... until ||F_{eps_k}(x^k + alpha d)|| <= sigma ||F_{eps_k}(x^k)||,
    then x^{k+1} = x^k + alpha d, eps_{k+1} = max(gamma eps_k, eps_min).
    on_step(k, x, eps) is called after every accepted update.
    """
    solve = linsolve or (lambda J, b: spla.spsolve(J, b))
    x = np.array(x0, dtype=np.float64, copy=True)
    eps = float(eps0)
    Fx = residual(x, eps)
    r = float(np.linalg.norm(Fx))
    r0 = r
    thresh = max(tol, (tol if tol_rel is None else tol_rel) * r0)
    k = 0
    backtracks = 0
    status = CONVERGED
    while (not (r <= thresh) or eps > eps_min) and k <= kmax:
        d = solve(jacobian(x, eps), -Fx)
        alpha = 1.0
        while True:
            rt = float(np.linalg.norm(residual(x + alpha * d, eps)))
            if rt <= sigma * r:
                break
            alpha *= 0.5
            backtracks += 1
            if alpha < alpha_min:
                status = LINESEARCH_FAIL
                break
        if status == LINESEARCH_FAIL:
            break
        x = x + alpha * d
        eps = max(gamma * eps, eps_min)
        k += 1
        Fx = residual(x, eps)
        r = float(np.linalg.norm(Fx))
        if on_step is not None:
            on_step(k, x, eps)
    if status == CONVERGED and (not (r <= thresh) or eps > eps_min):
        status = NOT_CONVERGED
    return x, NewtonInfo(status, k, backtracks, r, r0, eps)
