"""Monolithic Newton with eps-continuation, its Newton systems solved by GMRES with or
without a linear RAS preconditioner (Newton_RAS,eps and Newton_eps; oracle; test
infrastructure only).

Section 4.1 of the paper: Algorithm 1 on the whole system F_eps(x) = 0, where each
Newton system F'_eps(x^k) d = -F_eps(x^k) is solved by GMRES with a one-level
restricted additive Schwarz (RAS) preconditioner built on the partition of
Section 4.2:

    M^{-1} v = sum_i P~_i (R_i F'_eps(x^k) P_i)^{-1} R_i v,

the local matrices being the rows and columns of the global Jacobian at the current
iterate that belong to the overlapping box Omega_i.

Without the preconditioner (precond=False) this is the monolithic Newton_eps of
Section 4.1: GMRES on F'_eps(x^k) d = -F_eps(x^k) itself.

Readings taken where the paper leaves room:
  * the preconditioner is applied from the left: GMRES solves
    M^{-1} F'(x) d = -M^{-1} F(x), and its stopping test is relative to
    ||M^{-1} F(x)||;
  * the outer loop is Algorithm 1 exactly as for the monolithic Newton solves
    (oracle.newton.newton_continuation), with k_max = max_outer;
  * continuation NONE starts at eps_0 = eps_min (the method without eps,
    Newton_RAS), otherwise at the problem's eps_0.
"""
import numpy as np
import scipy.sparse.linalg as spla

from .krylov import gmres
from .newton import newton_continuation
from .schwarz import CONT_NONE, partition, prolong_core
from .system import System


class RasPreconditioner:
    """M^{-1} for the Jacobian J (sparse, the global F'_eps at the current iterate)."""

    def __init__(self, J, subs, n):
        self.subs, self.n = subs, n
        Jc = J.tocsr()
        # unknowns of Omega_i: its nodes in the y block, then in the p block (R_i)
        self.idx = [np.concatenate([s.rows, n + s.rows]) for s in subs]
        self.lu = [spla.splu(Jc[ix][:, ix].tocsc()) for ix in self.idx]

    def apply(self, v):
        out = np.zeros(2 * self.n)
        for sub, ix, lu in zip(self.subs, self.idx, self.lu):
            out += prolong_core(sub, lu.solve(v[ix]), self.n)
        return out


class NewtonRas:
    """Newton_RAS,eps (precond=True) or Newton_eps (precond=False) for one problem
    instance (prob: synth.Problem, opts: synth.Options)."""

    def __init__(self, prob, opts, yd, f=None, precond=True):
        self.prob, self.opts, self.precond = prob, opts, precond
        self.sys = System(prob, yd, f)
        self.n = self.sys.n
        self.subs = partition(prob.nx, prob.ny, prob.sx, prob.sy, prob.overlap)
        self.gmres_its = []     # GMRES products of every Newton system
        self.gmres_rel = []

    def linsolve(self, J, b):
        """d with M^{-1} J d = M^{-1} b by GMRES (left RAS preconditioning), or J d = b."""
        o = self.opts
        Jc = J.tocsr()
        if self.precond:
            M = RasPreconditioner(J, self.subs, self.n)
            d, used, rel = gmres(lambda v: M.apply(Jc @ v), M.apply(b), o.gmres_restart, o.gmres_rtol,
                                 o.max_gmres)
        else:
            d, used, rel = gmres(lambda v: Jc @ v, b, o.gmres_restart, o.gmres_rtol, o.max_gmres)
        self.gmres_its.append(used)
        self.gmres_rel.append(rel)
        return d

    def solve(self, x0=None):
        """Returns dict(x, y, p, u, status, iterations, backtracks, residual, gmres_its)."""
        p, o = self.prob, self.opts
        n = self.n
        x0 = np.zeros(2 * n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        eps0 = p.eps_min if o.continuation == CONT_NONE else p.eps0
        x, info = newton_continuation(self.sys.residual, self.sys.jacobian, x0, eps0, p.eps_min, p.gamma,
                                      o.sigma, o.tol_outer, o.max_outer, o.alpha_min, linsolve=self.linsolve)
        return dict(x=x, y=x[:n].copy(), p=x[n:].copy(), u=self.sys.control(x, p.eps_min),
                    status=info.status, iterations=info.iterations, backtracks=info.backtracks,
                    residual=info.residual, residual0=info.residual0, eps=info.eps,
                    gmres_its=list(self.gmres_its), gmres_rel=list(self.gmres_rel))
