"""Nonlinear restricted additive Schwarz and RASPEN (oracle; test infrastructure only).

Section 4.2 of the paper:
  * non-overlapping boxes Omega~_i, each enlarged by an overlap into Omega_i;
  * R_i restricts to Omega_i, P_i extends by zero from Omega_i, P~_i keeps only
    the values on Omega~_i (so R_i P_i = I and sum_i P~_i R_i = I);
  * local corrections C_i(x): K_i(C_i(x)) = R_i F_eps(x + P_i C_i(x)) = 0, eq. (c_i)
    (the correction form; eq. (c_i) writes the local solution, which differs by R_i x);
  * RASPEN residual  F_eps(x) = sum_i P~_i C_i(x), eq. (RASPEN def);
  * its Jacobian   F'_eps(x) d = sum_i P~_i C_i'(x) d,
      C_i'(x) = -(R_i F'_eps(x^(i)) P_i)^{-1} R_i F'_eps(x^(i)),  x^(i) = x + P_i C_i(x),
    eq. (raspen der) and eq. (DerC);
  * Algorithm 2 (outer Newton on F_eps = 0 with GMRES, undamped update),
    Algorithm 3 (evaluate F_eps: local Newton solves, assemble),
    Algorithm 4 (apply F'_eps(x) to d with the stored corrections).

Partition reading: per direction, s boxes of width B = ceil(N/s):
[jB, min((j+1)B, N)); Omega_i extends each box by ``overlap`` nodes on every side,
clipped to the grid.  Continuation (eps_0 -> eps_min by gamma) is used in the
local solves of the first evaluation only (Algorithm 2 and Section 5); later
evaluations start every local solve from c = 0 at eps = eps_min.
"""
import dataclasses
import math
from typing import List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .krylov import gmres
from .newton import newton_continuation, CONVERGED, NOT_CONVERGED, LINESEARCH_FAIL
from .system import System

CONT_FIRST, CONT_NONE, CONT_EVERY = 0, 1, 2


def inner_rel_tol(opts):
    """Relative branch of the local stopping test (tol_inner_rel < 0: tol_inner)."""
    r = getattr(opts, "tol_inner_rel", -1.0)
    return opts.tol_inner if r < 0 else r


def split_1d(n, s):
    """Non-overlapping intervals [jB, min((j+1)B, n)), B = ceil(n/s)."""
    if s < 1 or s > n:
        raise ValueError("need 1 <= s <= n")
    B = math.ceil(n / s)
    out = []
    for j in range(s):
        lo, hi = j * B, min((j + 1) * B, n)
        if lo >= hi:
            raise ValueError("empty subdomain: %d boxes of width %d exceed %d nodes" % (s, B, n))
        out.append((lo, hi))
    return out


@dataclasses.dataclass
class Subdomain:
    core: tuple          # (x0, x1, y0, y1) of Omega~_i, half-open
    box: tuple           # (x0, x1, y0, y1) of Omega_i, half-open
    rows: np.ndarray     # global node indices of Omega_i, local row-major order
    core_local: np.ndarray   # positions (in rows) of the Omega~_i nodes
    core_rows: np.ndarray    # their global node indices


def partition(nx, ny, sx, sy, overlap) -> List[Subdomain]:
    subs = []
    for (y0, y1) in split_1d(ny, sy):
        for (x0, x1) in split_1d(nx, sx):
            bx0, bx1 = max(0, x0 - overlap), min(nx, x1 + overlap)
            by0, by1 = max(0, y0 - overlap), min(ny, y1 + overlap)
            jj, ii = np.meshgrid(np.arange(by0, by1), np.arange(bx0, bx1), indexing="ij")
            rows = (jj * nx + ii).reshape(-1)
            core_mask = ((ii >= x0) & (ii < x1) & (jj >= y0) & (jj < y1)).reshape(-1)
            core_local = np.nonzero(core_mask)[0]
            subs.append(Subdomain((x0, x1, y0, y1), (bx0, bx1, by0, by1), rows,
                                  core_local, rows[core_local]))
    return subs


def restrict(sub, v, n):
    """R_i v for v = (v_y, v_p) in R^{2n}."""
    return np.concatenate([v[sub.rows], v[n + sub.rows]])


def prolong(sub, c, n):
    """P_i c: extend the local (c_y, c_p) by zero."""
    out = np.zeros(2 * n)
    m = sub.rows.size
    out[sub.rows] = c[:m]
    out[n + sub.rows] = c[m:]
    return out


def prolong_core(sub, c, n):
    """P~_i c: keep only the Omega~_i values of the local (c_y, c_p)."""
    out = np.zeros(2 * n)
    m = sub.rows.size
    out[sub.core_rows] = c[:m][sub.core_local]
    out[n + sub.core_rows] = c[m:][sub.core_local]
    return out


@dataclasses.dataclass
class EvalInfo:
    inner_iterations: List[int]
    backtracks: List[int]
    status: int


class Raspen:
    """One-level RASPEN for one problem instance (prob: synth.Problem, opts: synth.Options)."""

    def __init__(self, prob, opts, yd, f=None):
        self.prob, self.opts = prob, opts
        self.sys = System(prob, yd, f)
        self.n = self.sys.n
        self.subs = partition(prob.nx, prob.ny, prob.sx, prob.sy, prob.overlap)
        A = self.sys.A
        self.A_rows = [A[s.rows, :].tocsr() for s in self.subs]
        self.A_sub = [A[s.rows][:, s.rows].tocsr() for s in self.subs]
        self.x_loc = [None] * len(self.subs)    # x^(i) = x + P_i C_i(x)
        self.lu = [None] * len(self.subs)

    # -- local problem of subdomain i (eq. (c_i)) ---------------------------
    def local_residual(self, i, x, c, eps):
        sub = self.subs[i]
        return self.sys.residual_rows(x + prolong(sub, c, self.n), eps, sub.rows, self.A_rows[i])

    def local_jacobian(self, i, x, c, eps):
        sub = self.subs[i]
        return self.sys.jacobian_rows_cols(x + prolong(sub, c, self.n), eps, sub.rows, self.A_sub[i])

    def local_solve(self, i, x, eps0, record=None):
        """C_i(x) by Algorithm 1 from c = 0 (eps0 -> eps_min)."""
        p, o = self.prob, self.opts
        m = self.subs[i].rows.size
        cb = None
        if record is not None:
            record.append(np.zeros(2 * m))
            cb = lambda k, c, eps: record.append(c.copy())
        c, info = newton_continuation(
            lambda c, eps: self.local_residual(i, x, c, eps),
            lambda c, eps: self.local_jacobian(i, x, c, eps),
            np.zeros(2 * m), eps0, p.eps_min, p.gamma, o.sigma, o.tol_inner,
            o.max_inner, o.alpha_min, on_step=cb, tol_rel=inner_rel_tol(o))
        return c, info

    # -- Algorithm 3 ----------------------------------------------------------
    def eval_F(self, x, continuation, records=None):
        """F_eps(x) = sum_i P~_i C_i(x); stores x^(i) and the factorisation of
        R_i F'_eps(x^(i)) P_i for Algorithm 4.  records: optional list that gets,
        per subdomain, the list of local iterates c^(0), c^(1), ..."""
        p = self.prob
        eps0 = p.eps0 if continuation else p.eps_min
        out = np.zeros(2 * self.n)
        its, bts, status = [], [], CONVERGED
        for i, sub in enumerate(self.subs):
            rec = [] if records is not None else None
            c, info = self.local_solve(i, x, eps0, rec)
            if records is not None:
                records.append(rec)
            its.append(info.iterations)
            bts.append(info.backtracks)
            status = max(status, info.status)
            out += prolong_core(sub, c, self.n)
            xi = x + prolong(sub, c, self.n)
            self.x_loc[i] = xi
            self.lu[i] = spla.splu(self.sys.jacobian_rows_cols(xi, p.eps_min, sub.rows,
                                                               self.A_sub[i]))
        return out, EvalInfo(its, bts, status)

    # -- Algorithm 4, literal eq. (DerC) ---------------------------------------
    def jac_apply(self, d):
        out = np.zeros(2 * self.n)
        eps = self.prob.eps_min
        for i, sub in enumerate(self.subs):
            rhs = self.sys.jacobian_rows_apply(self.x_loc[i], eps, sub.rows, self.A_rows[i], d)
            out += prolong_core(sub, -self.lu[i].solve(rhs), self.n)
        return out

    # -- second level: coarse correction ---------------------------------------
    # The paper leaves a second level to future work (end of Section 5.3 and
    # Section 6).  Reading taken here: the hybrid two-level Schwarz preconditioner
    # P2 = Q + M^{-1}(I - F' Q) with the one-level RAS part M^{-1} = sum_i P~_i J_i^{-1} R_i
    # and the coarse correction Q = Z (Z^T F'(x) Z)^{-1} Z^T, where column (i, field)
    # of Z is the indicator of the non-overlapping box Omega~_i in that field.  With
    # F_RAS ~ -M^{-1} F and F_RAS' ~ -M^{-1} F' (exact for affine F), the Newton system
    # P2 F'(x) d = -P2 F(x) becomes
    #     F_RAS'(x)(d - Q F'(x) d) - Q F'(x) d = -F_RAS(x) + (F_RAS'(x) + I) Q F(x),
    # whose operator and right-hand side use only the Jacobian action of Algorithm 4,
    # F'(x) of the whole system and the coarse solve.  The outer iteration and its
    # stopping test are those of Algorithm 2.
    def coarse_basis(self):
        """Z: [2n][2S] sparse, column 2 i + f = indicator of Omega~_i in field f."""
        n, S = self.n, len(self.subs)
        rows, cols = [], []
        for i, sub in enumerate(self.subs):
            for fld in range(2):
                rows.append(fld * n + sub.core_rows)
                cols.append(np.full(sub.core_rows.size, 2 * i + fld))
        r = np.concatenate(rows)
        return sp.csr_matrix((np.ones(r.size), (r, np.concatenate(cols))), shape=(2 * n, 2 * S))

    def coarse_operator(self, x, Z=None):
        """A_0 = Z^T F'_eps_min(x) Z (dense [2S][2S])."""
        Z = self.coarse_basis() if Z is None else Z
        return (Z.T @ self.sys.jacobian(x, self.prob.eps_min) @ Z).toarray()

    def two_level_newton_step(self, x, Fx, Z):
        """The direction d of the two-level Newton system above (GMRES on its operator)."""
        o = self.opts
        eps = self.prob.eps_min
        J = self.sys.jacobian(x, eps)
        A0 = (Z.T @ J @ Z).toarray()

        def Q(v):
            return Z @ np.linalg.solve(A0, Z.T @ v)
        QF = Q(self.sys.residual(x, eps))
        rhs = -Fx + self.jac_apply(QF) + QF

        def op(v):
            qv = Q(J @ v)
            return self.jac_apply(v - qv) - qv
        return gmres(op, rhs, o.gmres_restart, o.gmres_rtol, o.max_gmres)

    # -- Algorithm 2 ----------------------------------------------------------
    def solve(self, x0=None, snapshots=False, coarse=None):
        """Returns dict(x, y, p, u, status, history[, snapshots]).  coarse (default: the
        options' `coarse`): the outer Newton systems with the second level above (same
        iteration otherwise)."""
        if coarse is None:
            coarse = bool(getattr(self.opts, "coarse", 0))
        p, o = self.prob, self.opts
        n = self.n
        x = np.zeros(2 * n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        records = [] if snapshots else None
        Fx, info = self.eval_F(x, continuation=(o.continuation != CONT_NONE), records=records)
        hist = [dict(norm=float(np.linalg.norm(Fx)), gmres=0, gmres_rel=0.0,
                     inner=info.inner_iterations, backtracks=info.backtracks)]
        snaps = None
        if snapshots:
            K = max(len(r) for r in records)
            snaps = []
            for k in range(K):
                v = x.copy()
                for sub, rec in zip(self.subs, records):
                    v += prolong_core(sub, rec[min(k, len(rec) - 1)], n)
                snaps.append(v)
        status = info.status
        F0 = hist[0]["norm"]
        k = 0
        Z = self.coarse_basis() if coarse else None
        while not (hist[-1]["norm"] <= max(o.tol_outer, o.tol_outer * F0)) and k < o.max_outer:
            if coarse:
                d, used, rel = self.two_level_newton_step(x, Fx, Z)
            else:
                d, used, rel = gmres(self.jac_apply, -Fx, o.gmres_restart, o.gmres_rtol, o.max_gmres)
            x = x + d
            k += 1
            Fx, info = self.eval_F(x, continuation=(o.continuation == CONT_EVERY))
            status = max(status, info.status)
            hist.append(dict(norm=float(np.linalg.norm(Fx)), gmres=used, gmres_rel=rel,
                             inner=info.inner_iterations, backtracks=info.backtracks))
        if not (hist[-1]["norm"] <= max(o.tol_outer, o.tol_outer * F0)) and status == CONVERGED:
            status = NOT_CONVERGED
        y, pp = x[:n].copy(), x[n:].copy()
        res = dict(x=x, y=y, p=pp, u=self.sys.control(x, p.eps_min), status=status,
                   history=hist, outer=k)
        if snapshots:
            res["snapshots"] = snaps
        return res


def global_newton(prob, opts, yd, f=None, x0=None, eps0=None):
    """Algorithm 1 on the whole system with a sparse direct solve (used by the
    tests as the monolithic reference: F_eps(x) = 0 directly)."""
    sys_ = System(prob, yd, f)
    n = sys_.n
    x0 = np.zeros(2 * n) if x0 is None else x0
    e0 = prob.eps0 if eps0 is None else eps0
    x, info = newton_continuation(sys_.residual, sys_.jacobian, x0, e0, prob.eps_min,
                                  prob.gamma, opts.sigma, opts.tol_outer,
                                  opts.max_inner, opts.alpha_min)
    return x, info, sys_
