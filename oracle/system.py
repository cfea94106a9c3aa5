"""Discrete smoothed optimality system on the whole grid (oracle; test infrastructure only).

Discretisation (Section 4, model problem; Section 5): Omega = (0,1)^2, A = -Laplacian
by the 5-point finite-difference stencil with homogeneous Dirichlet data, nodal
unknowns at the interior nodes, vectors ordered row-major [ny][nx] (x fastest).

Unknown x = (y, p) in R^{2n}, n = nx*ny.  With g(p) = p + mu P_eps(-p/mu):

  F_eps(x)  = [ A y + phi(y) - f + g(p)/nu ;  A p + phi'(y) p - y + y_d ]
  F'_eps(x) = [[ A + phi'(y),      g'(p)/nu  ],
               [ phi''(y) p - I,   A + phi'(y) ]]

(Section 4: the map F(x, eps) and its partial derivative in x.)
"""
import numpy as np
import scipy.sparse as sp

from . import pointwise as pw


def laplacian_1d(n, h):
    """tridiag(-1, 2, -1) / h^2 of order n."""
    e = np.ones(n)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr") / (h * h)


def laplacian(nx, ny):
    """5-point -Laplacian on the nx x ny interior grid, x index fastest:
    A = kron(I_ny, T_x) + kron(T_y, I_nx)."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    return (sp.kron(sp.identity(ny), laplacian_1d(nx, hx))
            + sp.kron(laplacian_1d(ny, hy), sp.identity(nx))).tocsr()


class System:
    """F_eps and F'_eps for one problem instance.

    prob: a synth.Problem (nx, ny, phi, kappa, nu, mu); yd, f: [ny][nx] arrays.
    """

    def __init__(self, prob, yd, f=None):
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        self.n = prob.nx * prob.ny
        self.A = laplacian(prob.nx, prob.ny)
        self.yd = np.asarray(yd, dtype=np.float64).reshape(-1).copy()
        self.f = (np.zeros(self.n) if f is None
                  else np.asarray(f, dtype=np.float64).reshape(-1).copy())

    # -- pointwise pieces --------------------------------------------------
    def _phi(self, y):
        return pw.phi(y, self.prob.phi, self.prob.kappa)

    def _dphi(self, y):
        return pw.dphi(y, self.prob.phi, self.prob.kappa)

    def _ddphi(self, y):
        return pw.ddphi(y, self.prob.phi, self.prob.kappa)

    def split(self, x):
        return x[: self.n], x[self.n:]

    # -- F on all rows ------------------------------------------------------
    def residual(self, x, eps):
        y, p = self.split(x)
        nu, mu = self.prob.nu, self.prob.mu
        r1 = self.A @ y + self._phi(y) - self.f + pw.g(p, mu, eps) / nu
        r2 = self.A @ p + self._dphi(y) * p - y + self.yd
        return np.concatenate([r1, r2])

    def jacobian(self, x, eps):
        y, p = self.split(x)
        nu, mu = self.prob.nu, self.prob.mu
        D = sp.diags(self._dphi(y))
        top = sp.hstack([self.A + D, sp.diags(pw.dg(p, mu, eps) / nu)])
        bot = sp.hstack([sp.diags(self._ddphi(y) * p - 1.0), self.A + D])
        return sp.vstack([top, bot]).tocsc()

    # -- F on a subset of node rows (R_i F) --------------------------------
    def residual_rows(self, x, eps, rows, A_rows):
        """Rows ``rows`` (node indices) of both equations of F_eps at the full vector x;
        A_rows must be A[rows, :].  Equals residual(x, eps)[[rows, n + rows]]."""
        y, p = self.split(x)
        nu, mu = self.prob.nu, self.prob.mu
        yr, pr = y[rows], p[rows]
        r1 = A_rows @ y + self._phi(yr) - self.f[rows] + pw.g(pr, mu, eps) / nu
        r2 = A_rows @ p + self._dphi(yr) * pr - yr + self.yd[rows]
        return np.concatenate([r1, r2])

    def jacobian_rows_cols(self, x, eps, rows, A_sub):
        """F'_eps(x) restricted to rows and columns ``rows`` of both fields;
        A_sub must be A[rows][:, rows]."""
        y, p = self.split(x)
        nu, mu = self.prob.nu, self.prob.mu
        yr, pr = y[rows], p[rows]
        D = sp.diags(self._dphi(yr))
        top = sp.hstack([A_sub + D, sp.diags(pw.dg(pr, mu, eps) / nu)])
        bot = sp.hstack([sp.diags(self._ddphi(yr) * pr - 1.0), A_sub + D])
        return sp.vstack([top, bot]).tocsc()

    def jacobian_rows_apply(self, x, eps, rows, A_rows, d):
        """(F'_eps(x) d) restricted to rows ``rows`` of both fields."""
        y, p = self.split(x)
        dy, dp = self.split(d)
        nu, mu = self.prob.nu, self.prob.mu
        yr, pr = y[rows], p[rows]
        a = self._dphi(yr)
        r1 = A_rows @ dy + a * dy[rows] + pw.dg(pr, mu, eps) / nu * dp[rows]
        r2 = (self._ddphi(yr) * pr - 1.0) * dy[rows] + A_rows @ dp + a * dp[rows]
        return np.concatenate([r1, r2])

    def control(self, x, eps):
        _, p = self.split(x)
        return pw.control(p, self.prob.nu, self.prob.mu, eps)
