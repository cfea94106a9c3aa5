"""Discrete smoothed optimality system on the whole grid (oracle; test infrastructure only).

Discretisation (Section 4, model problem; Section 5): Omega = (0,1)^2, A = -Laplacian
by the 5-point finite-difference stencil with homogeneous Dirichlet data, nodal
unknowns at the interior nodes, vectors ordered row-major [ny][nx] (x fastest).
Assumption 1 (3) allows any symmetric uniformly elliptic A = -div(a grad) + a0; for a
diagonal coefficient tensor (a1, a2) and a0 >= 0 the same stencil in flux form gives
  (A y)_ij = sum over the four faces f of node ij of a_f (y_ij - y_nb(f)) / h_f^2 + a0_ij y_ij
with a1 at the x-faces, a2 at the y-faces and y = 0 on the boundary
(``variable_operator``; face layout as ``synth.coefficient_fields``).

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


def variable_operator(nx, ny, ax, ay, a0):
    """A = Dx^T diag(ax / hx^2) Dx + Dy^T diag(ay / hy^2) Dy + diag(a0): Dx takes the
    difference y_i - y_{i-1} across each x-face (i = 0..nx, with the boundary values
    zero), Dy across each y-face.  ax: [ny][nx+1], ay: [ny+1][nx], a0: [ny][nx]."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    n = nx * ny
    rows, cols, vals = [], [], []
    for j in range(ny):
        for i in range(nx + 1):
            r = j * (nx + 1) + i
            if i < nx:
                rows.append(r); cols.append(j * nx + i); vals.append(1.0)
            if i > 0:
                rows.append(r); cols.append(j * nx + i - 1); vals.append(-1.0)
    Dx = sp.csr_matrix((vals, (rows, cols)), shape=(ny * (nx + 1), n))
    rows, cols, vals = [], [], []
    for j in range(ny + 1):
        for i in range(nx):
            r = j * nx + i
            if j < ny:
                rows.append(r); cols.append(j * nx + i); vals.append(1.0)
            if j > 0:
                rows.append(r); cols.append((j - 1) * nx + i); vals.append(-1.0)
    Dy = sp.csr_matrix((vals, (rows, cols)), shape=((ny + 1) * nx, n))
    A = (Dx.T @ sp.diags(np.ravel(ax) / (hx * hx)) @ Dx + Dy.T @ sp.diags(np.ravel(ay) / (hy * hy)) @ Dy
         + sp.diags(np.ravel(a0)))
    return A.tocsr()


class System:
    """F_eps and F'_eps for one problem instance.

    prob: a synth.Problem (nx, ny, phi, kappa, nu, mu; with coef set, A takes the
    problem's coefficient fields); yd, f: [ny][nx] arrays.
    """

    def __init__(self, prob, yd, f=None):
        self.prob = prob
        self.nx, self.ny = prob.nx, prob.ny
        self.n = prob.nx * prob.ny
        cf = prob.coefficients() if getattr(prob, "coef", 0) else None
        self.A = laplacian(prob.nx, prob.ny) if cf is None else variable_operator(prob.nx, prob.ny, *cf)
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
