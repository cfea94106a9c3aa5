"""Shared test problems built on the CPU (closed forms and the oracle only)."""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle.system import System


def lq_direct(nx, ny, nu, yd, f):
    """[[A, I/nu], [-I, A]] x = [f; -y_d], the eps-independent linear system for
    phi = 0, mu = 0, assembled here from kron and solved by SuperLU."""
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    Tx = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(nx, nx)) / hx ** 2
    Ty = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(ny, ny)) / hy ** 2
    A = sp.kron(sp.eye(ny), Tx) + sp.kron(Ty, sp.eye(nx))
    n = nx * ny
    K = sp.bmat([[A, sp.eye(n) / nu], [-sp.eye(n), A]]).tocsc()
    return spla.spsolve(K, np.concatenate([f.reshape(-1), -yd.reshape(-1)]))


def mms_problem(kind, nx, ny, sx, sy, ov, eps_min=1e-6):
    """Manufactured solution in the spirit of Section 4 (pick p crossing +-mu and y,
    derive f and y_d so that F_eps(y, p) = 0): f and y_d come from the oracle's own F."""
    prob = synth.Problem(nx=nx, ny=ny, phi=kind, nu=1e-2, mu=0.02, eps0=1.0,
                         eps_min=eps_min, gamma=0.5, sx=sx, sy=sy, overlap=ov)
    X, Y = synth.node_coords(nx, ny)
    ys = 0.6 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    ps = 0.05 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    s0 = System(prob, np.zeros((ny, nx)), np.zeros((ny, nx)))
    x = np.concatenate([ys.reshape(-1), ps.reshape(-1)])
    r = s0.residual(x, eps_min)
    f = r[:s0.n].reshape(ny, nx)              # F_1(x*) - f = r_1 with f = 0  =>  f := r_1
    yd = -r[s0.n:].reshape(ny, nx)            # F_2 = ... + y_d              =>  y_d := -r_2
    return prob, yd, f, x


def paper_model_problem(n, sx, sy, ov, eps_min, gamma=0.2, k=5, eps_bar=1e-15):
    """The numerical model problem of Section 4 (eqs. (ppp), (pppp), (ydpppp)): phi(y) = kappa (y^3 + exp(kappa y)),
    kappa = 0.1, nu = 1e-6, mu = 1, f = 0 on an n x n grid, with
      p_bar = 1.3 mu sin(2 pi k x1) sin(2 pi k x2)                            eq. (ppp),
      y_bar: A y + phi(y) - f + g_eps(p_bar) / nu = 0 at eps = eps_bar        eq. (pppp),
      y_d = -A p_bar - phi'(y_bar) p_bar + y_bar                              eq. (ydpppp),
    so (y_bar, p_bar) solves F_eps_bar = 0 (the sign of the g term as in F).  y_bar is
    found by damped Newton on that monotone equation (A + diag phi' is SPD)."""
    from oracle import pointwise as pw
    prob = synth.Problem(nx=n, ny=n, phi=synth.PHI_PAPER, kappa=0.1, nu=1e-6, mu=1.0, eps0=1.0,
                         eps_min=eps_min, gamma=gamma, sx=sx, sy=sy, overlap=ov)
    X, Y = synth.node_coords(n, n)
    pbar = (1.3 * prob.mu * np.sin(2 * math.pi * k * X) * np.sin(2 * math.pi * k * Y)).reshape(-1)
    zero = np.zeros((n, n))
    s = System(prob, zero, zero)
    c = pw.g(pbar, prob.mu, eps_bar) / prob.nu
    y = np.zeros(n * n)
    G = s.A @ y + s._phi(y) + c
    for _ in range(100):
        r = np.linalg.norm(G)
        if r <= 1e-9 * max(1.0, np.linalg.norm(c)):
            break
        d = spla.spsolve((s.A + sp.diags(s._dphi(y))).tocsc(), -G)
        a = 1.0
        while True:
            yt = y + a * d
            Gt = s.A @ yt + s._phi(yt) + c
            if np.linalg.norm(Gt) < r or a < 1e-12:
                break
            a *= 0.5
        y, G = yt, Gt
    else:
        raise RuntimeError("the state equation of the model problem did not converge")
    yd = (-(s.A @ pbar) - s._dphi(y) * pbar + y).reshape(n, n)
    return prob, yd, zero, np.concatenate([y, pbar])


def paper_inner_tol(nx, ny, tol=1e-8):
    """The absolute branch of the inner tolerance of Section 5 (1e-8) in the units of F
    here (the relative branch, tol |K(0)|, has no units and keeps 1e-8).

    F is the 5-point system with A = -Laplacian / h^2, unscaled.  The paper's tolerance
    is read as one on the residual of the equations multiplied by the cell area hx*hy
    (the scaling of a finite-element or h^2-scaled difference code), so it becomes
    tol / (hx hy) here.  Taken unscaled, 1e-8 lies below what FP64 can resolve in a
    local residual of the model problem: at N = 450 the rounding of one evaluation of
    F on a 45 x 45 box alone is about 4e-8 (test_model_problem_local_rounding_floor)."""
    return tol * (nx + 1) * (ny + 1)
