"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms
(Lemma 3.1), textbook eigenpairs of the 5-point stencil, manufactured solutions
built from those closed forms, the linear-quadratic case solved by a library
direct solve, RASPEN versus a monolithic Newton solve (F_eps(x) = 0 iff the RASPEN
residual vanishes, Section 4.2), central differences for every Jacobian, and the
algebraic identities of the restriction/prolongation operators.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import pointwise as pw
from oracle.krylov import gmres
from oracle.newton import newton_continuation, CONVERGED, LINESEARCH_FAIL
from oracle.schwarz import (Raspen, global_newton, partition, prolong, prolong_core,
                            restrict, split_1d)
from oracle.system import System, laplacian

from cases import lq_direct, mms_problem

EPS_LIST = [1e-10, 1e-6, 1e-3, 0.5, 3.0, 10.0]
T = np.concatenate([np.linspace(-5, 5, 2001), [-1.0, 0.0, 1.0, 1e-9, -1e-9]])


# ---------------------------------------------------------------- P1: P_eps, P'_eps
def test_P0_is_projection():
    # eq. (smoothProj) at eps = 0 is (|x+1| - |x-1|)/2 = proj_[-1,1] (Section 3.1)
    err = np.abs(pw.P_eps(T, 0.0) - np.clip(T, -1, 1))
    assert np.all(err <= 2.3e-16 * np.maximum(np.abs(T), 1e-300) + 1e-300)   # one rounding


@pytest.mark.parametrize("eps", EPS_LIST)
def test_P_eps_lemma_3_1(eps):
    P, dP = pw.P_eps(T, eps), pw.dP_eps(T, eps)
    # point (iv): |proj - P_eps| <= sqrt(eps)
    assert np.all(np.abs(np.clip(T, -1, 1) - P) <= math.sqrt(eps) + 1e-15)
    # point (i): range [-1, 1], odd, strictly increasing, limits +-1
    assert np.all(np.abs(P) <= 1.0)
    assert np.allclose(pw.P_eps(-T, eps), -P, rtol=0, atol=1e-16)
    assert np.all(np.diff(pw.P_eps(np.sort(T), eps)) >= 0)
    big = pw.P_eps(np.array([-1e9, 1e9]), eps)
    assert abs(big[0] + 1) < 1e-8 and abs(big[1] - 1) < 1e-8
    # point (ii): 0 < P' <= 1/sqrt(1+eps), maximum at 0
    assert np.all(dP > 0) and np.all(dP <= 1 / math.sqrt(1 + eps) * (1 + 1e-15))
    assert abs(pw.dP_eps(0.0, eps) - 1 / math.sqrt(1 + eps)) < 1e-15


@pytest.mark.parametrize("eps", [1e-6, 1e-3, 0.5, 3.0])
def test_dP_is_derivative_of_P(eps):
    h = 1e-5
    t = np.linspace(-3, 3, 601)
    fd = (pw.P_eps(t + h, eps) - pw.P_eps(t - h, eps)) / (2 * h)
    scale = max(1.0, 1.0 / eps) ** 1.5          # third derivative grows like eps^-3/2
    assert np.max(np.abs(fd - pw.dP_eps(t, eps))) < 10 * h * h * scale + 1e-9


@pytest.mark.parametrize("eps", [0.5, 3.0, 10.0])
def test_rationalised_equals_printed_form(eps):
    # Figure 1 plots eq. (smoothProj) on [-4, 4] for eps in {0.5, 3, 10}
    t = np.linspace(-4, 4, 101)
    assert np.max(np.abs(pw.P_eps(t, eps) - pw.P_eps_direct(t, eps))) < 1e-15
    # closed-form values at t = 1: (sqrt(4+eps) - sqrt(eps))/2; eps = 0.5 gives 1/sqrt(2)
    assert abs(pw.P_eps(1.0, eps) - 0.5 * (math.sqrt(4 + eps) - math.sqrt(eps))) < 1e-15
    assert abs(pw.P_eps(1.0, 0.5) - 1 / math.sqrt(2)) < 1e-15


def test_dP_pointwise_limits():
    # Lemma 3.1 (ii): P'_eps -> 1 on |x|<1, 1/2 at |x|=1, 0 on |x|>1 as eps -> 0
    e = 1e-14
    assert abs(pw.dP_eps(0.5, e) - 1) < 1e-12
    assert abs(pw.dP_eps(1.0, e) - 0.5) < 1e-6
    assert abs(pw.dP_eps(1.5, e)) < 1e-12


# ---------------------------------------------------------------- P2: soft threshold
def test_control_is_soft_threshold_at_eps0():
    p = np.linspace(-0.3, 0.3, 1201)
    mu, nu = 0.05, 1e-3
    S = np.where(p > mu, p - mu, np.where(p < -mu, p + mu, 0.0))   # written out, no oracle
    assert np.max(np.abs(pw.control(p, nu, mu, 0.0) + S / nu)) <= 1e-12


@pytest.mark.parametrize("eps", [1e-8, 1e-4, 1e-2, 1.0])
def test_control_soft_threshold_bound(eps):
    p = np.linspace(-0.3, 0.3, 1201)
    mu, nu = 0.05, 1e-3
    S = np.sign(p) * np.maximum(np.abs(p) - mu, 0)
    assert np.all(np.abs(pw.control(p, nu, mu, eps) + S / nu) <= mu * math.sqrt(eps) / nu * (1 + 1e-12))


def test_mu_zero_and_dg():
    p = np.linspace(-1, 1, 11)
    assert np.array_equal(pw.control(p, 0.1, 0.0, 1e-3), -p / 0.1)
    assert np.array_equal(pw.dg(p, 0.0, 1e-3), np.ones_like(p))
    mu, eps, h = 0.05, 1e-3, 1e-7
    q = np.linspace(-0.2, 0.2, 401)
    fd = (pw.g(q + h, mu, eps) - pw.g(q - h, mu, eps)) / (2 * h)
    assert np.max(np.abs(fd - pw.dg(q, mu, eps))) < 1e-6


@pytest.mark.parametrize("kind", [synth.PHI_ZERO, synth.PHI_CUBIC, synth.PHI_EXP, synth.PHI_PAPER])
def test_phi_family(kind):
    y = np.linspace(-2, 2, 81)
    h = 1e-5
    d1 = (pw.phi(y + h, kind) - pw.phi(y - h, kind)) / (2 * h)
    d2 = (pw.dphi(y + h, kind) - pw.dphi(y - h, kind)) / (2 * h)
    assert np.allclose(d1, pw.dphi(y, kind), rtol=1e-8, atol=1e-8)
    assert np.allclose(d2, pw.ddphi(y, kind), rtol=1e-8, atol=1e-8)
    assert np.all(pw.dphi(y, kind) >= 0)            # Assumption 1: phi monotone
    ref = {synth.PHI_ZERO: 0.0, synth.PHI_CUBIC: 8.0, synth.PHI_EXP: math.exp(2) - 1,
           synth.PHI_PAPER: 0.1 * (8 + math.exp(0.2))}[kind]
    assert abs(pw.phi(2.0, kind) - ref) < 1e-14


# ---------------------------------------------------------------- P3: the stencil
def eig(nx, ny, k, l):
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    X, Y = synth.node_coords(nx, ny)
    v = np.sin(k * math.pi * X) * np.sin(l * math.pi * Y)
    lam = 4 / hx ** 2 * math.sin(k * math.pi * hx / 2) ** 2 + 4 / hy ** 2 * math.sin(l * math.pi * hy / 2) ** 2
    return v.reshape(-1), lam


@pytest.mark.parametrize("nx,ny", [(7, 5), (12, 9), (1, 4)])
def test_laplacian_eigenpairs(nx, ny):
    A = laplacian(nx, ny)
    assert abs(A - A.T).max() == 0
    for k in range(1, nx + 1, max(1, nx // 3)):
        for l in range(1, ny + 1, max(1, ny // 3)):
            v, lam = eig(nx, ny, k, l)
            assert np.max(np.abs(A @ v - lam * v)) < 1e-9 * lam


# ---------------------------------------------------------------- P4: F_eps by closed-form MMS
@pytest.mark.parametrize("kind", [synth.PHI_CUBIC, synth.PHI_EXP, synth.PHI_PAPER])
def test_residual_vanishes_at_closed_form_mms(kind):
    nx, ny, nu, mu = 11, 8, 1e-2, 0.05
    vy, ly = eig(nx, ny, 1, 2)
    vp, lp = eig(nx, ny, 2, 1)
    ys, ps = 0.7 * vy, 0.12 * vp              # p* crosses +-mu
    # phi written out independently of the oracle
    ph = {synth.PHI_CUBIC: (ys ** 3, 3 * ys ** 2), synth.PHI_EXP: (np.exp(ys) - 1, np.exp(ys)),
          synth.PHI_PAPER: (0.1 * (ys ** 3 + np.exp(0.1 * ys)), 0.1 * (3 * ys ** 2 + 0.1 * np.exp(0.1 * ys)))}[kind]
    S = np.sign(ps) * np.maximum(np.abs(ps) - mu, 0)
    f = ly * ys + ph[0] + S / nu                       # state line with g_0 = soft threshold
    yd = ys - lp * ps - ph[1] * ps                     # adjoint line
    prob = synth.Problem(nx=nx, ny=ny, phi=kind, nu=nu, mu=mu)
    s = System(prob, yd.reshape(ny, nx), f.reshape(ny, nx))
    x = np.concatenate([ys, ps])
    r0 = s.residual(x, 0.0)
    assert np.max(np.abs(r0)) < 1e-10 * max(ly, lp)
    # eps > 0 only changes the state line, by at most mu sqrt(eps)/nu (Lemma 3.1 (iv))
    for eps in [1e-6, 1e-2]:
        r = s.residual(x, eps)
        assert np.max(np.abs(r[s.n:] - r0[s.n:])) == 0
        assert np.max(np.abs(r[:s.n])) <= mu * math.sqrt(eps) / nu + 1e-9 * ly


@pytest.mark.parametrize("kind", [synth.PHI_CUBIC, synth.PHI_EXP, synth.PHI_PAPER])
def test_jacobian_central_difference(kind):
    prob = synth.Problem(nx=9, ny=7, phi=kind, nu=1e-2, mu=0.02)
    rng = np.random.default_rng(0)
    s = System(prob, rng.standard_normal((7, 9)), rng.standard_normal((7, 9)))
    x = np.concatenate([0.5 * rng.standard_normal(s.n), 0.05 * rng.standard_normal(s.n)])
    d = rng.standard_normal(2 * s.n)
    for eps in [1e-3, 0.3]:
        t = 1e-6
        fd = (s.residual(x + t * d, eps) - s.residual(x - t * d, eps)) / (2 * t)
        Jd = s.jacobian(x, eps) @ d
        assert np.linalg.norm(fd - Jd) < 1e-6 * np.linalg.norm(Jd)


# ---------------------------------------------------------------- Algorithm 1 and GMRES
def test_newton_scalar_and_schedule():
    res = lambda x, e: np.array([x[0] ** 3 - 2.0 + e * 0.0])
    jac = lambda x, e: sp.csc_matrix([[3 * x[0] ** 2]])
    x, info = newton_continuation(res, jac, np.array([1.0]), 1.0, 1e-6, 0.5, 1.1, 1e-12, 200, 2 ** -30)
    assert abs(x[0] - 2 ** (1 / 3)) < 1e-12 and info.status == CONVERGED
    # the continuation must run until eps reaches eps_min: 2^-20 < 1e-6 <= 2^-19
    assert info.iterations == 20 and info.eps == 1e-6
    x, info = newton_continuation(res, jac, np.array([1.0]), 1e-6, 1e-6, 0.5, 1.1, 1e-12, 200, 2 ** -30)
    assert info.iterations < 8


def test_newton_backtracking():
    # undamped Newton on atan diverges from x0 = 1.5; backtracking with sigma = 1 converges
    res = lambda x, e: np.arctan(x)
    jac = lambda x, e: sp.csc_matrix([[1 / (1 + x[0] ** 2)]])
    x, info = newton_continuation(res, jac, np.array([1.5]), 1.0, 1.0, 1.0, 1.0, 1e-12, 100, 2 ** -30)
    assert info.status == CONVERGED and abs(x[0]) < 1e-12 and info.backtracks > 0
    # a residual that is NaN for every trial point is a line-search failure
    res2 = lambda x, e: np.array([1.0]) if x[0] == 0 else np.array([np.nan])
    x, info = newton_continuation(res2, lambda x, e: sp.csc_matrix([[1.0]]), np.array([0.0]),
                                  1.0, 1.0, 1.0, 1.1, 1e-12, 10, 2 ** -30)
    assert info.status == LINESEARCH_FAIL and x[0] == 0.0


@pytest.mark.parametrize("restart", [60, 7])
def test_gmres_against_direct_solve(restart):
    rng = np.random.default_rng(3)
    n = 60
    M = np.eye(n) * 4 + rng.standard_normal((n, n)) / math.sqrt(n)
    b = rng.standard_normal(n)
    x, used, rel = gmres(lambda v: M @ v, b, restart=restart, rtol=1e-12, maxiter=400)
    assert np.linalg.norm(M @ x - b) <= 2e-12 * np.linalg.norm(b)
    assert abs(np.linalg.norm(M @ x - b) / np.linalg.norm(b) - rel) < 1e-13
    assert np.allclose(x, np.linalg.solve(M, b), rtol=0, atol=1e-10)
    if restart >= n:
        assert used <= n
    x, used, rel = gmres(lambda v: M @ v, b, restart=restart, rtol=1e-30, maxiter=5)
    assert used == 5


# ---------------------------------------------------------------- P8: partition and operators
def test_partition_sizes_of_the_workloads():
    assert split_1d(63, 2) == [(0, 32), (32, 63)]
    subs = partition(63, 63, 2, 2, 2)
    assert sorted({s.box[1] - s.box[0] for s in subs}) == [33, 34]
    subs = partition(255, 255, 8, 8, 4)
    assert sorted({s.box[1] - s.box[0] for s in subs}) == [35, 36, 40]
    subs = partition(511, 511, 16, 16, 4)
    assert max(s.rows.size for s in subs) == 1600          # ~2 x 1600 local unknowns
    with pytest.raises(ValueError):
        split_1d(9, 4)                                       # ceil(9/4) = 3 leaves box 4 empty


@pytest.mark.parametrize("nx,ny,sx,sy,ov", [(15, 15, 2, 2, 1), (23, 17, 3, 2, 2), (20, 9, 4, 1, 3)])
def test_restriction_prolongation_identities(nx, ny, sx, sy, ov):
    n = nx * ny
    subs = partition(nx, ny, sx, sy, ov)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(2 * n)
    total = np.zeros(2 * n)
    cover = np.zeros(n, dtype=int)
    for s in subs:
        c = rng.standard_normal(2 * s.rows.size)
        assert np.array_equal(restrict(s, prolong(s, c, n), n), c)      # R_i P_i = I
        total += prolong_core(s, restrict(s, v, n), n)
        cover[s.core_rows] += 1
        bx0, bx1, by0, by1 = s.box
        assert s.rows.size == (bx1 - bx0) * (by1 - by0)
    assert np.array_equal(total, v)                                       # sum P~_i R_i = I
    assert np.all(cover == 1)                                             # disjoint cores


# ---------------------------------------------------------------- P5, P11: linear-quadratic case
def test_linear_quadratic_case():
    prob = synth.Problem(nx=21, ny=17, phi=synth.PHI_ZERO, nu=1e-3, mu=0.0, eps0=1e-6,
                         eps_min=1e-6, sx=2, sy=2, overlap=2, seed=7)
    yd, f = prob.inputs()
    f = f + 0.3
    xs = lq_direct(prob.nx, prob.ny, prob.nu, yd, f)
    opts = synth.Options(tol_outer=1e-13, tol_inner=1e-13, gmres_rtol=1e-14, max_gmres=500)
    x, info, _ = global_newton(prob, opts, yd, f)
    assert info.iterations == 1
    assert np.max(np.abs(x - xs)) <= 1e-12 * np.max(np.abs(xs))
    out = Raspen(prob, opts, yd, f).solve()
    assert out["outer"] == 1                              # affine F: one outer step (P11)
    assert np.max(np.abs(out["x"] - xs)) <= 1e-11 * np.max(np.abs(xs))
    assert np.max(np.abs(out["u"] + out["p"] / prob.nu)) <= 1e-12 * np.max(np.abs(out["u"]))


# ---------------------------------------------------------------- P4 (solvers), P6: RASPEN = global
@pytest.mark.parametrize("kind", [synth.PHI_CUBIC, synth.PHI_EXP])
def test_solvers_recover_manufactured_solution(kind):
    prob, yd, f, xs = mms_problem(kind, 19, 15, 2, 2, 2)
    opts = synth.Options(tol_outer=1e-12, tol_inner=1e-12, gmres_rtol=1e-13)
    x, info, _ = global_newton(prob, opts, yd, f)
    assert info.status == CONVERGED
    assert np.max(np.abs(x - xs)) <= 1e-11 * np.max(np.abs(xs))
    out = Raspen(prob, opts, yd, f).solve()
    assert out["status"] == CONVERGED
    assert np.max(np.abs(out["x"] - xs)) <= 1e-11 * np.max(np.abs(xs))


@pytest.mark.parametrize("nx,ny,sx,sy,ov,kind", [(15, 15, 2, 2, 1, synth.PHI_CUBIC),
                                                 (31, 31, 3, 3, 2, synth.PHI_CUBIC),
                                                 (23, 17, 3, 2, 2, synth.PHI_EXP)])
def test_raspen_equals_global_newton(nx, ny, sx, sy, ov, kind):
    prob = synth.Problem(nx=nx, ny=ny, phi=kind, nu=1e-2, mu=1e-2, eps0=1.0, eps_min=1e-6,
                         gamma=0.5, sx=sx, sy=sy, overlap=ov, seed=11)
    yd, f = prob.inputs()
    opts = synth.Options(tol_outer=1e-13, tol_inner=1e-13, gmres_rtol=1e-13)
    xg, info, s = global_newton(prob, opts, yd, f)
    assert info.status == CONVERGED
    out = Raspen(prob, opts, yd, f).solve()
    assert out["status"] == CONVERGED
    assert np.max(np.abs(out["x"] - xg)) <= 1e-11 * np.max(np.abs(xg))
    # the zero of the RASPEN residual is a zero of F_eps (Section 4.2)
    assert np.linalg.norm(s.residual(out["x"], prob.eps_min)) < 1e-9


# ---------------------------------------------------------------- P7, P12: RASPEN Jacobian
def test_raspen_jacobian_central_difference_and_halo_form():
    prob = synth.Problem(nx=17, ny=13, phi=synth.PHI_CUBIC, nu=1e-2, mu=1e-2, eps0=1e-4,
                         eps_min=1e-4, sx=2, sy=2, overlap=2, seed=5)
    yd, f = prob.inputs()
    opts = synth.Options(tol_inner=1e-14, max_inner=60)
    R = Raspen(prob, opts, yd, f)
    n = R.n
    rng = np.random.default_rng(2)
    x = np.concatenate([0.3 * rng.standard_normal(n), 0.02 * rng.standard_normal(n)])
    d = rng.standard_normal(2 * n)
    F0, _ = R.eval_F(x, continuation=False)
    Jd = R.jac_apply(d)
    # halo form: F'(x) d = -d - sum_i P~_i J_i^{-1} B_i d with B_i d = R_i diag(A, A)(I - P_i R_i) d
    halo = -d.copy()
    for i, sub in enumerate(R.subs):
        dout = d.copy()
        dout[sub.rows] = 0.0
        dout[n + sub.rows] = 0.0
        Bd = np.concatenate([R.A_rows[i] @ dout[:n], R.A_rows[i] @ dout[n:]])
        halo -= prolong_core(sub, R.lu[i].solve(Bd), n)
    assert np.max(np.abs(halo - Jd)) <= 1e-12 * np.max(np.abs(Jd))
    t = 1e-6
    Fp, _ = R.eval_F(x + t * d, continuation=False)
    Fm, _ = R.eval_F(x - t * d, continuation=False)
    fd = (Fp - Fm) / (2 * t)
    assert np.linalg.norm(fd - Jd) < 1e-6 * np.linalg.norm(Jd)


# ---------------------------------------------------------------- P9: eps -> 0 (weak)
def test_smoothing_error_decays_at_least_like_sqrt_eps():
    prob = synth.Problem(nx=15, ny=15, phi=synth.PHI_CUBIC, nu=1e-3, mu=0.05, seed=4)
    yd, f = prob.inputs()
    yd = 20 * yd
    opts = synth.Options(tol_outer=1e-12)
    ref = None
    errs = []
    epss = [1e-2, 1e-3, 1e-4]
    for e in [1e-12] + epss:
        p2 = synth.Problem(**{**prob.__dict__, "eps0": 1.0, "eps_min": e, "gamma": 0.2})
        x, info, _ = global_newton(p2, opts, yd, f)
        assert info.status == CONVERGED
        if ref is None:
            ref = x
        else:
            errs.append(np.linalg.norm(x - ref))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(epss))
    assert errs[0] > 0 and np.all(slopes >= 0.45)


# ---------------------------------------------------------------- Newton_RAS,eps (Section 4.1)
@pytest.mark.parametrize("nx,ny,sx,sy,ov,kind,cont", [(15, 15, 2, 2, 1, synth.PHI_CUBIC, 0),
                                                      (23, 17, 3, 2, 2, synth.PHI_EXP, 0),
                                                      (15, 15, 2, 2, 1, synth.PHI_CUBIC, 1)])
def test_newton_ras_equals_global_newton(nx, ny, sx, sy, ov, kind, cont):
    """RAS only preconditions the Newton systems: at tight GMRES tolerances the iterates
    are those of Algorithm 1 with a sparse direct solve (same steps, backtracks and
    answer)."""
    from oracle.newton_ras import NewtonRas
    prob = synth.Problem(nx=nx, ny=ny, phi=kind, nu=1e-2, mu=1e-2, eps0=1.0, eps_min=1e-6,
                         gamma=0.5, sx=sx, sy=sy, overlap=ov, seed=11)
    yd, f = prob.inputs()
    opts = synth.Options(tol_outer=1e-12, gmres_rtol=1e-13, continuation=cont)
    eps0 = prob.eps_min if cont == 1 else prob.eps0
    xg, info, s = global_newton(prob, synth.Options(tol_outer=1e-12, max_inner=opts.max_outer), yd, f,
                                eps0=eps0)
    out = NewtonRas(prob, opts, yd, f).solve()
    assert info.status == CONVERGED and out["status"] == CONVERGED
    assert out["iterations"] == info.iterations and out["backtracks"] == info.backtracks
    assert np.max(np.abs(out["x"] - xg)) <= 1e-11 * np.max(np.abs(xg))
    assert np.linalg.norm(s.residual(out["x"], prob.eps_min)) <= 1e-10
    assert all(1 <= g for g in out["gmres_its"])


def test_ras_of_one_subdomain_is_the_exact_inverse():
    """One subdomain covering the grid: M^{-1} = F'(x)^{-1}, so every preconditioned
    Newton system is solved by GMRES with a single product."""
    from oracle.newton_ras import NewtonRas
    prob = synth.Problem(nx=12, ny=9, phi=synth.PHI_PAPER, nu=1e-2, mu=1e-2, eps0=1.0, eps_min=1e-6,
                         gamma=0.5, sx=1, sy=1, overlap=2, seed=3)
    yd, f = prob.inputs()
    out = NewtonRas(prob, synth.Options(tol_outer=1e-12), yd, f).solve()
    assert out["status"] == CONVERGED
    assert out["gmres_its"] == [1] * out["iterations"]
    xg, info, _ = global_newton(prob, synth.Options(tol_outer=1e-12, max_inner=50), yd, f)
    assert np.max(np.abs(out["x"] - xg)) <= 1e-12 * np.max(np.abs(xg))


def test_ras_preconditioned_operator_halo_form():
    """M^{-1} F'(x) d = d + sum_i P~_i J_i^{-1} B_i d, J_i = R_i F'(x) P_i and
    B_i d = R_i diag(A, A)(I - P_i R_i) d: the halo form of Algorithm 4 with local
    Jacobians at x (the identity sum_i P~_i R_i = I and the locality of the
    pointwise terms)."""
    from oracle.newton_ras import RasPreconditioner
    prob = synth.Problem(nx=17, ny=13, phi=synth.PHI_CUBIC, nu=1e-2, mu=1e-2, eps0=1e-3, eps_min=1e-3,
                         sx=3, sy=2, overlap=2, seed=5)
    yd, f = prob.inputs()
    s = System(prob, yd, f)
    n = s.n
    rng = np.random.default_rng(4)
    x = np.concatenate([0.3 * rng.standard_normal(n), 0.02 * rng.standard_normal(n)])
    d = rng.standard_normal(2 * n)
    J = s.jacobian(x, 1e-3).tocsr()
    subs = partition(prob.nx, prob.ny, prob.sx, prob.sy, prob.overlap)
    M = RasPreconditioner(J, subs, n)
    lit = M.apply(J @ d)
    halo = d.copy()
    for sub, lu in zip(subs, M.lu):
        dout = d.copy()
        dout[sub.rows] = 0.0
        dout[n + sub.rows] = 0.0
        Ar = s.A[sub.rows, :]
        Bd = np.concatenate([Ar @ dout[:n], Ar @ dout[n:]])
        halo += prolong_core(sub, lu.solve(Bd), n)
    assert np.max(np.abs(halo - lit)) <= 1e-12 * np.max(np.abs(lit))


@pytest.mark.parametrize("cont", [0, 1])
def test_newton_gmres_equals_global_newton(cont):
    """Newton_eps (Section 4.1, GMRES without preconditioner): with GMRES run to a tight
    tolerance the iterates are those of the sparse direct Newton solve."""
    from oracle.newton_ras import NewtonRas
    prob = synth.Problem(nx=15, ny=11, phi=synth.PHI_CUBIC, nu=1e-2, mu=1e-2, eps0=1.0, eps_min=1e-6,
                         gamma=0.5, sx=2, sy=2, overlap=1, seed=12)
    yd, f = prob.inputs()
    opts = synth.Options(tol_outer=1e-11, gmres_rtol=1e-13, max_gmres=5000, continuation=cont)
    eps0 = prob.eps_min if cont == 1 else prob.eps0
    xg, info, s = global_newton(prob, synth.Options(tol_outer=1e-11, max_inner=opts.max_outer), yd, f,
                                eps0=eps0)
    out = NewtonRas(prob, opts, yd, f, precond=False).solve()
    assert info.status == CONVERGED and out["status"] == CONVERGED
    assert out["iterations"] == info.iterations and out["backtracks"] == info.backtracks
    assert np.max(np.abs(out["x"] - xg)) <= 1e-10 * np.max(np.abs(xg))
    # the unpreconditioned systems take far more products than the RAS ones
    ras = NewtonRas(prob, opts, yd, f).solve()
    assert np.mean(out["gmres_its"]) > 3 * np.mean(ras["gmres_its"])


def test_model_problem_local_rounding_floor():
    """The model problem of Section 4 at N = 450 (|y_bar| ~ 56, nu = 1e-6): the FP64
    rounding of one evaluation of F on a 45 x 45 box (the size of a subdomain of the
    11 x 11 partition with overlap 2h) exceeds an unscaled inner tolerance of 1e-8, and
    lies far below it once the equations are scaled by the cell area.  The reference
    evaluation is the same 5-point residual in extended precision; the constructed pair
    solves F = 0 at eps = 1e-15 to well within the unscaled floor on every box row."""
    from cases import paper_inner_tol, paper_model_problem
    n = 450
    prob, yd, f, xbar = paper_model_problem(n, 11, 11, 2, 1e-15)
    s = System(prob, yd, f)
    r64 = s.residual(xbar, 1e-15)
    y = xbar[:s.n].reshape(n, n).astype(np.longdouble)
    p = xbar[s.n:].reshape(n, n).astype(np.longdouble)
    h2 = np.longdouble(1.0) / np.longdouble((n + 1) ** 2)

    def lap(v):
        z = np.zeros((n + 2, n + 2), dtype=np.longdouble)
        z[1:-1, 1:-1] = v
        return (4 * z[1:-1, 1:-1] - z[:-2, 1:-1] - z[2:, 1:-1] - z[1:-1, :-2] - z[1:-1, 2:]) / h2

    k = np.longdouble(prob.kappa)
    g = pw.g(xbar[s.n:], prob.mu, 1e-15).reshape(n, n).astype(np.longdouble)
    r1 = lap(y) + k * (y ** 3 + np.exp(k * y)) + g / np.longdouble(prob.nu)
    r2 = lap(p) + k * (3 * y ** 2 + k * np.exp(k * y)) * p - y + yd.astype(np.longdouble)
    box = (slice(200, 245), slice(200, 245))
    err = np.hypot(np.linalg.norm((r64[:s.n].reshape(n, n) - r1)[box].astype(np.float64)),
                   np.linalg.norm((r64[s.n:].reshape(n, n) - r2)[box].astype(np.float64)))
    exact = np.hypot(np.linalg.norm(r1[box].astype(np.float64)), np.linalg.norm(r2[box].astype(np.float64)))
    assert err > 1e-8                       # unscaled: the tolerance is below the floor
    assert exact < 10 * err                 # x_bar is a solution to rounding level
    tol = paper_inner_tol(n, n)
    assert tol == pytest.approx(1e-8 * 451 ** 2)
    assert err < 1e-3 * tol                 # scaled: six orders of magnitude of room


# ---------------------------------------------------------------- second level (coarse correction)
def coarse_closed_form(prob, subs, dphi_sum, dg_sum, cpl_sum):
    """A_0 = Z^T F' Z written out: for the indicator of a core of cw x ch nodes, the
    5-point -Laplacian sums to h^-2 times the grid edges leaving the core (2 ch hx^-2 +
    2 cw hy^-2 on the core itself, -(shared edges) h^-2 with the four neighbouring
    cores, 0 otherwise); the pointwise blocks of F' sum over the core."""
    hx2, hy2 = (prob.nx + 1) ** 2, (prob.ny + 1) ** 2
    S = len(subs)
    A0 = np.zeros((2 * S, 2 * S))
    for i, a in enumerate(subs):
        ax0, ax1, ay0, ay1 = a.core
        for j, b in enumerate(subs):
            bx0, bx1, by0, by1 = b.core
            if i == j:
                lap = 2 * (ay1 - ay0) * hx2 + 2 * (ax1 - ax0) * hy2
            elif ay0 == by0 and (ax1 == bx0 or bx1 == ax0):
                lap = -(ay1 - ay0) * hx2
            elif ax0 == bx0 and (ay1 == by0 or by1 == ay0):
                lap = -(ax1 - ax0) * hy2
            else:
                continue
            for fld in range(2):
                A0[2 * i + fld, 2 * j + fld] = lap
        A0[2 * i, 2 * i] += dphi_sum[i]
        A0[2 * i + 1, 2 * i + 1] += dphi_sum[i]
        A0[2 * i, 2 * i + 1] = dg_sum[i]
        A0[2 * i + 1, 2 * i] = cpl_sum[i]
    return A0


@pytest.mark.parametrize("nx,ny,sx,sy,ov,kind", [(23, 17, 3, 2, 2, synth.PHI_EXP), (31, 29, 4, 3, 1, synth.PHI_CUBIC)])
def test_coarse_operator_closed_form(nx, ny, sx, sy, ov, kind):
    prob = synth.Problem(nx=nx, ny=ny, phi=kind, nu=1e-3, mu=5e-3, eps_min=1e-4, sx=sx, sy=sy, overlap=ov, seed=3)
    yd, f = prob.inputs()
    ora = Raspen(prob, synth.Options(), yd, f)
    rng = np.random.default_rng(4)
    n = ora.n
    x = np.concatenate([0.4 * rng.standard_normal(n), 0.01 * rng.standard_normal(n)])
    y, p = x[:n], x[n:]
    sums = [[], [], []]
    for s in ora.subs:
        r = s.core_rows
        sums[0].append(pw.dphi(y[r], kind, prob.kappa).sum())
        sums[1].append((pw.dg(p[r], prob.mu, prob.eps_min) / prob.nu).sum())
        sums[2].append((pw.ddphi(y[r], kind, prob.kappa) * p[r] - 1.0).sum())
    want = coarse_closed_form(prob, ora.subs, *sums)
    got = ora.coarse_operator(x)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_coarse_correction_galerkin_property():
    """Q = Z (Z^T F' Z)^{-1} Z^T makes the coarse residual of every correction vanish:
    Z^T F'(x)(v - Q F'(x) v) = 0."""
    prob = synth.Problem(nx=31, ny=29, phi=synth.PHI_EXP, nu=1e-3, mu=5e-3, eps_min=1e-6, sx=4, sy=3, overlap=2)
    yd, f = prob.inputs()
    ora = Raspen(prob, synth.Options(), yd, f)
    rng = np.random.default_rng(5)
    x = np.concatenate([0.3 * rng.standard_normal(ora.n), 0.01 * rng.standard_normal(ora.n)])
    Z = ora.coarse_basis()
    J = ora.sys.jacobian(x, prob.eps_min)
    A0 = ora.coarse_operator(x, Z)
    v = rng.standard_normal(2 * ora.n)
    w = v - Z @ np.linalg.solve(A0, Z.T @ (J @ v))
    r = Z.T @ (J @ w)
    assert np.abs(r).max() <= 1e-10 * np.abs(Z.T @ (J @ v)).max()


def test_two_level_operator_is_minus_identity_on_the_coarse_space():
    """Affine F (phi = 0, mu = 0): the RASPEN Jacobian is -M^{-1} F' exactly, so the
    two-level operator d -> F_RAS'(d - Q F' d) - Q F' d is minus the hybrid preconditioned
    operator P2 F', which maps every coarse vector Z c to itself."""
    prob = synth.Problem(nx=25, ny=21, phi=synth.PHI_ZERO, nu=1e-2, mu=0.0, eps0=1e-6, eps_min=1e-6,
                         sx=3, sy=2, overlap=2, seed=8)
    yd, f = prob.inputs()
    opts = synth.Options(tol_outer=1e-13, tol_inner=1e-13, gmres_rtol=1e-13)
    ora = Raspen(prob, opts, yd, f)
    x = np.zeros(2 * ora.n)
    ora.eval_F(x, continuation=False)
    Z = ora.coarse_basis()
    J = ora.sys.jacobian(x, prob.eps_min)
    A0 = ora.coarse_operator(x, Z)
    zc = Z @ np.random.default_rng(6).standard_normal(Z.shape[1])
    qv = Z @ np.linalg.solve(A0, Z.T @ (J @ zc))
    out = ora.jac_apply(zc - qv) - qv
    assert np.abs(out + zc).max() <= 1e-10 * np.abs(zc).max()


def test_two_level_raspen_linear_quadratic_case():
    prob = synth.Problem(nx=21, ny=17, phi=synth.PHI_ZERO, nu=1e-3, mu=0.0, eps0=1e-6,
                         eps_min=1e-6, sx=3, sy=2, overlap=2, seed=7)
    yd, f = prob.inputs()
    f = f + 0.3
    xs = lq_direct(prob.nx, prob.ny, prob.nu, yd, f)
    opts = synth.Options(tol_outer=1e-13, tol_inner=1e-13, gmres_rtol=1e-14, max_gmres=500)
    out = Raspen(prob, opts, yd, f).solve(coarse=True)
    assert out["outer"] == 1
    assert np.max(np.abs(out["x"] - xs)) <= 1e-11 * np.max(np.abs(xs))


@pytest.mark.parametrize("nx,ny,sx,sy,ov,kind", [(31, 31, 3, 3, 2, synth.PHI_CUBIC),
                                                 (23, 17, 3, 2, 2, synth.PHI_EXP)])
def test_two_level_raspen_equals_global_newton(nx, ny, sx, sy, ov, kind):
    prob = synth.Problem(nx=nx, ny=ny, phi=kind, nu=1e-2, mu=1e-2, eps0=1.0, eps_min=1e-6,
                         gamma=0.5, sx=sx, sy=sy, overlap=ov, seed=11)
    yd, f = prob.inputs()
    opts = synth.Options(tol_outer=1e-13, tol_inner=1e-13, gmres_rtol=1e-13)
    xg, info, s = global_newton(prob, opts, yd, f)
    out = Raspen(prob, opts, yd, f).solve(coarse=True)
    assert out["status"] == CONVERGED
    assert np.max(np.abs(out["x"] - xg)) <= 1e-11 * np.max(np.abs(xg))


def test_two_level_takes_fewer_gmres_products():
    """The purpose of the second level (end of Section 5.3): GMRES products per outer
    step no longer grow as much with the number of subdomains."""
    prob = synth.Problem(nx=63, ny=63, phi=synth.PHI_EXP, nu=1e-3, mu=5e-3, eps_min=1e-6, sx=4, sy=4,
                         overlap=3, seed=2)
    opts = synth.Options(tol_outer=1e-12, tol_inner=1e-11, gmres_rtol=1e-12)
    yd, f = prob.inputs()
    one = Raspen(prob, opts, yd, f).solve()
    two = Raspen(prob, opts, yd, f).solve(coarse=True)
    assert two["outer"] == one["outer"]
    assert sum(h["gmres"] for h in two["history"]) < 0.8 * sum(h["gmres"] for h in one["history"])
    assert np.max(np.abs(two["x"] - one["x"])) <= 1e-11 * np.max(np.abs(one["x"]))


# ---------------------------------------------------------------- variable coefficients of A
# Assumption 1 (3): A = -div(a grad) + a0 with a diagonal coefficient tensor (a1, a2) and
# a0 >= 0, in the 5-point flux form with face coefficients (oracle/system.py).
from oracle.system import variable_operator  # noqa: E402


def test_variable_operator_with_unit_coefficients_is_the_laplacian():
    for nx, ny in [(7, 5), (1, 4), (12, 9)]:
        A = variable_operator(nx, ny, np.ones((ny, nx + 1)), np.ones((ny + 1, nx)), np.zeros((ny, nx)))
        assert abs(A - laplacian(nx, ny)).max() == 0


@pytest.mark.parametrize("a1,a2,a0", [(2.5, 0.3, 0.0), (0.7, 4.0, 3.0)])
def test_variable_operator_constant_coefficients_eigenpairs(a1, a2, a0):
    """Constant coefficients: the sine vectors are eigenvectors with eigenvalue
    a1 (4/hx^2) sin^2(k pi hx/2) + a2 (4/hy^2) sin^2(l pi hy/2) + a0."""
    nx, ny = 9, 6
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    A = variable_operator(nx, ny, np.full((ny, nx + 1), a1), np.full((ny + 1, nx), a2), np.full((ny, nx), a0))
    X, Y = synth.node_coords(nx, ny)
    for k, l in [(1, 1), (3, 2), (9, 6), (5, 1)]:
        v = (np.sin(k * math.pi * X) * np.sin(l * math.pi * Y)).reshape(-1)
        lam = (a1 * 4 / hx ** 2 * math.sin(k * math.pi * hx / 2) ** 2
               + a2 * 4 / hy ** 2 * math.sin(l * math.pi * hy / 2) ** 2 + a0)
        assert np.max(np.abs(A @ v - lam * v)) < 1e-9 * lam


def test_variable_operator_energy_identity_and_symmetry():
    """y^T A y is the sum over all faces (boundary faces included, y = 0 outside) of
    a_f (jump of y)^2 / h^2 plus the sum of a0 y^2; A is symmetric."""
    nx, ny = 8, 6
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    ax, ay, a0 = synth.coefficient_fields(nx, ny, 4)
    A = variable_operator(nx, ny, ax, ay, a0)
    assert abs(A - A.T).max() == 0
    rng = np.random.default_rng(9)
    for _ in range(3):
        y = rng.standard_normal((ny, nx))
        yb = np.zeros((ny + 2, nx + 2))
        yb[1:-1, 1:-1] = y
        e = 0.0
        for j in range(ny):
            for i in range(nx + 1):            # x-face between nodes i-1 and i
                e += ax[j, i] * (yb[j + 1, i + 1] - yb[j + 1, i]) ** 2 / hx ** 2
        for j in range(ny + 1):
            for i in range(nx):                # y-face between rows j-1 and j
                e += ay[j, i] * (yb[j + 1, i + 1] - yb[j, i + 1]) ** 2 / hy ** 2
        e += float(np.sum(a0 * y * y))
        v = y.reshape(-1)
        assert abs(v @ (A @ v) - e) <= 1e-12 * e


def test_variable_operator_is_second_order_consistent():
    """With the face coefficients taken at the face midpoints, A applied to the nodal
    values of a smooth u converges to -d/dx(a1 u_x) - d/dy(a2 u_y) + a0 u (written out
    by hand below) at second order."""
    a1 = lambda x, y: 1.0 + x * x * y
    a1x = lambda x, y: 2.0 * x * y
    a2 = lambda x, y: 2.0 + np.sin(x)
    a2y = lambda x, y: 0.0 * x
    a0 = lambda x, y: 1.0 + x * y
    u = lambda x, y: np.sin(np.pi * x) * np.sin(2 * np.pi * y)
    ux = lambda x, y: np.pi * np.cos(np.pi * x) * np.sin(2 * np.pi * y)
    uy = lambda x, y: 2 * np.pi * np.sin(np.pi * x) * np.cos(2 * np.pi * y)
    uxx = lambda x, y: -np.pi ** 2 * u(x, y)
    uyy = lambda x, y: -4 * np.pi ** 2 * u(x, y)
    Lu = lambda x, y: -(a1x(x, y) * ux(x, y) + a1(x, y) * uxx(x, y)) - (a2y(x, y) * uy(x, y) + a2(x, y) * uyy(x, y)) \
        + a0(x, y) * u(x, y)
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / (n + 1)
        xf, yf = np.meshgrid((np.arange(n + 1) + 0.5) * h, (np.arange(n) + 1.0) * h, indexing="xy")
        xg, yg = np.meshgrid((np.arange(n) + 1.0) * h, (np.arange(n + 1) + 0.5) * h, indexing="xy")
        X, Y = synth.node_coords(n, n)
        A = variable_operator(n, n, a1(xf, yf), a2(xg, yg), a0(X, Y))
        errs.append(np.max(np.abs(A @ u(X, Y).reshape(-1) - Lu(X, Y).reshape(-1))))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_variable_coefficient_jacobian_central_difference():
    prob = synth.Problem(nx=9, ny=7, phi=synth.PHI_EXP, nu=1e-2, mu=0.02, coef=1, seed=3)
    rng = np.random.default_rng(1)
    s = System(prob, rng.standard_normal((7, 9)), rng.standard_normal((7, 9)))
    x = np.concatenate([0.5 * rng.standard_normal(s.n), 0.05 * rng.standard_normal(s.n)])
    d = rng.standard_normal(2 * s.n)
    t = 1e-6
    fd = (s.residual(x + t * d, 1e-3) - s.residual(x - t * d, 1e-3)) / (2 * t)
    Jd = s.jacobian(x, 1e-3) @ d
    assert np.linalg.norm(fd - Jd) < 1e-6 * np.linalg.norm(Jd)


@pytest.mark.parametrize("coarse", [False, True])
def test_variable_coefficient_raspen_equals_global_newton(coarse):
    prob = synth.Problem(nx=23, ny=17, phi=synth.PHI_EXP, nu=1e-2, mu=1e-2, eps0=1.0, eps_min=1e-6,
                         gamma=0.5, sx=3, sy=2, overlap=2, seed=11, coef=1)
    yd, f = prob.inputs()
    opts = synth.Options(tol_outer=1e-13, tol_inner=1e-13, gmres_rtol=1e-13)
    xg, info, s = global_newton(prob, opts, yd, f)
    assert info.status == CONVERGED
    out = Raspen(prob, opts, yd, f).solve(coarse=coarse)
    assert out["status"] == CONVERGED
    assert np.max(np.abs(out["x"] - xg)) <= 1e-11 * np.max(np.abs(xg))
    # a different operator: the solution moves away from the Laplacian one
    base = synth.Problem(**{**prob.__dict__, "coef": 0})
    xl, _, _ = global_newton(base, opts, yd, f)
    assert np.max(np.abs(xl - xg)) > 1e-3 * np.max(np.abs(xg))


def coarse_closed_form_variable(prob, subs, dphi_sum, dg_sum, cpl_sum):
    """Z^T F' Z for the variable-coefficient operator written out over faces: core I and
    a different core J are coupled by minus the sum of a_f / h^2 over the faces between
    them; the diagonal holds the sum of a_f / h^2 over every face with exactly one node
    in the core (domain boundary faces included) plus the sum of a0 over the core."""
    nx, ny = prob.nx, prob.ny
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    ax, ay, a0 = prob.coefficients()
    owner = -np.ones((ny, nx), dtype=int)
    for i, s in enumerate(subs):
        c = s.core_rows
        owner.reshape(-1)[c] = i
    S = len(subs)
    L = np.zeros((S, S))
    for j in range(ny):
        for i in range(nx + 1):
            l = owner[j, i - 1] if i > 0 else -1
            r = owner[j, i] if i < nx else -1
            w = ax[j, i] / hx ** 2
            if l != r:
                if l >= 0:
                    L[l, l] += w
                if r >= 0:
                    L[r, r] += w
                if l >= 0 and r >= 0:
                    L[l, r] -= w
                    L[r, l] -= w
    for j in range(ny + 1):
        for i in range(nx):
            d = owner[j - 1, i] if j > 0 else -1
            u = owner[j, i] if j < ny else -1
            w = ay[j, i] / hy ** 2
            if d != u:
                if d >= 0:
                    L[d, d] += w
                if u >= 0:
                    L[u, u] += w
                if d >= 0 and u >= 0:
                    L[d, u] -= w
                    L[u, d] -= w
    for i, s in enumerate(subs):
        L[i, i] += a0.reshape(-1)[s.core_rows].sum()
    A0 = np.zeros((2 * S, 2 * S))
    for fld in range(2):
        A0[fld::2, fld::2] = L
    for i in range(S):
        A0[2 * i, 2 * i] += dphi_sum[i]
        A0[2 * i + 1, 2 * i + 1] += dphi_sum[i]
        A0[2 * i, 2 * i + 1] = dg_sum[i]
        A0[2 * i + 1, 2 * i] = cpl_sum[i]
    return A0


def test_coarse_operator_closed_form_variable_coefficients():
    prob = synth.Problem(nx=23, ny=17, phi=synth.PHI_EXP, nu=1e-3, mu=5e-3, eps_min=1e-4, sx=3, sy=2, overlap=2,
                         seed=3, coef=1)
    yd, f = prob.inputs()
    ora = Raspen(prob, synth.Options(), yd, f)
    rng = np.random.default_rng(4)
    n = ora.n
    x = np.concatenate([0.4 * rng.standard_normal(n), 0.01 * rng.standard_normal(n)])
    y, p = x[:n], x[n:]
    sums = [[], [], []]
    for s in ora.subs:
        r = s.core_rows
        sums[0].append(pw.dphi(y[r], prob.phi, prob.kappa).sum())
        sums[1].append((pw.dg(p[r], prob.mu, prob.eps_min) / prob.nu).sum())
        sums[2].append((pw.ddphi(y[r], prob.phi, prob.kappa) * p[r] - 1.0).sum())
    want = coarse_closed_form_variable(prob, ora.subs, *sums)
    got = ora.coarse_operator(x)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
