"""The second level (rsp_options.coarse = 1) on the GPU against the oracle's two-level
RASPEN (oracle/schwarz.py: hybrid coarse correction, one coarse unknown per subdomain
core and field).

* The two-level operator (rsp_coarse_jac_apply) equals the oracle's within 1e-10, and is
  minus the identity on the coarse space for an affine F.
* Whole two-level solves land within 1e-10 of the oracle's with its outer steps, and take
  about its GMRES products; on the 511 x 511 workload they reach the one-level fixed
  point (the stored oracle answer) with far fewer products.
* Batches, the server and captured graphs give the same bits as single direct solves.
"""
import os

import numpy as np
import pytest

import synth
from oracle.schwarz import Raspen

from gpu_helpers import dev, host, lib, rel, solve

pytestmark = pytest.mark.gpu

TIGHT = synth.Options(tol_outer=1e-12, tol_inner=1e-11, gmres_rtol=1e-12, coarse=1)


@pytest.fixture(scope="module")
def R():
    return lib()


def with_(o, **kw):
    import copy
    o = copy.copy(o)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def problem(nx=37, ny=29, sx=3, sy=4, overlap=3, phi=synth.PHI_CUBIC, nu=1e-2, mu=1e-2, seed=1, eps_min=1e-6):
    return synth.Problem(nx=nx, ny=ny, phi=phi, nu=nu, mu=mu, eps0=1.0, eps_min=eps_min, gamma=0.5,
                         sx=sx, sy=sy, overlap=overlap, seed=seed)


def coarse_vector(ora, c):
    """Z c: the coarse value of (core i, field f) on every node of that core and field."""
    n = ora.n
    v = np.zeros(2 * n)
    for i, sub in enumerate(ora.subs):
        v[sub.core_rows] = c[2 * i]
        v[n + sub.core_rows] = c[2 * i + 1]
    return v


def gpu_operator(R, prob, opts, yd, f, x, d):
    ctx = R.rsp_context_create(0)
    try:
        R.rsp_setup(ctx, R.make_problem(prob), R.make_options(opts), dev(yd), dev(f))
        n = prob.nx * prob.ny
        out = dev(np.zeros(2 * n))
        R.rsp_eval(ctx, dev(x), 1, out)
        res = dev(np.zeros(2 * n))
        R.rsp_coarse_jac_apply(ctx, dev(x), dev(d), res)
        return host(res)
    finally:
        R.rsp_context_destroy(ctx)


def test_operator_is_minus_identity_on_the_coarse_space(R):
    prob = problem(nx=25, ny=21, sx=3, sy=2, overlap=2, phi=synth.PHI_ZERO, mu=0.0, seed=8)
    prob.eps0 = prob.eps_min
    yd, f = prob.inputs()
    ora = Raspen(prob, TIGHT, yd, f)
    zc = coarse_vector(ora, np.random.default_rng(6).standard_normal(2 * len(ora.subs)))
    out = gpu_operator(R, prob, TIGHT, yd, f, np.zeros(2 * ora.n), zc)
    assert np.abs(out + zc).max() <= 1e-10 * np.abs(zc).max()


@pytest.mark.parametrize("phi,nu,mu,precision", [(synth.PHI_CUBIC, 1e-2, 1e-2, 0), (synth.PHI_EXP, 1e-3, 5e-3, 0),
                                                 (synth.PHI_EXP, 1e-3, 5e-3, 1)])
def test_operator_matches_the_oracle(R, phi, nu, mu, precision):
    prob = problem(phi=phi, nu=nu, mu=mu)
    yd, f = prob.inputs()
    opts = with_(TIGHT, precision=precision, max_refine=0)
    rng = np.random.default_rng(13)
    n = prob.nx * prob.ny
    x = np.concatenate([0.05 * rng.standard_normal(n), 0.005 * rng.standard_normal(n)])
    d = rng.standard_normal(2 * n)
    ora = Raspen(prob, TIGHT, yd, f)
    ora.eval_F(x, continuation=True)
    Z = ora.coarse_basis()
    J = ora.sys.jacobian(x, prob.eps_min)
    A0 = ora.coarse_operator(x, Z)
    qv = Z @ np.linalg.solve(A0, Z.T @ (J @ d))
    want = ora.jac_apply(d - qv) - qv
    got = gpu_operator(R, prob, opts, yd, f, x, d)
    # FP32 line inverses: the error of an FP32 block LU (as for the one-level action)
    assert rel(got, want) <= (1e-10 if precision == 0 else 1e-5)


@pytest.mark.parametrize("name,phi,mu", [("ragged", synth.PHI_CUBIC, 1e-2), ("rect", synth.PHI_EXP, 1e-2),
                                         ("square", synth.PHI_CUBIC, 0.0)])
def test_two_level_solves_match_the_oracle(R, name, phi, mu):
    kw = {"ragged": {}, "rect": dict(nx=23, ny=17, sx=3, sy=2, overlap=2),
          "square": dict(nx=63, ny=63, sx=4, sy=4, overlap=3)}[name]
    prob = problem(phi=phi, mu=mu, nu=1e-3 if name == "square" else 1e-2, **kw)
    yd, f = prob.inputs()
    st, h, x, u = solve(R, prob, TIGHT, yd, f)
    ref = Raspen(prob, TIGHT, yd, f).solve()
    assert ref["status"] == 0 and st == 0
    assert h["outer"] == ref["outer"]
    assert rel(x, ref["x"]) <= 1e-10
    want = sum(e["gmres"] for e in ref["history"])
    print("%s: GMRES products %d (oracle %d)" % (name, sum(h["gmres_its"]), want))
    assert sum(h["gmres_its"]) <= 1.1 * want + 2
    # the same fixed point as the one-level method
    one = Raspen(prob, with_(TIGHT, coarse=0), yd, f).solve()
    assert rel(x, one["x"]) <= 1e-10


def test_two_level_on_the_precision_workload(R):
    """511 x 511, 16 x 16 subdomains: the fixed point of the one-level method (the
    oracle's stored answer at parity tolerances) within 1e-10 in FP64 and 1e-8 with
    FP32 line factors, with at most half the GMRES products of one level."""
    import importlib.util
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("refs", os.path.join(here, "golden", "make_oracle_refs.py"))
    refs = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(refs)
    ref = refs.load("precision_parity")
    prob = synth.config_precision()
    yd, f = prob.inputs()
    o = with_(refs.options_of("precision_parity"), coarse=1)
    st, h, x, u = solve(R, prob, o, yd, f)
    e64 = rel(x, ref["x"])
    st_m, h_m, x_m, u_m = solve(R, prob, with_(o, precision=1, max_refine=0), yd, f)
    em = rel(x_m, ref["x"])
    print("two-level 511^2: FP64 outer %d GMRES %s error %.3e; mixed outer %d GMRES %s error %.3e; one level "
          "(oracle) GMRES %s" % (h["outer"], h["gmres_its"], e64, h_m["outer"], h_m["gmres_its"], em,
                                 list(ref["gmres"][1:])))
    assert st == 0 and st_m == 0
    assert e64 <= 1e-10 and em <= 1e-8
    assert sum(h["gmres_its"]) <= 0.5 * int(np.sum(ref["gmres"]))


def test_two_level_batch_server_and_graphs_equal_single_solves(R):
    import torch
    probs = [problem(phi=synth.PHI_EXP, nu=1e-3, mu=5e-3, seed=s) for s in (1, 2, 3)]
    ins = [p.inputs() for p in probs]
    singles = [solve(R, p, TIGHT, *ins[q])[2] for q, p in enumerate(probs)]
    inp = [(dev(a), dev(b)) for a, b in ins]
    # batch
    ys, ps, us = ([dev(np.zeros((p.ny, p.nx))) for p in probs] for _ in range(3))
    ctx = R.rsp_context_create(0)
    try:
        st, hs = R.rsp_solve_batch(ctx, [R.make_problem(p) for p in probs], R.make_options(TIGHT),
                                   [a for a, _ in inp], [b for _, b in inp], None, None, ys, ps, us)
        torch.cuda.synchronize()
        assert st == 0
        for q in range(3):
            x = np.concatenate([host(ys[q]).reshape(-1), host(ps[q]).reshape(-1)])
            assert np.array_equal(x, singles[q]), q
        # captured graphs, replayed twice
        R.rsp_set_tuning(ctx, graphs=1, gm_chunk=8)
        for rep in range(2):
            y, p, u = (dev(np.zeros((probs[0].ny, probs[0].nx))) for _ in range(3))
            st, h = R.rsp_solve(ctx, R.make_problem(probs[0]), R.make_options(TIGHT), inp[0][0], inp[0][1], None,
                                None, y, p, u)
            torch.cuda.synchronize()
            x = np.concatenate([host(y).reshape(-1), host(p).reshape(-1)])
            assert st == 0 and np.array_equal(x, singles[0]), rep
    finally:
        R.rsp_context_destroy(ctx)
    # server
    outs = [[dev(np.zeros((p.ny, p.nx))) for _ in range(3)] for p in probs]
    srv = R.rsp_server_create(R.make_options(TIGHT))
    try:
        tickets = [R.rsp_server_submit(srv, R.make_problem(p), inp[q][0], inp[q][1], *outs[q])
                   for q, p in enumerate(probs)]
        res = [R.rsp_server_wait(srv, t, 60000.0) for t in tickets]
    finally:
        R.rsp_server_destroy(srv)
    for q, (st, h) in enumerate(res):
        x = np.concatenate([host(outs[q][0]).reshape(-1), host(outs[q][1]).reshape(-1)])
        assert st == 0 and np.array_equal(x, singles[q]), q


def test_second_level_is_rejected_by_the_monolithic_methods(R):
    prob = problem()
    yd, f = prob.inputs()
    with pytest.raises(R.RaspenError) as e:
        solve(R, prob, TIGHT, yd, f, method="newton_ras")
    assert e.value.code == R.RSP_EINVAL


@pytest.mark.parametrize("nx,sx", [(80, 20), (64, 16), (50, 13)])
def test_operator_matches_the_oracle_on_wide_rows_of_cores(R, nx, sx):
    """Rows of 2 sx coarse unknowns: 40 take the LDS form of the coarse block
    Gauss-Jordan, 32 and 26 the one-wave register form (26 with identity padding)."""
    prob = problem(nx=nx, ny=17, sx=sx, sy=2, overlap=2, phi=synth.PHI_EXP, nu=1e-3, mu=5e-3)
    yd, f = prob.inputs()
    rng = np.random.default_rng(21)
    n = prob.nx * prob.ny
    x = np.concatenate([0.05 * rng.standard_normal(n), 0.005 * rng.standard_normal(n)])
    d = rng.standard_normal(2 * n)
    ora = Raspen(prob, TIGHT, yd, f)
    ora.eval_F(x, continuation=True)
    Z = ora.coarse_basis()
    J = ora.sys.jacobian(x, prob.eps_min)
    A0 = ora.coarse_operator(x, Z)
    qv = Z @ np.linalg.solve(A0, Z.T @ (J @ d))
    want = ora.jac_apply(d - qv) - qv
    got = gpu_operator(R, prob, TIGHT, yd, f, x, d)
    assert rel(got, want) <= 1e-10


@pytest.mark.parametrize("nx,sx", [(50, 5), (80, 20)])
def test_operator_matches_the_oracle_when_rows_of_cores_need_pivoting(R, nx, sx):
    """nu = 1e-4: the sums of g'(p) / nu make the Schur complements of the rows of cores
    lose column dominance in the control field (checked with the oracle's A0), so the
    coarse factor takes its partial-pivoting form (rows of 10 and 40 unknowns)."""
    prob = problem(nx=nx, ny=34, sx=sx, sy=4, overlap=2, phi=synth.PHI_EXP, nu=1e-4, mu=5e-3, seed=3)
    yd, f = prob.inputs()
    rng = np.random.default_rng(1)
    n = prob.nx * prob.ny
    x = np.concatenate([0.1 * rng.standard_normal(n), rng.standard_normal(n)])
    d = rng.standard_normal(2 * n)
    ora = Raspen(prob, TIGHT, yd, f)
    ora.eval_F(x, continuation=True)
    Z = ora.coarse_basis()
    J = ora.sys.jacobian(x, prob.eps_min)
    A0 = ora.coarse_operator(x, Z)
    # the first row of cores is not column diagonally dominant
    nc = 2 * sx
    T0 = A0[:nc, :nc]
    assert (np.abs(np.diag(T0)) <= np.abs(T0).sum(0) - np.abs(np.diag(T0))).any()
    qv = Z @ np.linalg.solve(A0, Z.T @ (J @ d))
    want = ora.jac_apply(d - qv) - qv
    got = gpu_operator(R, prob, TIGHT, yd, f, x, d)
    assert rel(got, want) <= 1e-10
