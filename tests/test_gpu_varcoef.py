"""Variable coefficients of A on the GPU against the oracle (Assumption 1 (3) with a
diagonal coefficient tensor: A y = -d/dx(a1 dy/dx) - d/dy(a2 dy/dy) + a0 y in 5-point flux
form, rsp_problem.coef; oracle: oracle/system.py variable_operator, pinned in
test_oracle_pins.py).  Seeded smooth coefficient fields (synth.coefficient_fields: a1, a2
between e^-2 and e^2, a0 >= 0).

* F_eps on the whole grid and K_i on the tiles: within 64 u times the largest term.
* Local solves with the line factors (whose blocks and couplings between lines now vary
  node by node): 1e-11 relative to a sparse direct solve, FP64; 1e-4 with FP32 factors;
  the pivoting factorisation included.
* Algorithm 3 and 4 (F and its Jacobian action) and whole solves, one and two levels,
  FP64 within 1e-10 of the oracle with its outer step count, FP32 line factors within 1e-8.
* Batches mixing instances with and without coefficients, the server and the
  allocation-free residual give the same bits as single solves / rsp_local_residual.
"""
import numpy as np
import pytest

import synth
from oracle.schwarz import Raspen
from oracle.system import System

from gpu_helpers import dev, host, lib, problem_of, rel, solve

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def R():
    return lib()


def with_(o, **kw):
    import copy
    o = copy.copy(o)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


TIGHT = synth.Options(tol_outer=1e-12, tol_inner=1e-11, gmres_rtol=1e-12)


def problem(nx=37, ny=29, sx=3, sy=4, overlap=3, phi=synth.PHI_CUBIC, nu=1e-2, mu=1e-2, seed=1, eps_min=1e-6):
    return synth.Problem(nx=nx, ny=ny, phi=phi, nu=nu, mu=mu, eps0=1.0, eps_min=eps_min, gamma=0.5,
                         sx=sx, sy=sy, overlap=overlap, seed=seed, coef=1)


def to_tiles(subs, txm, tym, locs):
    T = np.zeros((len(subs), 2, tym, txm))
    for s, (sub, v) in enumerate(zip(subs, locs)):
        bx0, bx1, by0, by1 = sub.box
        tx, ty = bx1 - bx0, by1 - by0
        m = tx * ty
        T[s, 0, :ty, :tx] = v[:m].reshape(ty, tx)
        T[s, 1, :ty, :tx] = v[m:].reshape(ty, tx)
    return T


def from_tiles(subs, T):
    out = []
    for s, sub in enumerate(subs):
        bx0, bx1, by0, by1 = sub.box
        tx, ty = bx1 - bx0, by1 - by0
        out.append(np.concatenate([T[s, 0, :ty, :tx].reshape(-1), T[s, 1, :ty, :tx].reshape(-1)]))
    return out


class Case:
    def __init__(self, R, prob, opts):
        self.R, self.prob = R, prob
        self.yd, self.f = prob.inputs()
        self.rp, self.coef = problem_of(R, prob)
        self.ctx = R.rsp_context_create(0)
        R.rsp_setup(self.ctx, self.rp, R.make_options(opts), dev(self.yd), dev(self.f))
        self.S, self.txm, self.tym, _ = R.rsp_partition(self.rp)
        self.ora = Raspen(prob, opts, self.yd, self.f)
        self.n = prob.nx * prob.ny

    def close(self):
        self.R.rsp_context_destroy(self.ctx)


def rand_state(n, seed, sy=0.5, sp=0.05):
    rng = np.random.default_rng(seed)
    return np.concatenate([sy * rng.standard_normal(n), sp * rng.standard_normal(n)])


def stencil_scale(prob):
    ax, ay, a0 = prob.coefficients()
    hx2, hy2 = (prob.nx + 1) ** 2, (prob.ny + 1) ** 2
    return 2 * ax.max() * hx2 + 2 * ay.max() * hy2 + a0.max()


@pytest.mark.parametrize("phi", [synth.PHI_CUBIC, synth.PHI_EXP])
def test_residual_and_local_residual(R, phi):
    prob = problem(phi=phi)
    c = Case(R, prob, synth.Options())
    try:
        sysm = System(prob, c.yd, c.f)
        x = rand_state(c.n, 3)
        sc = stencil_scale(prob)
        for eps in [1.0, 1e-7]:
            out = dev(np.zeros(2 * c.n))
            R.rsp_residual(c.ctx, dev(x), eps, out)
            ref = sysm.residual(x, eps)
            assert np.abs(host(out) - ref).max() <= 64 * U * (sc * np.abs(x).max() + np.abs(ref).max() + 1 / prob.nu)
        rng = np.random.default_rng(8)
        locs = [np.concatenate([0.2 * rng.standard_normal(s.rows.size), 0.02 * rng.standard_normal(s.rows.size)])
                for s in c.ora.subs]
        C = to_tiles(c.ora.subs, c.txm, c.tym, locs)
        for eps in [0.5, 1e-7]:
            out = dev(np.full((c.S, 2, c.tym, c.txm), np.nan))
            norms = dev(np.zeros(c.S))
            R.rsp_local_residual(c.ctx, dev(x), dev(C), eps, out, norms)
            got = from_tiles(c.ora.subs, host(out))
            for i in range(c.S):
                ref = c.ora.local_residual(i, x, locs[i], eps)
                assert np.abs(got[i] - ref).max() <= 64 * U * (sc * 1.5 + np.abs(ref).max() + 1 / prob.nu)
            # the allocation-free entry point gives the same bits
            out2 = dev(np.full((c.S, 2, c.tym, c.txm), np.nan))
            norms2 = dev(np.zeros(c.S))
            R.rsp_local_residual_noalloc(c.rp, dev(c.yd), dev(c.f), dev(x), dev(C), eps, out2, norms2)
            assert np.array_equal(host(out2), host(out)) and np.array_equal(host(norms2), host(norms))
    finally:
        c.close()


@pytest.mark.parametrize("precision,nu,tol", [(0, 1e-2, 1e-11), (0, 1e-6, 1e-11), (1, 1e-2, 1e-4)])
def test_local_solve(R, precision, nu, tol):
    """nu = 1e-6 on this grid leaves line blocks that are not dominant (pivoting path)."""
    prob = problem(nx=23, ny=17, sx=3, sy=2, overlap=2, phi=synth.PHI_EXP, nu=nu)
    c = Case(R, prob, synth.Options(precision=precision))
    try:
        import scipy.sparse.linalg as spla
        x = rand_state(c.n, 11)
        rng = np.random.default_rng(12)
        locs = [np.concatenate([0.1 * rng.standard_normal(s.rows.size), 0.01 * rng.standard_normal(s.rows.size)])
                for s in c.ora.subs]
        rhs = [rng.standard_normal(2 * s.rows.size) for s in c.ora.subs]
        for eps in [1.0, 1e-6]:
            z = dev(np.full((c.S, 2, c.tym, c.txm), np.nan))
            R.rsp_local_solve(c.ctx, dev(x), dev(to_tiles(c.ora.subs, c.txm, c.tym, locs)), eps,
                              dev(to_tiles(c.ora.subs, c.txm, c.tym, rhs)), z)
            got = from_tiles(c.ora.subs, host(z))
            for i in range(c.S):
                ref = spla.spsolve(c.ora.local_jacobian(i, x, locs[i], eps), rhs[i])
                assert np.abs(got[i] - ref).max() <= tol * np.abs(ref).max(), (i, eps)
    finally:
        c.close()


def test_eval_and_jacobian_action(R):
    prob = problem(phi=synth.PHI_EXP, nu=1e-3, mu=5e-3)
    c = Case(R, prob, TIGHT)
    try:
        n = c.n
        x = rand_state(n, 13, 0.05, 0.005)
        for cont in [1, 0]:
            out = dev(np.zeros(2 * n))
            st, nrm = R.rsp_eval(c.ctx, dev(x), cont, out)
            ref, info = c.ora.eval_F(x, continuation=bool(cont))
            assert st == 0 and info.status == 0
            assert rel(host(out), ref) <= 1e-10
            d = np.random.default_rng(14).standard_normal(2 * n)
            jd = dev(np.zeros(2 * n))
            R.rsp_jac_apply(c.ctx, dev(d), jd)
            assert rel(host(jd), c.ora.jac_apply(d)) <= 1e-10
    finally:
        c.close()


@pytest.mark.parametrize("name,coarse", [("ragged", 0), ("ragged", 1), ("square", 0), ("square", 1)])
def test_solves_match_the_oracle(R, name, coarse):
    kw = {"ragged": dict(phi=synth.PHI_CUBIC), "square": dict(nx=63, ny=63, sx=4, sy=4, phi=synth.PHI_EXP, nu=1e-3,
                                                             mu=5e-3)}[name]
    prob = problem(**kw)
    yd, f = prob.inputs()
    o = with_(TIGHT, coarse=coarse)
    st, h, x, u = solve(R, prob, o, yd, f)
    ref = Raspen(prob, o, yd, f).solve()
    e64 = rel(x, ref["x"])
    st_m, h_m, x_m, _ = solve(R, prob, with_(o, precision=1, max_refine=0), yd, f)
    em = rel(x_m, ref["x"])
    print("%s coarse %d: FP64 outer %d (oracle %d) error %.3e; FP32 factors error %.3e" % (
        name, coarse, h["outer"], ref["outer"], e64, em))
    assert st == 0 and ref["status"] == 0 and st_m == 0
    assert h["outer"] == ref["outer"]
    assert e64 <= 1e-10 and em <= 1e-8
    # the operator matters: the Laplacian gives another solution
    base = synth.Problem(**{**prob.__dict__, "coef": 0})
    _, _, xl, _ = solve(R, base, o, yd, f)
    assert rel(xl, x) > 1e-3


def test_batch_and_server_equal_single_solves(R):
    import torch
    probs = [problem(phi=synth.PHI_EXP, nu=1e-3, mu=5e-3, seed=s) for s in (1, 2)]
    probs.append(synth.Problem(**{**problem(seed=3).__dict__, "coef": 0}))   # the Laplacian beside them
    ins = [p.inputs() for p in probs]
    o = with_(TIGHT, precision=1, max_refine=0)
    singles = [solve(R, p, o, *ins[q])[2] for q, p in enumerate(probs)]
    rps = [problem_of(R, p) for p in probs]
    inp = [(dev(a), dev(b)) for a, b in ins]
    ys, ps, us = ([dev(np.zeros((p.ny, p.nx))) for p in probs] for _ in range(3))
    ctx = R.rsp_context_create(0)
    try:
        st, hs = R.rsp_solve_batch(ctx, [rp for rp, _ in rps], R.make_options(o), [a for a, _ in inp],
                                   [b for _, b in inp], None, None, ys, ps, us)
        torch.cuda.synchronize()
    finally:
        R.rsp_context_destroy(ctx)
    assert st == 0
    for q in range(3):
        x = np.concatenate([host(ys[q]).reshape(-1), host(ps[q]).reshape(-1)])
        assert np.array_equal(x, singles[q]), q
    outs = [[dev(np.zeros((p.ny, p.nx))) for _ in range(3)] for p in probs]
    srv = R.rsp_server_create(R.make_options(o))
    try:
        tickets = [R.rsp_server_submit(srv, rps[q][0], inp[q][0], inp[q][1], *outs[q]) for q in range(3)]
        res = [R.rsp_server_wait(srv, t, 60000.0) for t in tickets]
    finally:
        R.rsp_server_destroy(srv)
    for q, (st, h) in enumerate(res):
        x = np.concatenate([host(outs[q][0]).reshape(-1), host(outs[q][1]).reshape(-1)])
        assert st == 0 and np.array_equal(x, singles[q]), q


def test_monolithic_newton_with_coefficients(R):
    """Newton_eps (the whole-system Jacobian on the GPU) reaches the oracle's solution."""
    prob = problem(nx=23, ny=17, sx=3, sy=2, overlap=2, phi=synth.PHI_CUBIC)
    yd, f = prob.inputs()
    st, h, x, u = solve(R, prob, TIGHT, yd, f, method="newton")
    ref = Raspen(prob, TIGHT, yd, f).solve()
    assert st == 0 and rel(x, ref["x"]) <= 1e-10


def test_full_size_workload_against_the_stored_oracle_answer(R):
    """255 x 255, 8 x 8 subdomains with the seeded coefficients, at the workload's own
    tolerances: the oracle's solution is stored (tests/golden/oracle_plain_coef_cfg.npz,
    written from the oracle alone).  FP64 within 1e-9 with the oracle's outer step count,
    FP32 factors within 1e-8, one and two levels."""
    import importlib.util
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("refs", os.path.join(here, "golden", "make_oracle_refs.py"))
    refs = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(refs)
    ref = refs.load("plain_coef_cfg")
    prob = refs.REFS["plain_coef_cfg"][0]()
    assert prob.coef == 1
    yd, f = prob.inputs()
    o = refs.options_of("plain_coef_cfg")
    for coarse in (0, 1):
        st, h, x, u = solve(R, prob, with_(o, coarse=coarse), yd, f)
        st_m, h_m, x_m, _ = solve(R, prob, with_(o, coarse=coarse, precision=1, max_refine=0), yd, f)
        e64, em = rel(x, ref["x"]), rel(x_m, ref["x"])
        print("255^2 with coefficients, coarse %d: FP64 outer %d (oracle %d) error %.3e; FP32 factors %.3e" % (
            coarse, h["outer"], int(ref["outer"]), e64, em))
        assert st == 0 and st_m == 0
        if coarse == 0:
            assert h["outer"] == int(ref["outer"])
        assert e64 <= 1e-9 and em <= 1e-8
