"""GPU tests of the batched solve (rsp_solve_batch): many instances of uneven sizes
in the same launches, each with its own Algorithm 2 iteration.

  * Same padded line-block size in the batch as alone: every instance's y, p, u
    and history are bit-identical to its own rsp_solve (reductions are
    per instance and in a fixed order).
  * Mixed tile sizes (the batch pads every line block to the widest): each
    instance against the CPU oracle at the FP64 solve tolerance (1e-10 max-norm
    relative, iteration tolerances 1e-12 .. 1e-11 as in the single-solve parity).
"""
import numpy as np
import pytest

import synth
from oracle.schwarz import Raspen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_00546_amd import raspen
    raspen.load()
    return raspen


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


TIGHT = synth.Options(tol_outer=1e-12, tol_inner=1e-11, gmres_rtol=1e-12)


def prob(nx, ny, sx, sy, ov, phi=synth.PHI_CUBIC, nu=1e-2, mu=1e-2, seed=1, eps_min=1e-6):
    return synth.Problem(nx=nx, ny=ny, phi=phi, nu=nu, mu=mu, eps0=1.0, eps_min=eps_min, gamma=0.5,
                         sx=sx, sy=sy, overlap=ov, seed=seed)


# tiles 33..40 nodes wide: padded line block 80 in every instance
SAME_M = [
    prob(63, 63, 2, 2, 2, seed=11),
    prob(127, 95, 4, 3, 4, phi=synth.PHI_EXP, nu=3e-3, mu=2e-2, seed=12),
    prob(80, 40, 2, 1, 0, phi=synth.PHI_PAPER, mu=0.0, seed=13),
    prob(70, 127, 2, 4, 4, nu=1e-3, mu=5e-3, seed=14, eps_min=1e-8),
    prob(66, 66, 2, 2, 3, phi=synth.PHI_ZERO, mu=3e-2, seed=15),
]


def run_batch(R, probs, opts, x0s=None, ctx=None):
    import torch
    ys = [dev(np.zeros((p.ny, p.nx))) for p in probs]
    ps = [dev(np.zeros((p.ny, p.nx))) for p in probs]
    us = [dev(np.zeros((p.ny, p.nx))) for p in probs]
    inputs = [p.inputs() for p in probs]
    yd = [dev(a) for a, _ in inputs]
    f = [dev(b) for _, b in inputs]
    y0 = p0 = None
    if x0s is not None:
        y0 = [None if x is None else dev(x[:p.nx * p.ny].reshape(p.ny, p.nx)) for p, x in zip(probs, x0s)]
        p0 = [None if x is None else dev(x[p.nx * p.ny:].reshape(p.ny, p.nx)) for p, x in zip(probs, x0s)]
    own = ctx is None
    if own:
        ctx = R.rsp_context_create(0)
    try:
        st, hists = R.rsp_solve_batch(ctx, [R.make_problem(p) for p in probs], R.make_options(opts),
                                      yd, f, y0, p0, ys, ps, us)
        torch.cuda.synchronize()
    finally:
        if own:
            R.rsp_context_destroy(ctx)
    out = [(np.concatenate([host(y).reshape(-1), host(p).reshape(-1)]), host(u).reshape(-1))
           for y, p, u in zip(ys, ps, us)]
    return st, hists, out


def run_single(R, p, opts, ctx):
    import torch
    yd, f = p.inputs()
    y, pp, u = (dev(np.zeros((p.ny, p.nx))) for _ in range(3))
    st, hist = R.rsp_solve(ctx, R.make_problem(p), R.make_options(opts), dev(yd), dev(f), None, None, y, pp, u)
    torch.cuda.synchronize()
    return st, hist, (np.concatenate([host(y).reshape(-1), host(pp).reshape(-1)]), host(u).reshape(-1))


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_same_line_block_size_in_every_instance(R):
    for p in SAME_M:
        _, txm, _, _ = R.rsp_partition(R.make_problem(p))
        assert 64 < 2 * txm <= 80


@pytest.mark.parametrize("precision,restart", [(synth.Options().precision, 30), (1, 30), (0, 8)])
def test_batch_bitwise_equals_single_solves(R, precision, restart):
    opts = synth.Options(precision=precision, max_refine=0 if precision else 1, gmres_restart=restart)
    st, hists, out = run_batch(R, SAME_M, opts)
    ctx = R.rsp_context_create(0)
    try:
        for q, p in enumerate(SAME_M):
            st1, h1, (x1, u1) = run_single(R, p, opts, ctx)
            xb, ub = out[q]
            assert np.array_equal(xb, x1), (q, np.abs(xb - x1).max())
            assert np.array_equal(ub, u1), q
            hb = hists[q]
            assert hb["status"] == st1 == 0
            assert hb["outer"] == h1["outer"]
            assert hb["norm"] == h1["norm"]
            assert hb["gmres_its"] == h1["gmres_its"]
            assert hb["residual_final"] == h1["residual_final"]
            assert hb["newton_iterations"] == h1["newton_iterations"]
    finally:
        R.rsp_context_destroy(ctx)
    assert st == 0
    # the instances really do stop at different outer iterations / GMRES counts
    assert len({tuple(h["gmres_its"]) for h in hists}) > 1


# nu = 1e-4 on a 23 x 17 grid: 1/nu exceeds the 2/hy^2 margin, so line blocks of the
# local Jacobians lose column diagonal dominance and those subdomains take the
# partial-pivoting factorisation, in the same launches as the others
MIXED = [
    prob(23, 17, 3, 2, 2, nu=1e-4, seed=21),
    prob(31, 31, 2, 2, 2, phi=synth.PHI_EXP, mu=0.0, seed=22),
    prob(12, 9, 1, 1, 2, phi=synth.PHI_PAPER, seed=23),
    prob(37, 29, 3, 4, 3, nu=3e-3, mu=2e-2, seed=24),
    prob(5, 33, 1, 3, 1, phi=synth.PHI_ZERO, seed=25),
]


def test_batch_of_mixed_tile_sizes_matches_oracle(R):
    st, hists, out = run_batch(R, MIXED, TIGHT)
    assert st == 0
    for q, p in enumerate(MIXED):
        yd, f = p.inputs()
        ref = Raspen(p, TIGHT, yd, f).solve()
        xb, ub = out[q]
        assert ref["status"] == 0
        assert rel(xb, ref["x"]) <= 1e-10, (q, rel(xb, ref["x"]))
        uref = ref["u"].reshape(-1)
        assert rel(ub, uref) <= 1e-10 * max(1.0, np.abs(ref["x"]).max() / p.nu / np.abs(uref).max()), q
        assert hists[q]["status"] == 0
        assert hists[q]["residual_final"] <= 1e-9 * max(1.0, hists[q]["norm"][0])


def test_batch_of_one_equals_rsp_solve(R):
    p = SAME_M[1]
    st, hists, out = run_batch(R, [p], synth.Options())
    ctx = R.rsp_context_create(0)
    try:
        st1, h1, (x1, u1) = run_single(R, p, synth.Options(), ctx)
    finally:
        R.rsp_context_destroy(ctx)
    assert np.array_equal(out[0][0], x1) and np.array_equal(out[0][1], u1)
    assert hists[0]["norm"] == h1["norm"]


def test_instance_started_at_its_solution_stops_at_once(R):
    ctx = R.rsp_context_create(0)
    try:
        _, h1, (x1, _) = run_single(R, SAME_M[0], TIGHT, ctx)
    finally:
        R.rsp_context_destroy(ctx)
    # instance 0 warm-started at its own solution, the others from 0
    st, hists, out = run_batch(R, SAME_M[:3], TIGHT, x0s=[x1, None, None])
    assert st == 0
    assert hists[0]["outer"] <= 1 and rel(out[0][0], x1) <= 1e-10
    assert hists[1]["outer"] > hists[0]["outer"] and hists[2]["outer"] > hists[0]["outer"]


def test_context_reuse_across_batches_and_single_calls(R):
    """One context: a batch, then a different batch, then rsp_setup + single calls."""
    import torch
    ctx = R.rsp_context_create(0)
    try:
        st, hist_a, out_a = run_batch(R, SAME_M[:2], synth.Options(), ctx=ctx)
        st2, _, out_b = run_batch(R, SAME_M[2:], synth.Options(), ctx=ctx)
        st3, _, out_a2 = run_batch(R, SAME_M[:2], synth.Options(), ctx=ctx)
        assert st == st2 == st3 == 0
        for a, b in zip(out_a, out_a2):
            assert np.array_equal(a[0], b[0])
        p = SAME_M[0]
        yd, f = p.inputs()
        R.rsp_setup(ctx, R.make_problem(p), R.make_options(synth.Options()), dev(yd), dev(f))
        out = dev(np.zeros(2 * p.nx * p.ny))
        R.rsp_residual(ctx, dev(out_a[0][0]), p.eps_min, out)
        torch.cuda.synchronize()
        nrm = np.linalg.norm(host(out))
        assert abs(nrm - hist_a[0]["residual_final"]) <= 1e-10 * nrm
    finally:
        R.rsp_context_destroy(ctx)


def test_batch_rejects_bad_input(R):
    import torch
    ctx = R.rsp_context_create(0)
    try:
        good = SAME_M[0]
        bad = prob(200, 31, 2, 1, 4)          # tile wider than supported
        opts = R.make_options(synth.Options())
        y = [dev(np.zeros((p.ny, p.nx))) for p in (good, bad)]
        yd = [dev(p.inputs()[0]) for p in (good, bad)]
        with pytest.raises(R.RaspenError) as e:
            R.rsp_solve_batch(ctx, [R.make_problem(good), R.make_problem(bad)], opts, yd, None, None,
                              None, y, y, y)
        assert e.value.code == R.RSP_EINVAL
        with pytest.raises(R.RaspenError) as e:
            R.rsp_solve_batch(ctx, [], opts, [], None, None, None, [], [], [])
        assert e.value.code == R.RSP_EINVAL
        torch.cuda.synchronize()
    finally:
        R.rsp_context_destroy(ctx)


def test_batch_budget(R):
    opts = R.make_options(synth.Options())
    probs = [R.make_problem(p) for p in SAME_M]
    need = R.rsp_batch_workspace_bytes(probs, opts)
    assert need > max(R.rsp_workspace_bytes(p, opts) for p in probs)
    ctx = R.rsp_context_create(0, need - 1)
    try:
        y = [dev(np.zeros((p.ny, p.nx))) for p in SAME_M]
        yd = [dev(p.inputs()[0]) for p in SAME_M]
        with pytest.raises(R.RaspenError) as e:
            R.rsp_solve_batch(ctx, probs, opts, yd, None, None, None, y, y, y)
        assert e.value.code == R.RSP_ENOMEM
    finally:
        R.rsp_context_destroy(ctx)


# draws of the uneven batch workload (synth.batch_instances: nu = 10^U(-4,-1), mu ~ U(0, 0.05),
# phi in {y^3, exp(y) - 1}, 32 x 32-node subdomains, overlap 4, eps 1 -> 1e-8); the draws
# with grids up to 127 x 127, whose oracle solves take seconds
PARITY = synth.Options(tol_outer=1e-12, tol_inner=1e-9, gmres_rtol=1e-12)


def batch_draws():
    """The two draws with the smallest nu and the first two others (the smaller grids)."""
    out = [p for p in synth.batch_instances(24) if max(p.nx, p.ny) <= 127]
    low = sorted(out, key=lambda p: p.nu)[:2]
    return low + [p for p in out if p not in low][:2]


@pytest.fixture(scope="module")
def draws():
    probs = batch_draws()
    refs = []
    for p in probs:
        yd, f = p.inputs()
        refs.append(Raspen(p, PARITY, yd, f).solve()["x"])
    return probs, refs


@pytest.mark.parametrize("precision,coarse", [(0, 0), (1, 0), (1, 1)])
def test_batch_workload_draws_match_oracle(R, draws, precision, coarse):
    """FP64 within 1e-10 of the oracle, the mixed form (FP32 line factors, no refinement
    step) within 1e-8, one level and two."""
    probs, refs = draws
    assert min(p.nu for p in probs) < 1e-3 and len({(p.nx, p.ny) for p in probs}) > 1
    o = synth.Options(tol_outer=PARITY.tol_outer, tol_inner=PARITY.tol_inner, gmres_rtol=PARITY.gmres_rtol,
                      precision=precision, max_refine=0, coarse=coarse)
    st, hists, out = run_batch(R, probs, o)
    assert st == 0
    for q, p in enumerate(probs):
        err = rel(out[q][0], refs[q])
        print("draw %d (%dx%d, nu %.1e, mu %.3f, phi %d): error %.3e" % (q, p.nx, p.ny, p.nu, p.mu, p.phi, err))
        assert err <= (1e-10 if precision == 0 else 1e-8), (q, err)
