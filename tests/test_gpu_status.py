"""Status codes of the boundary on the GPU path, and the per-eps-step snapshots.

* RSP_ENUMERIC (-4): a local residual, Newton direction or assembled residual that is
  not finite (NaN or Inf in the data) ends the solve as a hard error, in every method,
  and in a batch only for the instance concerned.
* RSP_REFINE_FALLBACK (4): with FP32 line factors an instance that stalls leaves them
  for FP64 factors and continues from its iterate; fallback_rho = 0 forces the switch
  after outer step 1, and the answer is then the FP64 one (within 1e-10 of the oracle).
* Snapshots of the first evaluation (record_eps_snapshots): x^0 + sum_i P~_i c_i^(k)
  after each local Newton (eps) step k of Algorithm 1, against the oracle's iterates.
"""
import numpy as np
import pytest

import synth
from oracle.schwarz import Raspen

from gpu_helpers import dev, host, lib, rel, solve

pytestmark = pytest.mark.gpu

TIGHT = synth.Options(tol_outer=1e-12, tol_inner=1e-11, gmres_rtol=1e-12)


@pytest.fixture(scope="module")
def R():
    return lib()


def ragged(phi=synth.PHI_CUBIC, nu=1e-2, mu=1e-2, seed=1, nx=37, ny=29, sx=3, sy=4, overlap=3):
    return synth.Problem(nx=nx, ny=ny, phi=phi, nu=nu, mu=mu, eps0=1.0, eps_min=1e-6, gamma=0.5,
                         sx=sx, sy=sy, overlap=overlap, seed=seed)


def opts_with(base, **kw):
    import copy
    o = copy.copy(base)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------ RSP_ENUMERIC
@pytest.mark.parametrize("method", ["raspen", "newton_ras", "newton"])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("bad", ["nan", "inf", "overflow"])
def test_nonfinite_data_is_a_numeric_error(R, method, precision, bad):
    if method == "newton" and precision == 1:
        pytest.skip("Newton_eps has no line factors")
    prob = ragged()
    yd, f = prob.inputs()
    if bad == "nan":
        yd[3, 4] = np.nan
    elif bad == "inf":
        f[10, 20] = np.inf
    else:
        yd = yd * 1e200          # |K|^2 overflows: the residual norm is not finite
    with pytest.raises(R.RaspenError) as e:
        solve(R, prob, opts_with(TIGHT, precision=precision, max_outer=5), yd, f, method=method)
    assert e.value.code == R.RSP_ENUMERIC and "finite" in str(e.value)


def test_numeric_error_in_a_batch_is_per_instance(R):
    """One instance with a NaN in its data: it alone ends with RSP_ENUMERIC, the call
    returns that code, and the other instances converge to their own answers."""
    import torch
    probs = [ragged(seed=s) for s in (1, 2, 3)]
    ins = [p.inputs() for p in probs]
    ins[1][0][5, 5] = np.nan
    ys, ps, us = ([dev(np.zeros((p.ny, p.nx))) for p in probs] for _ in range(3))
    ctx = R.rsp_context_create(0)
    try:
        st, hs = R.rsp_solve_batch(ctx, [R.make_problem(p) for p in probs], R.make_options(TIGHT),
                                   [dev(a) for a, _ in ins], [dev(b) for _, b in ins], None, None, ys, ps, us)
        torch.cuda.synchronize()
    finally:
        R.rsp_context_destroy(ctx)
    assert st == R.RSP_ENUMERIC
    assert [h["status"] for h in hs] == [0, R.RSP_ENUMERIC, 0]
    for q in (0, 2):
        ref = Raspen(probs[q], TIGHT, *ins[q]).solve()
        x = np.concatenate([host(ys[q]).reshape(-1), host(ps[q]).reshape(-1)])
        assert rel(x, ref["x"]) <= 1e-10


# ------------------------------------------------------------------ RSP_REFINE_FALLBACK
FORCED = opts_with(TIGHT, precision=1, max_refine=0, fallback_rho=0.0)


@pytest.mark.parametrize("phi,nu,mu", [(synth.PHI_EXP, 1e-3, 5e-3), (synth.PHI_CUBIC, 1e-4, 1e-2)])
def test_forced_fallback_ends_with_the_fp64_answer(R, phi, nu, mu):
    prob = ragged(phi=phi, nu=nu, mu=mu)
    yd, f = prob.inputs()
    st, h, x, u = solve(R, prob, FORCED, yd, f)
    ref = Raspen(prob, TIGHT, yd, f).solve()
    assert ref["outer"] >= 2          # not converged at step 1, so the switch happens there
    assert st == R.RSP_REFINE_FALLBACK and h["status"] == st
    assert h["fallback_outer"] == 1
    assert rel(x, ref["x"]) <= 1e-10


def test_no_fallback_when_fp32_converges(R):
    for phi, nu, mu in [(synth.PHI_EXP, 1e-3, 5e-3), (synth.PHI_CUBIC, 1e-2, 1e-2)]:
        prob = ragged(phi=phi, nu=nu, mu=mu)
        yd, f = prob.inputs()
        st, h, x, u = solve(R, prob, opts_with(TIGHT, precision=1, max_refine=0), yd, f)
        assert st == 0 and h["fallback_outer"] == -1


def test_fp64_solves_never_fall_back(R):
    prob = ragged(phi=synth.PHI_EXP, nu=1e-3, mu=5e-3)
    yd, f = prob.inputs()
    st, h, x, u = solve(R, prob, opts_with(TIGHT, fallback_rho=0.0), yd, f)
    assert st == 0 and h["fallback_outer"] == -1


def test_forced_fallback_in_a_batch(R):
    """Every member is switched after its step 1 (one FP64 layout for all of them) and
    ends with the oracle's answer; an instance that converges in one step keeps its
    FP32 result."""
    import torch
    probs = [ragged(phi=synth.PHI_EXP, nu=1e-3, mu=5e-3, seed=s) for s in (1, 2)]
    probs.append(ragged(nx=12, ny=9, sx=1, sy=1, overlap=2, seed=4))   # one subdomain: 1 step
    ins = [p.inputs() for p in probs]
    ys, ps, us = ([dev(np.zeros((p.ny, p.nx))) for p in probs] for _ in range(3))
    ctx = R.rsp_context_create(0)
    try:
        st, hs = R.rsp_solve_batch(ctx, [R.make_problem(p) for p in probs], R.make_options(FORCED),
                                   [dev(a) for a, _ in ins], [dev(b) for _, b in ins], None, None, ys, ps, us)
        torch.cuda.synchronize()
    finally:
        R.rsp_context_destroy(ctx)
    assert [h["status"] for h in hs] == [R.RSP_REFINE_FALLBACK, R.RSP_REFINE_FALLBACK, 0]
    assert [h["fallback_outer"] for h in hs] == [1, 1, -1]
    for q, p in enumerate(probs):
        ref = Raspen(p, TIGHT, *ins[q]).solve()
        x = np.concatenate([host(ys[q]).reshape(-1), host(ps[q]).reshape(-1)])
        assert rel(x, ref["x"]) <= (1e-10 if q < 2 else 1e-8)


def test_forced_fallback_in_the_server(R):
    """Served requests that leave the FP32 factors finish in the server's FP64 batch."""
    probs = [ragged(phi=synth.PHI_EXP, nu=1e-3, mu=5e-3, seed=s) for s in (1, 2, 3)]
    ins = [p.inputs() for p in probs]
    inp = [(dev(a), dev(b)) for a, b in ins]      # inputs stay alive until the tickets are done
    outs = [[dev(np.zeros((p.ny, p.nx))) for _ in range(3)] for p in probs]
    srv = R.rsp_server_create(R.make_options(FORCED))
    try:
        tickets = [R.rsp_server_submit(srv, R.make_problem(p), inp[q][0], inp[q][1], *outs[q])
                   for q, p in enumerate(probs)]
        res = [R.rsp_server_wait(srv, t, 60000.0) for t in tickets]
    finally:
        R.rsp_server_destroy(srv)
    for q, (st, h) in enumerate(res):
        assert st == R.RSP_REFINE_FALLBACK and h["fallback_outer"] == 1
        ref = Raspen(probs[q], TIGHT, *ins[q]).solve()
        x = np.concatenate([host(outs[q][0]).reshape(-1), host(outs[q][1]).reshape(-1)])
        assert rel(x, ref["x"]) <= 1e-10


# ------------------------------------------------------------------ eps-step snapshots
@pytest.mark.parametrize("name,phi,nu,mu", [("ragged", synth.PHI_CUBIC, 1e-2, 1e-2),
                                            ("ragged", synth.PHI_EXP, 1e-3, 5e-3),
                                            ("rect", synth.PHI_CUBIC, 1e-4, 0.0)])
def test_snapshots_match_the_oracle(R, name, phi, nu, mu):
    """Snapshot k is x^0 + sum_i P~_i c_i^(k) with c_i^(k) the k-th local Newton iterate of
    the first evaluation (the last one for a subdomain that has stopped): every snapshot
    within 1e-10 of the oracle's, with eps_k = max(gamma^k eps_0, eps_min)."""
    kw = {} if name == "ragged" else dict(nx=23, ny=17, sx=3, sy=2, overlap=2)
    prob = ragged(phi=phi, nu=nu, mu=mu, **kw)
    yd, f = prob.inputs()
    K = 40
    st, h, x, u, snaps = solve(R, prob, TIGHT, yd, f, snapshots=K)
    ref = Raspen(prob, TIGHT, yd, f).solve(snapshots=True)
    want = ref["snapshots"]
    assert st == 0 and h["snapshots"] == len(want) <= K
    for k, v in enumerate(want):
        scale = max(np.abs(v).max(), 1e-300)
        assert np.abs(snaps[k] - v).max() <= 1e-10 * scale, k
    eps = [prob.eps0]
    for _ in range(1, len(want)):
        eps.append(max(prob.gamma * eps[-1], prob.eps_min))
    assert np.allclose(h["snapshot_eps"], eps, rtol=0, atol=0)
    assert np.all(np.isnan(snaps[len(want):]))      # slots beyond the recorded ones untouched


def test_snapshots_fp32_factors_and_truncation(R):
    """FP32 line factors: the local Newton directions carry the FP32 inverses' error, so
    the intermediate iterates differ from the oracle's by up to that error times the
    step (bounded by 1e-4 relative, the accuracy of an FP32 block LU here); the residual
    is FP64, so the last snapshot, at the converged local solutions, is within 1e-8.
    With fewer slots than steps only the first ones are written."""
    prob = ragged(phi=synth.PHI_EXP, nu=1e-3, mu=5e-3)
    yd, f = prob.inputs()
    ref = Raspen(prob, TIGHT, yd, f).solve(snapshots=True)["snapshots"]
    o = opts_with(TIGHT, precision=1, max_refine=0)
    st, h, x, u, snaps = solve(R, prob, o, yd, f, snapshots=8)
    assert st == 0 and h["snapshots"] == 8
    for k in range(8):
        assert np.abs(snaps[k] - ref[k]).max() <= 1e-4 * max(np.abs(ref[k]).max(), 1e-300), k
    st, h, x, u, snaps = solve(R, prob, o, yd, f, snapshots=40)
    K = h["snapshots"]
    assert st == 0 and K == len(ref)
    worst = max(np.abs(snaps[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300) for k in range(1, K))
    print("FP32 snapshots: worst intermediate error %.3e, last %.3e" %
          (worst, np.abs(snaps[K - 1] - ref[-1]).max() / np.abs(ref[-1]).max()))
    assert np.abs(snaps[K - 1] - ref[-1]).max() <= 1e-8 * np.abs(ref[-1]).max()


def test_snapshots_only_in_single_solves(R):
    prob = ragged()
    yd, f = prob.inputs()
    o = opts_with(TIGHT, record_eps_snapshots=4)
    buf = dev(np.zeros((4, 2, prob.ny, prob.nx)))
    y, p, u = (dev(np.zeros((prob.ny, prob.nx))) for _ in range(3))
    ctx = R.rsp_context_create(0)
    try:
        with pytest.raises(R.RaspenError) as e:
            R.rsp_solve_batch(ctx, [R.make_problem(prob)], R.make_options(o, buf), [dev(yd)], [dev(f)],
                              None, None, [y], [p], [u])
        assert e.value.code == R.RSP_EINVAL
        with pytest.raises(R.RaspenError) as e:
            R.rsp_solve_newton_ras(ctx, R.make_problem(prob), R.make_options(o, buf), dev(yd), dev(f),
                                   None, None, y, p, u)
        assert e.value.code == R.RSP_EINVAL
    finally:
        R.rsp_context_destroy(ctx)
