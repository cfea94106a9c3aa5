"""The model problem of Section 5 at the paper's size (N = 450) against the Newton step
counts the paper prints (tests/golden/paper_model_problem_newton_steps.txt).

Algorithm 1 on the whole system, its Newton systems solved by RAS-preconditioned GMRES
(rsp_solve_newton_ras; 11 x 11 subdomains with the paper's overlap 2h, GMRES run to a
tight tolerance so that the steps are those of Newton's method).  Without continuation
the step counts are the paper's for every eps_min.  With continuation the paper's count
is reached at eps_min = 1e-15 and at eps_min = 1; for larger eps_min our loop (which
stops once |F| meets the tolerance and eps_k = eps_min) takes fewer steps than the
paper reports.
"""
import os

import numpy as np
import pytest

import synth
from cases import paper_model_problem

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "paper_model_problem_newton_steps.txt")


def golden():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                e, a, b = line.split()
                rows[float(e)] = (int(a), int(b))
    return rows


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_00546_amd import raspen
    raspen.load()
    return raspen


@pytest.fixture(scope="module")
def model():
    return paper_model_problem(450, 11, 11, 2, 1e-15)


def solve(R, prob, yd, f, cont):
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    opts = synth.Options(tol_outer=1e-10, gmres_rtol=1e-12, max_gmres=4000, max_outer=60, continuation=cont)
    y, p, u = (t(np.zeros((prob.ny, prob.nx))) for _ in range(3))
    ctx = R.rsp_context_create(0)
    try:
        st, h = R.rsp_solve_newton_ras(ctx, R.make_problem(prob), R.make_options(opts), t(yd), t(f), None,
                                       None, y, p, u)
        torch.cuda.synchronize()
    finally:
        R.rsp_context_destroy(ctx)
    return st, h, np.concatenate([y.cpu().numpy().reshape(-1), p.cpu().numpy().reshape(-1)])


def test_newton_steps_without_continuation_are_the_papers(R, model):
    prob, yd, f, xbar = model
    for eps_min, (steps, _) in sorted(golden().items()):
        prob.eps_min = eps_min
        st, h, x = solve(R, prob, yd, f, cont=1)
        assert st == 0, eps_min
        assert h["outer"] == steps, (eps_min, h["outer"], steps)
        if eps_min == 1e-15:
            # the constructed pair solves F_eps = 0 at eps = 1e-15
            assert np.abs(x - xbar).max() <= 1e-10 * np.abs(xbar).max()


@pytest.mark.parametrize("eps_min", [1.0, 1e-15])
def test_newton_steps_with_continuation_at_the_ends(R, model, eps_min):
    prob, yd, f, xbar = model
    prob.eps_min = eps_min
    st, h, x = solve(R, prob, yd, f, cont=0)
    assert st == 0
    assert h["outer"] == golden()[eps_min][1]
