"""rsp_local_residual_noalloc (no context, no device allocation) against the entry point
it varies, rsp_local_residual on a context set up with the same problem and data: the
same kernels on the same inputs, so the tiles and norms are bitwise equal.  Two calls in
a row, the second with a smaller problem (the shared staging array keeps the first
call's contents), and one problem beyond the staging limit."""
import numpy as np
import pytest

import synth

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


def case(R, prob, seed, with_f):
    """Inputs, the context result and the no-allocation result of one problem."""
    S, txm, tym, _ = R.rsp_partition(R.make_problem(prob))
    n = prob.nx * prob.ny
    rng = np.random.default_rng(seed)
    yd, f = prob.inputs()
    f = f + 0.1 * rng.standard_normal(f.shape) if with_f else f
    x = np.concatenate([0.3 * rng.standard_normal(n), 0.02 * rng.standard_normal(n)])
    c = 0.01 * rng.standard_normal((S, 2, tym, txm))
    eps = 1e-4
    want_out, want_nrm = dev(np.zeros((S, 2, tym, txm))), dev(np.zeros(S))
    ctx = R.rsp_context_create(0)
    try:
        R.rsp_setup(ctx, R.make_problem(prob), R.make_options(synth.Options()), dev(yd),
                    dev(f) if with_f else None)
        R.rsp_local_residual(ctx, dev(x), dev(c), eps, want_out, want_nrm)
        a, b = host(want_out), host(want_nrm)
    finally:
        R.rsp_context_destroy(ctx)
    got_out, got_nrm = dev(np.full((S, 2, tym, txm), np.nan)), dev(np.full(S, np.nan))
    R.rsp_local_residual_noalloc(R.make_problem(prob), dev(yd), dev(f) if with_f else None, dev(x), dev(c),
                                 eps, got_out, got_nrm)
    return a, b, host(got_out), host(got_nrm)


def test_noalloc_local_residual_equals_the_context_path(R):
    big = synth.Problem(nx=255, ny=255, phi=synth.PHI_EXP, nu=1e-3, mu=5e-3, sx=8, sy=8, overlap=4, seed=2)
    small = synth.Problem(nx=37, ny=29, phi=synth.PHI_CUBIC, nu=1e-2, mu=0.0, sx=3, sy=4, overlap=3, seed=5)
    for prob, seed, with_f in ((big, 1, True), (small, 2, False)):
        a, b, got_a, got_b = case(R, prob, seed, with_f)
        assert np.array_equal(got_a, a), prob
        assert np.array_equal(got_b, b), prob
        assert np.all(np.isfinite(got_b))


def test_noalloc_rejects_a_problem_beyond_its_staging(R):
    # 2046 x 2046 nodes in 64 x 64 subdomains of 32 (+4 overlap) nodes: 4096 halo tiles of
    # 42 x 42 nodes, 115 MB of staging, beyond the 32 MiB array
    prob = synth.Problem(nx=2046, ny=2046, sx=64, sy=64, overlap=4)
    z = dev(np.zeros(1))
    with pytest.raises(R.RaspenError) as e:
        R.rsp_local_residual_noalloc(R.make_problem(prob), z, None, z, z, 1e-4, z, z)
    assert e.value.code == R.RSP_EINVAL
