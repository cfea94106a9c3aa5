"""Helpers of the GPU tests: device arrays and whole solves through the C ABI."""
import numpy as np


def lib():
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


def rel(a, b):
    """Max-norm relative difference |a - b|_inf / |b|_inf."""
    return float(np.abs(a - b).max() / np.abs(b).max())


def problem_of(R, prob):
    """(rsp_problem, coefficient tensor or None): the tensor must stay alive while the
    problem is in use."""
    cf = prob.coefficients() if getattr(prob, "coef", 0) else None
    if cf is None:
        return R.make_problem(prob), None
    import synth
    t = dev(synth.pack_coefficients(*cf))
    return R.make_problem(prob, t), t


def solve(R, prob, opts, yd, f=None, snapshots=0, method="raspen"):
    """One solve on a fresh context.  Returns (status, history, x = (y, p), u[, snaps]),
    snaps: [snapshots][2 n] host array when snapshots > 0.  A hard error raises
    R.RaspenError."""
    import copy
    import torch
    n = prob.nx * prob.ny
    y, p, u = (dev(np.zeros((prob.ny, prob.nx))) for _ in range(3))
    snap = None
    o = opts
    if snapshots:
        o = copy.copy(opts)
        o.record_eps_snapshots = snapshots
        snap = dev(np.full((snapshots, 2, prob.ny, prob.nx), np.nan))
    fn = {"raspen": R.rsp_solve, "newton_ras": R.rsp_solve_newton_ras, "newton": R.rsp_solve_newton}[method]
    ctx = R.rsp_context_create(0)
    rp, coef = problem_of(R, prob)
    try:
        st, h = fn(ctx, rp, R.make_options(o, snap), dev(yd),
                   None if f is None else dev(f), None, None, y, p, u)
        torch.cuda.synchronize()
    finally:
        R.rsp_context_destroy(ctx)
    x = np.concatenate([host(y).reshape(-1), host(p).reshape(-1)])
    out = (st, h, x, host(u).reshape(-1))
    if snapshots:
        out = out + (host(snap).reshape(snapshots, 2 * n),)
    return out
