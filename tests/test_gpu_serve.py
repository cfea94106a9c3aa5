"""GPU tests of the serving loop (rsp_server_*): continuous batching of solves.

Requests that arrive while a batch runs join it at the next outer iteration; a
request's y, p, u and history must be bit-identical to its own rsp_solve (all
instances here share the padded line-block size, see test_gpu_batch.py).
"""
import time

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


def prob(nx, ny, sx, sy, ov, phi=synth.PHI_CUBIC, nu=1e-2, mu=1e-2, seed=1, eps_min=1e-6):
    return synth.Problem(nx=nx, ny=ny, phi=phi, nu=nu, mu=mu, eps0=1.0, eps_min=eps_min, gamma=0.5,
                         sx=sx, sy=sy, overlap=ov, seed=seed)


REQS = [
    prob(63, 63, 2, 2, 2, seed=31),
    prob(127, 95, 4, 3, 4, phi=synth.PHI_EXP, nu=3e-3, mu=2e-2, seed=32),
    prob(80, 40, 2, 1, 0, phi=synth.PHI_PAPER, mu=0.0, seed=33),
    prob(70, 127, 2, 4, 4, nu=1e-3, mu=5e-3, seed=34, eps_min=1e-8),
    prob(66, 66, 2, 2, 3, phi=synth.PHI_ZERO, mu=3e-2, seed=35),
    prob(127, 127, 4, 4, 4, nu=1e-3, mu=5e-3, seed=36, eps_min=1e-8),
]


class Buffers:
    def __init__(self, p):
        yd, f = p.inputs()
        self.yd, self.f = dev(yd), dev(f)
        self.y, self.p, self.u = (dev(np.zeros((p.ny, p.nx))) for _ in range(3))

    def result(self):
        return np.concatenate([host(self.y).reshape(-1), host(self.p).reshape(-1)]), host(self.u).reshape(-1)


def single(R, p, opts):
    import torch
    b = Buffers(p)
    ctx = R.rsp_context_create(0)
    try:
        st, h = R.rsp_solve(ctx, R.make_problem(p), R.make_options(opts), b.yd, b.f, None, None, b.y, b.p, b.u)
        torch.cuda.synchronize()
    finally:
        R.rsp_context_destroy(ctx)
    return st, h, b.result()


@pytest.mark.parametrize("precision,graphs", [(0, 0), (1, 0), (1, 1)])
def test_served_results_equal_single_solves(R, precision, graphs):
    import torch
    opts = synth.Options(precision=precision, max_refine=0)
    tune = R.rsp_tuning(graphs=1, gm_chunk=5) if graphs else None
    srv = R.rsp_server_create(R.make_options(opts), tune=tune)
    try:
        bufs = [Buffers(p) for p in REQS]
        torch.cuda.synchronize()
        tickets = []
        for q, (p, b) in enumerate(zip(REQS, bufs)):
            tickets.append(R.rsp_server_submit(srv, R.make_problem(p), b.yd, b.f, b.y, b.p, b.u))
            if q % 2 == 1:
                time.sleep(0.03)      # later requests join a batch that is already running
        results = [R.rsp_server_wait(srv, t) for t in tickets]
        stats = R.rsp_server_stats(srv)
    finally:
        R.rsp_server_destroy(srv)
    assert stats["completed"] == len(REQS) and stats["failed"] == 0
    assert stats["mean_batch"] > 1.0
    assert 0 < stats["p50_ms"] <= stats["p99_ms"]
    for q, p in enumerate(REQS):
        st1, h1, (x1, u1) = single(R, p, opts)
        st, h = results[q]
        x, u = bufs[q].result()
        assert st == st1 == 0
        assert np.array_equal(x, x1), (q, np.abs(x - x1).max())
        assert np.array_equal(u, u1), q
        assert h["norm"] == h1["norm"] and h["gmres_its"] == h1["gmres_its"]


def test_budget_limits_the_batch_and_rejects_what_never_fits(R):
    import torch
    opts = synth.Options()
    o = R.make_options(opts)
    small = [REQS[0], REQS[2], REQS[4]]
    two = R.rsp_batch_workspace_bytes([R.make_problem(p) for p in small[:2]], o)
    big = REQS[5]
    assert R.rsp_workspace_bytes(R.make_problem(big), o) > two
    srv = R.rsp_server_create(o, max_batch=0, hbm_budget=two)
    try:
        bufs = [Buffers(p) for p in small + [big]]
        torch.cuda.synchronize()
        tickets = [R.rsp_server_submit(srv, R.make_problem(p), b.yd, b.f, b.y, b.p, b.u)
                   for p, b in zip(small + [big], bufs)]
        for t in tickets[:3]:
            st, h = R.rsp_server_wait(srv, t)
            assert st == 0
        with pytest.raises(R.RaspenError) as e:
            R.rsp_server_wait(srv, tickets[3])
        assert e.value.code == R.RSP_ENOMEM
        stats = R.rsp_server_stats(srv)
        assert stats["completed"] == 3 and stats["failed"] == 1
        assert stats["mean_batch"] <= 2.0
    finally:
        R.rsp_server_destroy(srv)
    for p, b in zip(small, bufs[:3]):
        _, _, (x1, _) = single(R, p, opts)
        assert np.array_equal(b.result()[0], x1)


def test_max_batch_one_serialises(R):
    import torch
    opts = synth.Options()
    srv = R.rsp_server_create(R.make_options(opts), max_batch=1)
    try:
        bufs = [Buffers(p) for p in REQS[:3]]
        torch.cuda.synchronize()
        tickets = [R.rsp_server_submit(srv, R.make_problem(p), b.yd, b.f, b.y, b.p, b.u)
                   for p, b in zip(REQS[:3], bufs)]
        for t in tickets:
            assert R.rsp_server_wait(srv, t)[0] == 0
        assert R.rsp_server_stats(srv)["mean_batch"] == 1.0
    finally:
        R.rsp_server_destroy(srv)


def test_invalid_requests(R):
    srv = R.rsp_server_create(R.make_options(synth.Options()))
    try:
        bad = prob(200, 31, 2, 1, 4)           # tile wider than supported
        b = Buffers(REQS[0])
        with pytest.raises(R.RaspenError) as e:
            R.rsp_server_submit(srv, R.make_problem(bad), b.yd, b.f, b.y, b.p, b.u)
        assert e.value.code == R.RSP_EINVAL
        with pytest.raises(R.RaspenError) as e:
            R.rsp_server_poll(srv, 12345)
        assert e.value.code == R.RSP_EINVAL
        t = R.rsp_server_submit(srv, R.make_problem(REQS[0]), b.yd, b.f, b.y, b.p, b.u)
        assert R.rsp_server_poll(srv, t) in (R.RSP_TICKET_QUEUED, R.RSP_TICKET_RUNNING, R.RSP_TICKET_DONE)
        assert R.rsp_server_wait(srv, t)[0] == 0
        with pytest.raises(R.RaspenError):
            R.rsp_server_wait(srv, t)           # released by the first wait
    finally:
        R.rsp_server_destroy(srv)
    with pytest.raises(R.RaspenError) as e:
        R.rsp_server_create(R.make_options(synth.Options(gmres_restart=0)))
    assert e.value.code == R.RSP_EINVAL


def test_served_full_size_request_matches_oracle(R):
    """A 255 x 255 request (8 x 8 subdomains) served among smaller ones, at the
    workload's own tolerances: within 1e-8 of the oracle's stored solution of the same
    problem and tolerances with FP32 line factors, one level and two."""
    import importlib.util
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("refs", os.path.join(here, "golden", "make_oracle_refs.py"))
    refs = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(refs)
    ref = refs.load("plain_cfg")["x"]
    big = synth.config_plain()
    for coarse in (0, 1):
        o = synth.Options(precision=1, max_refine=0, coarse=coarse)
        srv = R.rsp_server_create(R.make_options(o))
        try:
            bufs = [Buffers(p) for p in (REQS[0], big, REQS[5])]
            tickets = [R.rsp_server_submit(srv, R.make_problem(p), b.yd, b.f, b.y, b.p, b.u)
                       for p, b in zip((REQS[0], big, REQS[5]), bufs)]
            res = [R.rsp_server_wait(srv, t, 120000.0) for t in tickets]
        finally:
            R.rsp_server_destroy(srv)
        assert all(st == 0 for st, _ in res)
        x, _ = bufs[1].result()
        err = np.abs(x - ref).max() / np.abs(ref).max()
        print("served 255^2 request, coarse %d: error vs oracle %.3e" % (coarse, err))
        assert err <= 1e-8
