"""The full-size workloads against the oracle, element by element.

255 x 255 (8 x 8 subdomains of 32 x 32, overlap 4, phi = y^3) and 511 x 511 (16 x 16
subdomains, overlap 4, phi = exp(y) - 1): the oracle needs 1.5 to 25 minutes of one core
per solve here, so its answers are stored (tests/golden/oracle_*.npz, written by
tests/golden/make_oracle_refs.py from the oracle alone) and each GPU solve is compared
with them.

* Parity tolerances (outer and GMRES 1e-12, inner 1e-9, above the rounding floor of a
  local residual on these grids): FP64 within 1e-10 of the oracle with its outer step
  count, the mixed form as benchmarked (FP32 line factors, no refinement step) within
  1e-8.
* The workloads' own tolerances (outer 1e-10, inner 1e-8, GMRES 1e-10 with at most 300
  products): the error against the oracle's solution at the same tolerances is
  printed; FP64 within 1e-9, mixed within 1e-8.
* Snapshots of the first evaluation (one per local Newton step): on sampled subdomains
  the snapshot's core values are the oracle's local Newton iterates c_i^(k), which the
  oracle computes one subdomain at a time.  FP64: every snapshot within 1e-10.  FP32
  line factors: the directions carry the FP32 inverses' error, so the intermediate
  iterates may differ by up to 1e-4 relative (the accuracy of an FP32 block LU), and
  the last snapshot, at the converged local solutions (FP64 residuals), within 1e-8.
"""
import os

import numpy as np
import pytest

import synth
from oracle import pointwise as pw
from oracle.schwarz import Raspen

from gpu_helpers import lib, rel, solve

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def refs():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_oracle_refs",
                                                  os.path.join(HERE, "golden", "make_oracle_refs.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


REFS = refs()


@pytest.fixture(scope="module")
def R():
    return lib()


def with_(o, **kw):
    import copy
    o = copy.copy(o)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


WORKLOADS = {"plain": synth.config_plain, "precision": synth.config_precision}
MIXED = dict(precision=1, max_refine=0)      # the benchmarked mixed form


@pytest.mark.parametrize("work", ["plain", "precision"])
def test_parity_fp64_and_mixed(R, work):
    name = work + "_parity"
    ref = REFS.load(name)
    prob = WORKLOADS[work]()
    yd, f = prob.inputs()
    o = REFS.options_of(name)
    st, h, x, u = solve(R, prob, o, yd, f)
    e64 = rel(x, ref["x"])
    print("%s FP64: outer %d (oracle %d), error vs oracle %.3e" % (work, h["outer"], ref["outer"], e64))
    assert st == 0 and int(ref["status"]) == 0
    assert h["outer"] == int(ref["outer"])
    assert e64 <= 1e-10
    u_ref = pw.control(ref["x"][prob.nx * prob.ny:], prob.nu, prob.mu, prob.eps_min)
    assert rel(u, u_ref) <= 1e-10 * max(1.0, np.abs(ref["x"]).max() / prob.nu / np.abs(u_ref).max())
    st, h, x, u = solve(R, prob, with_(o, **MIXED), yd, f)
    em = rel(x, ref["x"])
    print("%s mixed: outer %d, error vs oracle %.3e" % (work, h["outer"], em))
    assert st == 0 and em <= 1e-8


@pytest.mark.parametrize("work", ["plain", "precision"])
def test_workload_tolerances(R, work):
    name = work + "_cfg"
    ref = REFS.load(name)
    prob = WORKLOADS[work]()
    yd, f = prob.inputs()
    o = REFS.options_of(name)
    st, h, x, u = solve(R, prob, o, yd, f)
    e64 = rel(x, ref["x"])
    st_m, h_m, x_m, u_m = solve(R, prob, with_(o, **MIXED), yd, f)
    em = rel(x_m, ref["x"])
    print("%s at its tolerances: FP64 outer %d (oracle %d) error %.3e; mixed outer %d error %.3e, "
          "%.3e from FP64" % (work, h["outer"], ref["outer"], e64, h_m["outer"], em, rel(x_m, x)))
    assert st == 0 and st_m == 0
    assert h["outer"] == int(ref["outer"])
    assert e64 <= 1e-9
    assert em <= 1e-8


def oracle_local_iterates(prob, opts, yd, f, i):
    """c_i^(0), c_i^(1), ... of subdomain i in the first evaluation (x^0 = 0, from eps_0)."""
    ora = Raspen(prob, opts, yd, f)
    rec = []
    ora.local_solve(i, np.zeros(2 * prob.nx * prob.ny), prob.eps0, record=rec)
    return ora.subs[i], rec


@pytest.mark.parametrize("work,precision", [("plain", 0), ("precision", 0), ("precision", 1)])
def test_snapshots_on_sampled_subdomains(R, work, precision):
    prob = WORKLOADS[work]()
    yd, f = prob.inputs()
    o = with_(synth.Options(), precision=precision, max_refine=0)
    K = 40
    st, h, x, u, snaps = solve(R, prob, o, yd, f, snapshots=K)
    assert st == 0 and 0 < h["snapshots"] <= K
    n = prob.nx * prob.ny
    S = prob.sx * prob.sy
    tol = 1e-10 if precision == 0 else 1e-4
    tol_last = 1e-10 if precision == 0 else 1e-8
    worst = last = 0.0
    for i in sorted({0, prob.sx - 1, S // 2 + prob.sx // 2, S - prob.sx, S - 1, prob.sx + 1}):
        sub, rec = oracle_local_iterates(prob, o, yd, f, i)
        m = sub.rows.size
        assert len(rec) <= h["snapshots"]
        scale = max(np.abs(rec[-1]).max(), 1e-300)
        for k in range(h["snapshots"]):
            c = rec[min(k, len(rec) - 1)]
            want = np.concatenate([c[:m][sub.core_local], c[m:][sub.core_local]])
            got = np.concatenate([snaps[k][sub.core_rows], snaps[k][n + sub.core_rows]])
            err = np.abs(got - want).max() / scale
            worst = max(worst, err)
            assert err <= tol, (i, k, err)
        last = max(last, err)
        assert err <= tol_last, (i, err)
    print("%s precision %d: %d snapshots, worst sampled error %.3e, last %.3e"
          % (work, precision, h["snapshots"], worst, last))
