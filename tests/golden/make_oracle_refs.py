"""Writes the oracle's solutions of the full-size workloads (tests/golden/oracle_*.npz).

Only the oracle (``oracle/``) and the seeded inputs (``synth``) run here; nothing
comes from the HIP path.  The oracle takes minutes to tens of minutes per workload on
one core, far longer than a GPU test may run, so its answers are stored once and the
GPU tests and ``bench.py`` compare against them.

    python tests/golden/make_oracle_refs.py [name ...]

Each file holds x = (y, p) (float64, [2 nx ny]; u follows from p), the status, the
outer iteration count, the history of |F(x^k)|_2 and GMRES products and the oracle's
time; names are listed in REFS.
"""
import dataclasses
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.schwarz import Raspen  # noqa: E402

# Parity tolerances for the full-size grids: the outer and GMRES tolerances of the
# parity runs (1e-12), and an inner tolerance above the FP64 rounding floor of a local
# residual there (the 5-point entries are 4/h^2 ~ 2.6e5 at 255^2 and 1.0e6 at 511^2,
# so one evaluation of K_i on a 40 x 40 tile carries ~1e-10 of rounding).
PARITY = dict(tol_outer=1e-12, tol_inner=1e-9, gmres_rtol=1e-12)

REFS = {
    # 255 x 255, 8 x 8 subdomains: at the workload's own tolerances and at parity ones
    "plain_cfg": (synth.config_plain, {}),
    "plain_parity": (synth.config_plain, PARITY),
    # 511 x 511, 16 x 16 subdomains, phi = exp(y) - 1 (at its own tolerances GMRES stops
    # at the 300-product cap in most outer steps; the parity run lets it converge)
    "precision_cfg": (synth.config_precision, {}),
    "precision_parity": (synth.config_precision, dict(PARITY, max_gmres=1000)),
    # the 255 x 255 workload with the seeded variable coefficients of A
    "plain_coef_cfg": (lambda: dataclasses.replace(synth.config_plain(), coef=1), {}),
}


def path_of(name):
    return os.path.join(HERE, "oracle_%s.npz" % name)


def options_of(name):
    return synth.Options(**REFS[name][1])


def make(name):
    prob = REFS[name][0]()
    opts = options_of(name)
    yd, f = prob.inputs()
    t0 = time.perf_counter()
    r = Raspen(prob, opts, yd, f).solve()
    dt = time.perf_counter() - t0
    h = r["history"]
    np.savez_compressed(path_of(name), x=r["x"], status=r["status"], outer=r["outer"],
                        norms=np.array([e["norm"] for e in h]),
                        gmres=np.array([e["gmres"] for e in h]),
                        inner_max=np.array([max(e["inner"]) for e in h]), seconds=dt)
    print("%s: status %d, %d outer, %.1f s" % (name, r["status"], r["outer"], dt), flush=True)


def load(name):
    """The stored reference as a dict (raises if it has not been made)."""
    with np.load(path_of(name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(REFS)):
        make(n)
