"""Seeded synthetic workloads shared by the HIP path's tests/bench and the CPU oracle.

This module only draws numbers and lays them out on the grid.  It holds none of
the method's arithmetic (no operator, no nonlinearity, no solver), so that the
oracle and the HIP path, which share nothing else, can be fed identical inputs.

Grid convention (both sides): the unit square, ``nx`` x ``ny`` interior nodes,
``hx = 1/(nx+1)``, ``hy = 1/(ny+1)``; node (i, j) sits at ((i+1) hx, (j+1) hy);
arrays are row-major ``[ny][nx]`` (x index fastest), float64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

PHI_ZERO, PHI_CUBIC, PHI_EXP, PHI_PAPER = 0, 1, 2, 3
PHI_NAMES = {PHI_ZERO: "0", PHI_CUBIC: "y^3", PHI_EXP: "exp(y)-1",
             PHI_PAPER: "kappa(y^3+exp(kappa y))"}


def node_coords(nx: int, ny: int):
    """Coordinates (X, Y), each ``[ny][nx]``, of the interior nodes."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    xs = (np.arange(nx, dtype=np.float64) + 1.0) * hx
    ys = (np.arange(ny, dtype=np.float64) + 1.0) * hy
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return X, Y


def gaussian_bumps(nx: int, ny: int, seed: int, nbumps: int = 8) -> np.ndarray:
    """Desired state y_d: a sum of ``nbumps`` Gaussian bumps at the interior nodes.

    Draw order (one ``numpy.random.default_rng(seed)``), per bump:
    centre x ~ U[0.1, 0.9], centre y ~ U[0.1, 0.9], width w ~ U[0.05, 0.2],
    amplitude a ~ U[-1, 1]; bump = a * exp(-|X - c|^2 / (2 w^2)).
    """
    rng = np.random.default_rng(seed)
    X, Y = node_coords(nx, ny)
    yd = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(nbumps):
        cx = rng.uniform(0.1, 0.9)
        cy = rng.uniform(0.1, 0.9)
        w = rng.uniform(0.05, 0.2)
        a = rng.uniform(-1.0, 1.0)
        yd += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * w * w))
    return yd


def random_state(nx: int, ny: int, seed: int, scale_y: float = 0.5,
                 scale_p: float = 0.05):
    """A random (y, p) pair for kernel-level parity checks (smooth + noise)."""
    rng = np.random.default_rng(seed)
    X, Y = node_coords(nx, ny)
    base = np.sin(np.pi * X) * np.sin(np.pi * Y)
    y = scale_y * (base * rng.uniform(-1, 1) + 0.3 * rng.standard_normal((ny, nx)))
    p = scale_p * (base * rng.uniform(-1, 1) + 0.5 * rng.standard_normal((ny, nx)))
    return y, p


def smooth_field(xs, ys, seed: int, nbumps: int = 4) -> np.ndarray:
    """A smooth field at the points (xs, ys) (equal-shape arrays): the sum of
    ``nbumps`` Gaussian bumps.  Draw order (one ``numpy.random.default_rng(seed)``), per
    bump: centre x ~ U[0, 1], centre y ~ U[0, 1], width ~ U[0.1, 0.3], amplitude ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    out = np.zeros(np.shape(xs), dtype=np.float64)
    for _ in range(nbumps):
        cx = rng.uniform(0.0, 1.0)
        cy = rng.uniform(0.0, 1.0)
        w = rng.uniform(0.1, 0.3)
        a = rng.uniform(-1.0, 1.0)
        out += a * np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2.0 * w * w))
    return out


def coefficient_fields(nx: int, ny: int, seed: int):
    """Coefficients of A y = -d/dx(a1 dy/dx) - d/dy(a2 dy/dy) + a0 y (a diagonal
    coefficient tensor): a1 at the x-faces, a2 at the y-faces, a0 at the nodes.

    a1 = exp(B1), a2 = exp(B2), a0 = 5 B3^2 with B1, B2, B3 smooth_field draws with
    seeds 3 seed + 1, 3 seed + 2, 3 seed + 3.  Face (i, j) of ``ax`` ([ny][nx+1]) lies
    between nodes i-1 and i of row j, at ((i + 1/2) hx, (j + 1) hy); face (i, j) of
    ``ay`` ([ny+1][nx]) between rows j-1 and j of column i, at ((i + 1) hx, (j + 1/2) hy);
    index -1 and nx (ny) are the Dirichlet boundary."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    xf, yf = np.meshgrid((np.arange(nx + 1) + 0.5) * hx, (np.arange(ny) + 1.0) * hy, indexing="xy")
    ax = np.exp(smooth_field(xf, yf, 3 * seed + 1))
    xg, yg = np.meshgrid((np.arange(nx) + 1.0) * hx, (np.arange(ny + 1) + 0.5) * hy, indexing="xy")
    ay = np.exp(smooth_field(xg, yg, 3 * seed + 2))
    X, Y = node_coords(nx, ny)
    a0 = 5.0 * smooth_field(X, Y, 3 * seed + 3) ** 2
    return ax, ay, a0


def pack_coefficients(ax, ay, a0) -> np.ndarray:
    """The coefficient layout of the C ABI: ax, ay, a0 back to back, float64."""
    return np.concatenate([np.ravel(ax), np.ravel(ay), np.ravel(a0)]).astype(np.float64)


@dataclasses.dataclass
class Problem:
    """Problem data of the smoothed optimality system (paper, eq. (P) and the
    reduced smoothed system of Section 3.2) plus the Schwarz partition.

    ``coef`` = 0: A = -Laplacian (the model problem); 1: A with the seeded variable
    coefficients of ``coefficient_fields(nx, ny, seed)``."""
    nx: int
    ny: int
    phi: int = PHI_CUBIC
    kappa: float = 0.1
    nu: float = 1e-2
    mu: float = 1e-2
    eps0: float = 1.0
    eps_min: float = 1e-6
    gamma: float = 0.5
    sx: int = 2
    sy: int = 2
    overlap: int = 2
    seed: int = 1
    coef: int = 0

    def inputs(self):
        """(y_d, f) for this problem: bumps for y_d, f = 0."""
        yd = gaussian_bumps(self.nx, self.ny, self.seed)
        f = np.zeros((self.ny, self.nx), dtype=np.float64)
        return yd, f

    def coefficients(self):
        """(ax, ay, a0) of the operator, or None for the Laplacian (coef = 0)."""
        if not self.coef:
            return None
        return coefficient_fields(self.nx, self.ny, self.seed)


@dataclasses.dataclass
class Options:
    """Solver options (paper Section 5 defaults where it states them)."""
    tol_outer: float = 1e-10
    tol_inner: float = 1e-8
    gmres_rtol: float = 1e-10
    sigma: float = 1.1
    alpha_min: float = 2.0 ** -30
    gmres_restart: int = 30
    max_outer: int = 50
    max_inner: int = 200
    max_gmres: int = 300
    precision: int = 0          # 0 FP64, 1 FP32 factors + FP64 refinement
    max_refine: int = 1
    continuation: int = 0       # 0 first evaluation, 1 none, 2 every evaluation
    record_eps_snapshots: int = 0   # snapshots of the first evaluation (GPU path only)
    tol_inner_rel: float = -1.0     # relative branch of the inner test (< 0: tol_inner)
    fallback_rho: float = 1.0       # FP32 -> FP64 switch (GPU path only; < 0: never)
    coarse: int = 0                 # 1: second level for the outer Newton systems


def subdomains_for(n: int, size: int = 32) -> int:
    """Number of subdomains per side so that each non-overlapping box is ``size`` wide."""
    return max(1, math.ceil(n / size))


# ---- the named workloads ----------------------------------------------------

def config_small() -> Problem:
    """63x63 grid, phi=y^3, nu=mu=1e-2, eps 1 -> 1e-6 halving, 2x2 subdomains, overlap 2."""
    return Problem(nx=63, ny=63, phi=PHI_CUBIC, nu=1e-2, mu=1e-2, eps0=1.0,
                   eps_min=1e-6, gamma=0.5, sx=2, sy=2, overlap=2, seed=1)


def config_plain() -> Problem:
    """255x255 grid, phi=y^3, nu=1e-3, mu=5e-3, eps 1 -> 1e-8 halving,
    8x8 subdomains (32x32 non-overlapping), overlap 4."""
    return Problem(nx=255, ny=255, phi=PHI_CUBIC, nu=1e-3, mu=5e-3, eps0=1.0,
                   eps_min=1e-8, gamma=0.5, sx=8, sy=8, overlap=4, seed=2)


def config_precision() -> Problem:
    """511x511 grid, phi=exp(y)-1, 16x16 subdomains, overlap 4 (nu, mu and the eps
    schedule are not stated for this workload: taken from the 255x255 one)."""
    return Problem(nx=511, ny=511, phi=PHI_EXP, nu=1e-3, mu=5e-3, eps0=1.0,
                   eps_min=1e-8, gamma=0.5, sx=16, sy=16, overlap=4, seed=3)


def batch_instances(count: int = 64, base_seed: int = 1000,
                    sizes=(63, 127, 255)) -> List[Problem]:
    """Uneven batch: instance k draws (with seed base_seed + k, in this order)
    nx, ny from ``sizes``, log10(nu) ~ U[-4, -1], mu ~ U[0, 0.05],
    phi from {y^3, exp(y)-1}; 32x32 subdomains, overlap 4, eps 1 -> 1e-8 halving."""
    out = []
    for k in range(count):
        rng = np.random.default_rng(base_seed + k)
        nx = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        nu = float(10.0 ** rng.uniform(-4.0, -1.0))
        mu = float(rng.uniform(0.0, 0.05))
        phi = int(rng.choice([PHI_CUBIC, PHI_EXP]))
        out.append(Problem(nx=nx, ny=ny, phi=phi, nu=nu, mu=mu, eps0=1.0,
                           eps_min=1e-8, gamma=0.5, sx=subdomains_for(nx),
                           sy=subdomains_for(ny), overlap=4, seed=base_seed + k))
    return out


def request_stream(count: int, rate: float, seed: int = 5,
                   sizes=(127, 255, 511)):
    """Poisson request stream: exponential inter-arrival times with ``rate``
    (requests/s); each request is a Problem drawn like ``batch_instances``
    from ``sizes``.  Returns (arrival_times, problems)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    probs = batch_instances(count, base_seed=seed * 100000, sizes=sizes)
    return arrivals, probs


def config_by_name(name: str) -> Problem:
    return {"small": config_small, "plain": config_plain,
            "precision": config_precision}[name]()
