"""Pointwise functions of the smoothed optimality system (oracle; test infrastructure only).

* proj_[-1,1]                          -- Section 1 (definition of the projection)
* P_eps, rationalised form             -- proof of Lemma 3.1, point (i)
* P_eps, direct form                   -- Section 3.1, eq. (smoothProj)
* P'_eps                               -- Section 3.1, eq. (smoothProjDer)
* g(p) = p + mu P_eps(-p/mu), g'(p)    -- Section 3.2, eq. (reg_OS_red), and the
                                          Jacobian of F in Section 4 (x-derivative)
* u(p) = -g(p)/nu (smoothed soft-threshold, the control eliminated through the
  stationarity line of eq. (reg_OS))
* phi families allowed by Assumption 1 (phi in C^2, monotone increasing).
"""
import numpy as np

from synth import PHI_ZERO, PHI_CUBIC, PHI_EXP, PHI_PAPER


def proj(t):
    """Projection onto [-1, 1] (Section 1)."""
    return np.clip(t, -1.0, 1.0)


def P_eps(t, eps):
    """Smoothed projection, in the cancellation-free form 2t / (sqrt((t+1)^2+eps)
    + sqrt((t-1)^2+eps)) that the proof of Lemma 3.1 (i) derives from eq. (smoothProj)."""
    t = np.asarray(t, dtype=np.float64)
    return 2.0 * t / (np.sqrt((t + 1.0) ** 2 + eps) + np.sqrt((t - 1.0) ** 2 + eps))


def P_eps_direct(t, eps):
    """eq. (smoothProj) as printed: half the difference of the two shifted roots."""
    t = np.asarray(t, dtype=np.float64)
    return 0.5 * (np.sqrt((t + 1.0) ** 2 + eps) - np.sqrt((t - 1.0) ** 2 + eps))


def dP_eps(t, eps):
    """eq. (smoothProjDer): derivative of P_eps (eps > 0)."""
    t = np.asarray(t, dtype=np.float64)
    return 0.5 * ((t + 1.0) / np.sqrt((t + 1.0) ** 2 + eps)
                  - (t - 1.0) / np.sqrt((t - 1.0) ** 2 + eps))


def g(p, mu, eps):
    """p + mu * P_eps(-p/mu): the bracket of the state equation in eq. (reg_OS_red).
    For mu = 0 the term mu * P_eps is identically zero (|P_eps| <= 1), so g = p."""
    p = np.asarray(p, dtype=np.float64)
    if mu == 0.0:
        return p.copy()
    return p + mu * P_eps(-p / mu, eps)


def dg(p, mu, eps):
    """dg/dp = 1 - P'_eps(-p/mu) (the (1,2) block of the Jacobian in Section 4, times nu)."""
    p = np.asarray(p, dtype=np.float64)
    if mu == 0.0:
        return np.ones_like(p)
    return 1.0 - dP_eps(-p / mu, eps)


def control(p, nu, mu, eps):
    """u = -(1/nu) (p + mu P_eps(-p/mu)): stationarity line of eq. (reg_OS) solved for u."""
    return -g(p, mu, eps) / nu


def soft_threshold(p, mu):
    """sign(p) max(|p| - mu, 0): the eps -> 0 limit of g (Section 2, eq.
    (non-smooth_OS_reduced) with proj written out)."""
    p = np.asarray(p, dtype=np.float64)
    return np.sign(p) * np.maximum(np.abs(p) - mu, 0.0)


def phi(y, kind, kappa=0.1):
    y = np.asarray(y, dtype=np.float64)
    if kind == PHI_ZERO:
        return np.zeros_like(y)
    if kind == PHI_CUBIC:
        return y ** 3
    if kind == PHI_EXP:
        return np.exp(y) - 1.0
    if kind == PHI_PAPER:                       # Section 4 model problem
        return kappa * (y ** 3 + np.exp(kappa * y))
    raise ValueError(kind)


def dphi(y, kind, kappa=0.1):
    y = np.asarray(y, dtype=np.float64)
    if kind == PHI_ZERO:
        return np.zeros_like(y)
    if kind == PHI_CUBIC:
        return 3.0 * y ** 2
    if kind == PHI_EXP:
        return np.exp(y)
    if kind == PHI_PAPER:
        return kappa * (3.0 * y ** 2 + kappa * np.exp(kappa * y))
    raise ValueError(kind)


def ddphi(y, kind, kappa=0.1):
    y = np.asarray(y, dtype=np.float64)
    if kind == PHI_ZERO:
        return np.zeros_like(y)
    if kind == PHI_CUBIC:
        return 6.0 * y
    if kind == PHI_EXP:
        return np.exp(y)
    if kind == PHI_PAPER:
        return kappa * (6.0 * y + kappa * kappa * np.exp(kappa * y))
    raise ValueError(kind)
