"""Plain reference of the LLG driver -- TEST INFRASTRUCTURE ONLY.

The Landau-Lifshitz-Gilbert equation of Sec. 2 for the unit magnetization,
with the damping term read as dissipative (gamma > 0):

    m_t = -g (m x H) - alpha g (m x (m x H)),   g = gamma / (1 + alpha^2),

H = H_demag(m) from the DM oracle plus a uniform external field, integrated by
explicit Heun steps with the predictor and the result renormalised to unit
length.  numpy, FP64, every step written out.
"""
from __future__ import annotations

import numpy as np


def rhs(m: np.ndarray, H: np.ndarray, alpha: float, gamma: float) -> np.ndarray:
    """m_t for fields stored [3][...] (component first)."""
    g = gamma / (1.0 + alpha * alpha)
    mh = np.cross(m, H, axis=0)
    return -g * mh - alpha * g * np.cross(m, mh, axis=0)


def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.sqrt((v * v).sum(axis=0, keepdims=True))


def heun(field, m: np.ndarray, alpha: float, gamma: float, H_ext, dt: float, steps: int) -> np.ndarray:
    """`steps` Heun steps from m; field(m) returns H_demag(m) ([3][nz][ny][nx])."""
    hext = np.asarray(H_ext, dtype=np.float64).reshape(3, *([1] * (m.ndim - 1)))
    m = np.array(m, dtype=np.float64)
    for _ in range(steps):
        k1 = rhs(m, field(m) + hext, alpha, gamma)
        ms = _unit(m + dt * k1)
        k2 = rhs(ms, field(ms) + hext, alpha, gamma)
        m = _unit(m + 0.5 * dt * (k1 + k2))
    return m
