"""Radial basis of an edge (FP64, test oracle).

This project's reading of the per-edge radial features (the paper only says that
pair energies live within a finite cutoff, Sec. 2.1):
  * polynomial cutoff u(x), x = d/r_c, of order p:
    u = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2) for x < 1, else 0;
  * Bessel functions B_n(d) = (2/r_c) sin(n pi d / r_c) / d, n = 1..n_b.
"""
from __future__ import annotations

import math

import numpy as np


def envelope(x: np.ndarray, p: int):
    """u(x) and du/dx."""
    x = np.asarray(x, dtype=np.float64)
    inside = x < 1.0
    xs = np.where(inside, x, 0.0)
    c0 = (p + 1) * (p + 2) / 2.0
    c1 = p * (p + 2)
    c2 = p * (p + 1) / 2.0
    u = 1.0 - c0 * xs ** p + c1 * xs ** (p + 1) - c2 * xs ** (p + 2)
    du = -c0 * p * xs ** (p - 1) + c1 * (p + 1) * xs ** p - c2 * (p + 2) * xs ** (p + 1)
    return np.where(inside, u, 0.0), np.where(inside, du, 0.0)


def bessel(d: np.ndarray, r_cut: float, n_b: int):
    """B [E, n_b] and dB/dd [E, n_b]."""
    d = np.asarray(d, dtype=np.float64)[:, None]
    k = (np.arange(1, n_b + 1, dtype=np.float64) * math.pi / r_cut)[None, :]
    s, c = np.sin(k * d), np.cos(k * d)
    pref = 2.0 / r_cut
    B = pref * s / d
    dB = pref * (k * c / d - s / (d * d))
    return B, dB
