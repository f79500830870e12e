"""Seeded synthetic weights: W ~ N(0, 1/fan_in), drawn in blob order.

The caller passes the list of (fan_in, fan_out) segments; each segment is a
row-major [fan_in, fan_out] matrix of a linear map y = x W. Standard normals come
from numpy's PCG64 generator in segment order and are scaled by fan_in^-1/2.
"""
from __future__ import annotations

import numpy as np


def weight_blob(seed: int, segments) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in segments:
        parts.append(rng.standard_normal(int(fan_in) * int(fan_out)) / np.sqrt(float(fan_in)))
    if not parts:
        return np.zeros(0)
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float64)
