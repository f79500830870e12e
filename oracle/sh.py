"""Real spherical harmonics and Clebsch-Gordan coupling tables (FP64, test oracle).

Part of the test oracle: tensors up to rank l and their products over
irreducible representations (Sec. 2.1). Conventions (this project's reading; the
paper prints none):
  * component normalisation, sum_m Y_lm(r)^2 = 2l+1 on the unit sphere;
  * order l=1: sqrt3 (x, y, z);
    l=2: (sqrt15 xy, sqrt15 yz, sqrt5/2 (3z^2-1), sqrt15 xz, sqrt15/2 (x^2-y^2));
  * paths (l1,l2,l3) with l_i <= lmax, |l1-l2| <= l3 <= l1+l2 and l1+l2+l3 even,
    in lexicographic order (natural-parity irreps only, so E is also invariant
    under inversion);
  * C^(l1,l2,l3) is the real Gaunt tensor (1/4pi) * integral of
    Y_l1m1 Y_l2m2 Y_l3m3 over the sphere, scaled to unit Frobenius norm, with the
    sign chosen so that its first non-zero entry in (m1,m2,m3) order is positive.
    The integral is evaluated by a product rule (Gauss-Legendre in z, uniform in
    phi) that is exact for these polynomial degrees.
"""
from __future__ import annotations

import math

import numpy as np

S3 = math.sqrt(3.0)
S5 = math.sqrt(5.0)
S15 = math.sqrt(15.0)
LMAX_SUPPORTED = 2


def real_sh(l: int, rhat: np.ndarray) -> np.ndarray:
    """Y_l(rhat) for unit vectors rhat [..., 3] -> [..., 2l+1]."""
    x, y, z = rhat[..., 0], rhat[..., 1], rhat[..., 2]
    if l == 0:
        return np.ones(rhat.shape[:-1] + (1,))
    if l == 1:
        return S3 * np.stack([x, y, z], axis=-1)
    if l == 2:
        return np.stack([S15 * x * y, S15 * y * z, 0.5 * S5 * (3.0 * z * z - 1.0),
                         S15 * x * z, 0.5 * S15 * (x * x - y * y)], axis=-1)
    raise ValueError(f"l={l} > {LMAX_SUPPORTED} not supported")


def real_sh_grad(l: int, rhat: np.ndarray) -> np.ndarray:
    """Gradient of the polynomial extension of Y_l at rhat: [..., 2l+1, 3].

    Only its component tangent to the sphere matters; callers project it with
    (I - rhat rhat^T)/d.
    """
    x, y, z = rhat[..., 0], rhat[..., 1], rhat[..., 2]
    zero = np.zeros_like(x)
    if l == 0:
        return np.zeros(rhat.shape[:-1] + (1, 3))
    if l == 1:
        g = np.zeros(rhat.shape[:-1] + (3, 3))
        g[..., 0, 0] = g[..., 1, 1] = g[..., 2, 2] = S3
        return g
    if l == 2:
        rows = [
            (S15 * y, S15 * x, zero),
            (zero, S15 * z, S15 * y),
            (zero, zero, 3.0 * S5 * z),
            (S15 * z, zero, S15 * x),
            (S15 * x, -S15 * y, zero),
        ]
        return np.stack([np.stack(r, axis=-1) for r in rows], axis=-2)
    raise ValueError(f"l={l} > {LMAX_SUPPORTED} not supported")


def tp_paths(lmax: int):
    """Coupling paths (l1, l2, l3) in lexicographic order."""
    out = []
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for l3 in range(lmax + 1):
                if abs(l1 - l2) <= l3 <= l1 + l2 and (l1 + l2 + l3) % 2 == 0:
                    out.append((l1, l2, l3))
    return out


def _sphere_rule(n_z: int = 8, n_phi: int = 16):
    """Product quadrature on the unit sphere; weights sum to 1 (mean over sphere)."""
    zs, wz = np.polynomial.legendre.leggauss(n_z)
    phis = 2.0 * math.pi * np.arange(n_phi) / n_phi
    Z, P = np.meshgrid(zs, phis, indexing="ij")
    s = np.sqrt(1.0 - Z * Z)
    pts = np.stack([s * np.cos(P), s * np.sin(P), Z], axis=-1).reshape(-1, 3)
    w = (wz[:, None] * np.ones(n_phi)[None, :] / (2.0 * n_phi)).reshape(-1)
    return pts, w


def gaunt(l1: int, l2: int, l3: int) -> np.ndarray:
    """Real Gaunt tensor (1/4pi) * int Y_l1 Y_l2 Y_l3 dOmega, shape [2l1+1, 2l2+1, 2l3+1]."""
    pts, w = _sphere_rule()
    a, b, c = real_sh(l1, pts), real_sh(l2, pts), real_sh(l3, pts)
    return np.einsum("q,qa,qb,qc->abc", w, a, b, c)


def clebsch_gordan(l1: int, l2: int, l3: int, tol: float = 1e-12) -> np.ndarray:
    """Unit-Frobenius-norm coupling tensor with the canonical sign."""
    g = gaunt(l1, l2, l3)
    g[np.abs(g) < tol] = 0.0
    nrm = math.sqrt(float((g * g).sum()))
    if nrm == 0.0:
        raise ValueError(f"path {(l1, l2, l3)} vanishes")
    g = g / nrm
    first = g.reshape(-1)[np.flatnonzero(g.reshape(-1))[0]]
    return g if first > 0 else -g
