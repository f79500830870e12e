"""Seeded liquid-ammonia-shaped configurations (stand-ins for the paper's NH3 systems).

Recipe (the paper's systems are liquid NH3; its data set is not available):
  * M = N/4 molecules in a cubic periodic box of side L = (N/rho)^(1/3),
    rho = 0.0965 atoms/A^3.
  * n = ceil(M^(1/3)) lattice sites per side, spacing a = L/n; M sites are taken
    from a seeded permutation of the n^3 sites.
  * The N atom sits at its site plus uniform jitter in [-0.1a, 0.1a]^3.
  * Three H atoms at 1.01 A from N with H-N-H = 107 degrees (pyramid half-angle
    from the C3 axis: sin^2(theta) = (1 - cos 107deg)/1.5), then a uniformly
    random rotation (Shoemake's quaternion method).
  * Molecules with an intermolecular atom pair closer than 1.0 A are redrawn
    (rotation and jitter) until no such pair is left.
  * Coordinates are wrapped into [0, L). Species: H = 0, N = 1.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

from .configs import DENSITY

NH_BOND = 1.01
HNH_ANGLE_DEG = 107.0
MIN_INTER = 1.0
MASS = {0: 1.008, 1: 14.007, 2: 12.011}
KB_EV = 8.617333262e-5           # eV/K
EV_PER_AMU_A2FS2 = 1.0 / 9.648533212e-3  # 1 amu A^2/fs^2 in eV


def _random_rotations(rng: np.random.Generator, k: int) -> np.ndarray:
    """k uniformly random proper rotations from Shoemake's method."""
    u1, u2, u3 = rng.random(k), rng.random(k), rng.random(k)
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    x, y, z, w = q.T
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def random_rotation(seed: int) -> np.ndarray:
    return _random_rotations(np.random.default_rng(seed), 1)[0]


def _molecule_template() -> np.ndarray:
    """N at the origin, three H on a pyramid around +z (4 x 3, order N,H,H,H)."""
    cos_hnh = math.cos(math.radians(HNH_ANGLE_DEG))
    sin_t = math.sqrt((1.0 - cos_hnh) / 1.5)
    cos_t = math.sqrt(1.0 - sin_t * sin_t)
    out = np.zeros((4, 3))
    for k in range(3):
        phi = 2.0 * math.pi * k / 3.0
        out[k + 1] = NH_BOND * np.array([sin_t * math.cos(phi), sin_t * math.sin(phi), cos_t])
    return out


def make_system(n_atoms: int, seed: int, density: float = DENSITY):
    """Return (pos [N,3] float64 in [0,L), species [N] int32, box L)."""
    if n_atoms % 4:
        raise ValueError("n_atoms must be a multiple of 4 (NH3 molecules)")
    m = n_atoms // 4
    L = (n_atoms / density) ** (1.0 / 3.0)
    n = int(math.ceil(m ** (1.0 / 3.0) - 1e-9))
    a = L / n
    rng = np.random.default_rng(seed)
    sites = rng.permutation(n ** 3)[:m]
    grid = np.stack(np.unravel_index(sites, (n, n, n)), axis=1).astype(np.float64) * a
    tmpl = _molecule_template()

    def draw(idx):
        R = _random_rotations(rng, len(idx))
        jit = rng.uniform(-0.1 * a, 0.1 * a, size=(len(idx), 3))
        return grid[idx, None, :] + jit[:, None, :] + np.einsum("kab,tb->kta", R, tmpl)

    mol = draw(np.arange(m))
    for _ in range(100):
        flat = np.mod(mol.reshape(-1, 3), L)
        tree = cKDTree(flat, boxsize=L)
        pairs = tree.query_pairs(MIN_INTER, output_type="ndarray")
        if len(pairs):
            mi, mj = pairs[:, 0] // 4, pairs[:, 1] // 4
            pairs = pairs[mi != mj]
        if not len(pairs):
            break
        bad = np.unique(np.maximum(pairs[:, 0] // 4, pairs[:, 1] // 4))
        mol[bad] = draw(bad)
    else:
        raise RuntimeError("could not place molecules without close contacts")
    pos = np.mod(mol.reshape(-1, 3), L)
    pos[pos >= L] -= L
    species = np.tile(np.array([1, 0, 0, 0], dtype=np.int32), m)
    return np.ascontiguousarray(pos), species, L


def masses(species: np.ndarray) -> np.ndarray:
    return np.array([MASS[int(s)] for s in range(3)])[species]


def maxwell_boltzmann(species: np.ndarray, temperature: float, seed: int) -> np.ndarray:
    """Velocities in A/fs at `temperature` K, centre-of-mass motion removed and
    rescaled so that the kinetic temperature with 3N-3 degrees of freedom is exact."""
    rng = np.random.default_rng(seed)
    m = masses(species)
    sigma = np.sqrt(KB_EV * temperature / (m * EV_PER_AMU_A2FS2))
    v = rng.standard_normal((len(species), 3)) * sigma[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    ekin = 0.5 * (m[:, None] * v * v).sum() * EV_PER_AMU_A2FS2
    dof = 3 * len(species) - 3
    v *= math.sqrt(0.5 * dof * KB_EV * temperature / ekin)
    return v
