"""Ring-polymer (path-integral) coupling of replicas in FP64 (test oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's application runs path-integral MD: every atom is represented by a
number of replicas that are harmonically coupled to each other as a ring
polymer, and the replicas' energies and forces are independent evaluations of
the potential (Sec. 5). The paper prints no coupling formula; this module uses
the standard primitive discretisation, written out directly:

  E_spring = 1/2 sum_a m_a w_P^2 sum_{k=0}^{P-1} |r_{k+1,a} - r_{k,a}|^2,  r_P = r_0,
  w_P = P k_B T / hbar,

with bead separations taken by minimum image, and forces -dE_spring/dr.
Units: A, amu, K, eV; 1 amu A^2/fs^2 = 1 / 9.648533212e-3 eV.
"""
from __future__ import annotations

import numpy as np

KB_EV = 8.617333262e-5        # eV / K
HBAR_EVFS = 0.6582119569      # eV fs
EV_PER_AMU_A2FS2 = 1.0 / 9.648533212e-3


def omega_p(n_beads: int, temperature: float) -> float:
    """Ring-polymer frequency P k_B T / hbar in 1/fs."""
    return n_beads * KB_EV * temperature / HBAR_EVFS


def ring_polymer(pos, masses, box, temperature):
    """pos [P, n, 3] (A), masses [n] (amu), cubic or orthorhombic box, T (K).
    Returns (E_spring in eV, F [P, n, 3] in eV/A)."""
    pos = np.asarray(pos, dtype=np.float64)
    P = pos.shape[0]
    L = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    m = np.asarray(masses, dtype=np.float64)
    kappa = m * omega_p(P, temperature) ** 2 * EV_PER_AMU_A2FS2  # eV / A^2 per atom
    E = 0.0
    F = np.zeros_like(pos)
    for k in range(P):
        nxt = (k + 1) % P
        d = pos[nxt] - pos[k]
        d -= L * np.round(d / L)
        E += 0.5 * float((kappa[:, None] * d * d).sum())
        # the bond (k, k+1) pulls bead k toward k+1 and bead k+1 toward k
        F[k] += kappa[:, None] * d
        F[nxt] -= kappa[:, None] * d
    return E, F
