"""Velocity-Verlet integration of Newton's equations in FP64 (test oracle).

Integrates m_i d^2 r_i/dt^2 = f_i = -dE/dr_i (Sec. 2.1, Eq. 1) with the
velocity-Verlet scheme: v += dt/2 f/m; r += dt v (wrapped into the box);
f = F(r); v += dt/2 f/m. Units: A, fs, amu, eV; 1 eV/(amu A) = 9.648533212e-3 A/fs^2.
"""
from __future__ import annotations

import numpy as np

ACC = 9.648533212e-3  # A/fs^2 per eV/(amu A)
EV_PER_AMU_A2FS2 = 1.0 / ACC


def velocity_verlet(pos, vel, masses, box, n_steps, dt, force_fn):
    """force_fn(pos) -> (E, F). Returns (pos, vel, epot[n], ekin[n]) after each step."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    _, F = force_fn(pos)
    epot, ekin = np.zeros(n_steps), np.zeros(n_steps)
    for s in range(n_steps):
        vel += 0.5 * dt * ACC * F / m
        pos += dt * vel
        pos -= box * np.floor(pos / box)
        E, F = force_fn(pos)
        vel += 0.5 * dt * ACC * F / m
        epot[s] = E
        ekin[s] = 0.5 * float((m * vel * vel).sum()) * EV_PER_AMU_A2FS2
    return pos, vel, epot, ekin
