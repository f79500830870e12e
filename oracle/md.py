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


KB_EV = 8.617333262e-5  # eV / K


def nose_hoover(pos, vel, masses, box, n_steps, dt, force_fn, temperature, tau, xi=0.0, eta=0.0):
    """Velocity Verlet with one Nose-Hoover thermostat (constant-temperature
    runs of the robustness protocol, paper Sec. 3.2). The paper names the
    thermostat only; this is the standard single-thermostat scheme with mass
    Q = N_f k_B T tau^2 (N_f = 3N - 3) and a symmetric splitting: a thermostat
    half step, the velocity-Verlet step, a thermostat half step. Thermostat
    half step of length h = dt/2, with G(K) = (2K - N_f k_B T) / Q:
        xi += G(K) h/2;  v *= exp(-xi h);  K *= exp(-2 xi h);  eta += xi h;  xi += G(K) h/2.
    The extended energy K + E + Q xi^2/2 + N_f k_B T eta is conserved.
    Returns (pos, vel, epot[n], ekin[n], ethermo[n], xi, eta) with ethermo the
    thermostat terms Q xi^2/2 + N_f k_B T eta after each step (eV); xi in 1/fs."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    nf = 3 * len(pos) - 3
    kT = KB_EV * temperature
    Q = nf * kT * tau * tau  # eV fs^2

    def kinetic(v):
        return 0.5 * float((m * v * v).sum()) * EV_PER_AMU_A2FS2

    def thermostat_half(v, K, xi, eta):
        h = 0.5 * dt
        xi += (2.0 * K - nf * kT) / Q * 0.5 * h
        s = np.exp(-xi * h)
        v = v * s
        K = K * s * s
        eta += xi * h
        xi += (2.0 * K - nf * kT) / Q * 0.5 * h
        return v, K, xi, eta

    _, F = force_fn(pos)
    K = kinetic(vel)
    epot, ekin, eth = np.zeros(n_steps), np.zeros(n_steps), np.zeros(n_steps)
    for s in range(n_steps):
        vel, K, xi, eta = thermostat_half(vel, K, xi, eta)
        vel += 0.5 * dt * ACC * F / m
        pos += dt * vel
        pos -= box * np.floor(pos / box)
        E, F = force_fn(pos)
        vel += 0.5 * dt * ACC * F / m
        K = kinetic(vel)
        vel, K, xi, eta = thermostat_half(vel, K, xi, eta)
        epot[s], ekin[s] = E, K
        eth[s] = 0.5 * Q * xi * xi + nf * kT * eta
    return pos, vel, epot, ekin, eth, xi, eta
