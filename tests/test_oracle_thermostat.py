"""Pins of the Nose-Hoover oracle (CPU) on an anharmonic toy potential with a
known exact force: the extended energy is conserved, an infinitely heavy
thermostat reproduces plain velocity Verlet, the thermostat pulls the kinetic
temperature toward its target, and the scheme is time reversible."""
import numpy as np

import oracle
from oracle.md import KB_EV


def _toy(n=24, seed=0, L=30.0, spread=0.3):
    rng = np.random.default_rng(seed)
    anchor = rng.uniform(5, 25, size=(n, 3))
    pos0 = anchor + rng.normal(scale=spread, size=(n, 3))
    m = rng.uniform(1.0, 14.0, size=n)

    def force(p):
        d = p - anchor
        r2 = (d * d).sum(1)
        E = float((0.5 * r2 + 0.25 * r2 * r2).sum())  # eV, A
        F = -(d * (1.0 + r2)[:, None])
        return E, F

    return pos0, m, L, force


def _v(m, T, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(len(m), 3)) * np.sqrt(KB_EV * T / (m * oracle.md.EV_PER_AMU_A2FS2))[:, None]
    return v - (m[:, None] * v).sum(0) / m.sum()


def test_extended_energy_is_conserved():
    pos, m, L, f = _toy()
    v = _v(m, 500.0, 1)
    _, _, ep, ek, eth, _, _ = oracle.nose_hoover(pos, v, m, L, 400, 0.5, f, 300.0, 20.0)
    h = ep + ek + eth
    # bounded velocity-Verlet fluctuation (dt^2 error), no drift
    assert np.abs(h - h[0]).max() < 2e-3 * np.abs(ek).mean()
    assert abs(h[-100:].mean() - h[:100].mean()) < 5e-4 * np.abs(ek).mean()
    # the thermostat did work (the test is not trivially passing)
    assert np.abs(eth).max() > 1e-2 * np.abs(ek).mean()


def test_heavy_thermostat_is_velocity_verlet():
    pos, m, L, f = _toy()
    v = _v(m, 300.0, 2)
    a = oracle.nose_hoover(pos, v, m, L, 50, 0.5, f, 300.0, 1e9)
    b = oracle.velocity_verlet(pos, v, m, L, 50, 0.5, f)
    np.testing.assert_allclose(a[0], b[0], atol=1e-9)
    np.testing.assert_allclose(a[3], b[3], rtol=1e-8)


def test_temperature_is_pulled_toward_target():
    pos, m, L, f = _toy(n=48, seed=3, spread=0.0)
    v = _v(m, 50.0, 4)
    nf = 3 * len(m) - 3
    _, _, _, ek, _, _, _ = oracle.nose_hoover(pos, v, m, L, 2000, 0.5, f, 400.0, 10.0)
    T = 2 * ek / (nf * KB_EV)
    assert T[0] < 100.0  # starts cold (at the potential minimum, 50 K)
    assert abs(T[1000:].mean() - 400.0) < 40.0  # ends near the target on average


def test_time_reversible():
    pos, m, L, f = _toy()
    v = _v(m, 300.0, 5)
    p1, v1, _, _, _, xi, eta = oracle.nose_hoover(pos, v, m, L, 100, 0.5, f, 300.0, 20.0)
    p2, v2, _, _, _, xi2, _ = oracle.nose_hoover(p1, -v1, m, L, 100, 0.5, f, 300.0, 20.0, xi=-xi, eta=eta)
    np.testing.assert_allclose(p2, pos, atol=1e-8)
    np.testing.assert_allclose(-v2, v, atol=1e-8)
