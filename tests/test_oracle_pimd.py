"""Pins of the ring-polymer coupling oracle (CPU): closed forms, finite
differences and invariances that a dropped term, a wrong sign or a missing
minimum image would break."""
import numpy as np

import oracle
from oracle.pimd import EV_PER_AMU_A2FS2


def _beads(P, n, seed, box=12.0, spread=0.3):
    rng = np.random.default_rng(seed)
    centre = rng.uniform(0, box, size=(n, 3))
    return (centre[None] + rng.normal(scale=spread, size=(P, n, 3))) % box, rng.uniform(1.0, 16.0, size=n)


def test_two_beads_closed_form():
    # P = 2: two bonds between the same pair, E = m w^2 |d|^2, F_0 = m w^2 d
    pos = np.array([[[1.0, 2.0, 3.0]], [[1.3, 1.6, 3.2]]])
    m, T, box = np.array([14.007]), 300.0, 20.0
    E, F = oracle.ring_polymer(pos, m, box, T)
    w = 2 * 8.617333262e-5 * T / 0.6582119569
    d = pos[1, 0] - pos[0, 0]
    k = 14.007 * w * w * EV_PER_AMU_A2FS2
    assert np.isclose(E, k * d @ d, rtol=1e-14)
    np.testing.assert_allclose(F[0, 0], 2 * k * d, rtol=1e-14)
    np.testing.assert_allclose(F[1, 0], -F[0, 0], rtol=1e-14)


def test_single_bead_is_free():
    pos, m = _beads(1, 5, 0)
    E, F = oracle.ring_polymer(pos, m, 12.0, 300.0)
    assert E == 0.0 and not F.any()


def test_forces_are_minus_gradient():
    pos, m = _beads(4, 3, 1)
    E, F = oracle.ring_polymer(pos, m, 12.0, 250.0)
    h = 1e-6
    for k, a, c in [(0, 0, 0), (1, 2, 1), (3, 1, 2), (2, 0, 2)]:
        pp, pm = pos.copy(), pos.copy()
        pp[k, a, c] += h
        pm[k, a, c] -= h
        fd = -(oracle.ring_polymer(pp, m, 12.0, 250.0)[0] - oracle.ring_polymer(pm, m, 12.0, 250.0)[0]) / (2 * h)
        assert abs(fd - F[k, a, c]) <= 1e-6 * max(1.0, abs(F[k, a, c]))


def test_invariances_and_minimum_image():
    pos, m = _beads(6, 4, 2)
    E, F = oracle.ring_polymer(pos, m, 12.0, 300.0)
    # each atom's ring exerts no net force
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-12 * np.abs(F).max())
    # rigid translation, also across the periodic boundary
    E2, F2 = oracle.ring_polymer((pos + np.array([5.7, -3.1, 11.9])) % 12.0, m, 12.0, 300.0)
    assert np.isclose(E2, E, rtol=1e-12)
    np.testing.assert_allclose(F2, F, rtol=1e-9, atol=1e-12)
    # a bead moved by a box vector is the same configuration
    shifted = pos.copy()
    shifted[3, 1, 0] += 12.0
    assert np.isclose(oracle.ring_polymer(shifted, m, 12.0, 300.0)[0], E, rtol=1e-12)


def test_scaling_with_temperature_and_beads():
    pos, m = _beads(4, 3, 3)
    E1, _ = oracle.ring_polymer(pos, m, 12.0, 100.0)
    E2, _ = oracle.ring_polymer(pos, m, 12.0, 200.0)
    assert np.isclose(E2, 4 * E1, rtol=1e-13)  # w_P^2 ~ T^2
