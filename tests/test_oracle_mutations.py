"""The oracle's pins catch plausible mistakes.

Each test plants one mistake in the oracle (CPU only, through monkeypatch) and
checks that one of the pins used in test_oracle_*.py now fails: a dropped term
in the reverse pass, a wrong sign, a perturbed coupling coefficient, a wrong
spherical-harmonic component, an index mix-up in the channel mixing.
"""
import numpy as np
import pytest

import oracle
import oracle.model as om
from synth import config, make_system, weight_blob
from synth.nh3 import random_rotation

MAIN = config("nh3_1024_l2").model


def _weights(desc):
    return weight_blob(0, [(a, b) for _, a, b in oracle.weight_segments(desc)])


def _cluster():
    pos, z, L = make_system(64, 5)
    d = pos - pos[0]
    d -= L * np.round(d / L)
    mol = np.argsort(np.linalg.norm(d[::4], axis=1))[:3]
    idx = (mol[:, None] * 4 + np.arange(4)[None, :]).reshape(-1)
    return d[idx] + 20.0, z[idx], 40.0


def _fd_ok(h=1e-4):
    pos, z, box = _cluster()
    w = _weights(MAIN)
    _, F = oracle.energy_forces(pos, z, box, MAIN, w)
    for a in (0, 5):
        for k in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[a, k] += h
            pm[a, k] -= h
            fd = -(oracle.energy_forces(pp, z, box, MAIN, w, forces=False)[0]
                   - oracle.energy_forces(pm, z, box, MAIN, w, forces=False)[0]) / (2 * h)
            if abs(fd - F[a, k]) > 1e-6 * max(1.0, np.abs(F).max()):
                return False
    return True


def _invariant_ok():
    pos, z, box = _cluster()
    w = _weights(MAIN)
    E0, _ = oracle.energy_forces(pos, z, box, MAIN, w, forces=False)
    R = random_rotation(401)
    ctr = pos.mean(0)
    E1, _ = oracle.energy_forces((pos - ctr) @ R.T + ctr, z, box, MAIN, w, forces=False)
    return abs(E1 - E0) < 1e-12 * abs(E0)


def test_unmutated_oracle_passes_both_pins():
    assert _fd_ok() and _invariant_ok()


def test_dropped_environment_term_in_reverse_pass(monkeypatch):
    monkeypatch.setattr(om, "_tp_grad_g", lambda C, V, gT: np.zeros(V.shape[:2] + (C.shape[1],)))
    assert not _fd_ok()


def test_wrong_sign_of_cutoff_derivative(monkeypatch):
    real = om.envelope
    monkeypatch.setattr(om, "envelope", lambda x, p: (real(x, p)[0], -real(x, p)[1]))
    assert not _fd_ok()


def test_wrong_harmonic_gradient(monkeypatch):
    real = om.real_sh_grad
    monkeypatch.setattr(om, "real_sh_grad", lambda l, r: real(l, r) * (1.1 if l == 2 else 1.0))
    assert not _fd_ok()


def test_perturbed_coupling_coefficient(monkeypatch):
    real = om.clebsch_gordan

    def bad(l1, l2, l3):
        C = real(l1, l2, l3).copy()
        if (l1, l2, l3) == (1, 1, 2):
            C[0, 1, 0] *= 1.05
        return C
    monkeypatch.setattr(om, "clebsch_gordan", bad)
    assert not _invariant_ok()


def test_wrong_spherical_harmonic_component(monkeypatch):
    real = om.real_sh

    def bad(l, r):
        Y = real(l, r)
        if l == 2:
            Y = Y.copy()
            Y[..., 2] += 0.2  # a constant added to the (3z^2-1) component
        return Y
    monkeypatch.setattr(om, "real_sh", bad)
    assert not _invariant_ok()


def test_transposed_mixing_block(monkeypatch):
    real = om.unpack_weights

    def bad(desc, blob):
        W = real(desc, blob)
        # mix up (path, channel) rows of one mixing block: rows reordered path-major -> channel-major
        key = "layer1.mix.1"
        P, C = W[key].shape[0] // desc.channels, desc.channels
        W[key] = W[key].reshape(P, C, C).transpose(1, 0, 2).reshape(P * C, C)
        return W
    pos, z, box = _cluster()
    w = _weights(MAIN)
    E_ok, _ = oracle.energy_forces(pos, z, box, MAIN, w, forces=False)
    monkeypatch.setattr(om, "unpack_weights", bad)
    E_bad, _ = oracle.energy_forces(pos, z, box, MAIN, w, forces=False)
    # the GPU parity tests compare against these values: a layout mix-up changes E
    assert abs(E_bad - E_ok) > 1e-6 * abs(E_ok)
