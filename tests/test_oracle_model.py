"""Pins of the oracle's energy and forces (CPU).

Energy: invariance under proper rotations of an isolated cluster, under
inversion, translation (with wrapping) and permutation of a periodic system;
locality (E_i only sees atoms within the cutoff of i); vanishing beyond the
cutoff; the pair-potential special case (environment weights zero -> E is a sum
of dimer energies); the scalar coupling paths against plain dot products.
Forces: central finite differences of the energy (h = 1e-4 A), covariance under
rotation, and zero net force.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle.model import unpack_weights, weight_segments
from synth import config, make_system, weight_blob
from synth.nh3 import random_rotation

SMALL = config("nh3_64_l1").model
MAIN = config("nh3_1024_l2").model


def _weights(desc, seed=0):
    return weight_blob(seed, [(a, b) for _, a, b in weight_segments(desc)])


def _cluster(n_mol=4, seed=5, box=40.0):
    """A few NH3 molecules cut from a periodic sample, centred in a vacuum box."""
    pos, z, L = make_system(64, seed)
    c = pos[0]
    d = pos - c
    d -= L * np.round(d / L)
    mol = np.argsort(np.linalg.norm(d[::4], axis=1))[:n_mol]
    idx = (mol[:, None] * 4 + np.arange(4)[None, :]).reshape(-1)
    return d[idx] + box / 2.0, z[idx], box


@pytest.mark.parametrize("desc", [SMALL, MAIN], ids=["l1", "l2"])
def test_rotation_invariance_and_force_covariance(desc):
    pos, z, box = _cluster()
    w = _weights(desc)
    E0, F0 = oracle.energy_forces(pos, z, box, desc, w)
    assert abs(E0) > 1e-3
    ctr = pos.mean(0)
    for s in range(3):
        R = random_rotation(400 + s)
        p2 = (pos - ctr) @ R.T + ctr
        E1, F1 = oracle.energy_forces(p2, z, box, desc, w)
        assert abs(E1 - E0) < 1e-12 * max(1.0, abs(E0))
        np.testing.assert_allclose(F1, F0 @ R.T, atol=1e-12)


@pytest.mark.parametrize("desc", [SMALL, MAIN], ids=["l1", "l2"])
def test_inversion_translation_permutation(desc):
    cf = config("nh3_64_l1")
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    if desc is MAIN:  # a cutoff of 6 A needs a box wider than 12 A
        pos, z, L = make_system(512, 7)
    w = _weights(desc)
    E0, F0 = oracle.energy_forces(pos, z, L, desc, w)
    E1, F1 = oracle.energy_forces(np.mod(-pos, L), z, L, desc, w)
    assert abs(E1 - E0) < 1e-11 * abs(E0)
    np.testing.assert_allclose(F1, -F0, atol=1e-11)
    shift = np.array([1.3, -7.1, 2.9])
    E2, F2 = oracle.energy_forces(np.mod(pos + shift, L), z, L, desc, w)
    assert abs(E2 - E0) < 1e-11 * abs(E0)
    np.testing.assert_allclose(F2, F0, atol=1e-11)
    perm = np.random.default_rng(8).permutation(len(pos))
    E3, F3 = oracle.energy_forces(pos[perm], z[perm], L, desc, w)
    assert abs(E3 - E0) < 1e-11 * abs(E0)
    np.testing.assert_allclose(F3, F0[perm], atol=1e-11)
    np.testing.assert_allclose(F0.sum(0), 0.0, atol=1e-12 * np.abs(F0).sum())


def _fd_check(pos, z, box, desc, w, atoms, centers=None, h=1e-4):
    _, F = oracle.energy_forces(pos, z, box, desc, w, centers=centers)
    for a in atoms:
        for k in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[a, k] += h
            pm[a, k] -= h
            Ep, _ = oracle.energy_forces(pp, z, box, desc, w, centers=centers, forces=False)
            Em, _ = oracle.energy_forces(pm, z, box, desc, w, centers=centers, forces=False)
            fd = -(Ep - Em) / (2 * h)
            assert abs(fd - F[a, k]) < 1e-6 * max(1.0, np.abs(F).max()), (a, k, fd, F[a, k])


def test_forces_finite_differences_small_periodic():
    cf = config("nh3_64_l1")
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    _fd_check(pos, z, L, cf.model, _weights(cf.model), atoms=range(0, 64, 5))


def test_forces_finite_differences_l2_cluster():
    pos, z, box = _cluster(n_mol=4)
    _fd_check(pos, z, box, MAIN, _weights(MAIN), atoms=range(len(pos)))


def test_forces_finite_differences_l2_periodic_local():
    """On the 1,024-atom system, F_a only needs the centres a and its neighbours."""
    cf = config("nh3_1024_l2")
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    w = _weights(cf.model)
    rng = np.random.default_rng(300)
    for a in rng.choice(len(pos), 2, replace=False):
        ei, ej = oracle.edge_list(pos, L, cf.model.r_cut, centers=[a])
        centers = np.concatenate([[a], ej])
        _fd_check(pos, z, L, cf.model, w, atoms=[a], centers=centers)


def test_locality():
    cf = config("nh3_1024_l2")
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    w = _weights(cf.model)
    a = 17
    d = pos - pos[a]
    d -= L * np.round(d / L)
    dist = np.linalg.norm(d, axis=1)
    near = np.flatnonzero((dist < cf.model.r_cut) & (dist > 0))[:3]
    far = np.flatnonzero(dist > cf.model.r_cut + 0.2)[:3]
    cs = np.concatenate([near, far])
    _, _, e0 = oracle.energy_forces(pos, z, L, cf.model, w, centers=cs, forces=False, atom_energy=True)
    p2 = pos.copy()
    p2[a] += np.array([0.05, -0.03, 0.02])
    _, _, e1 = oracle.energy_forces(p2, z, L, cf.model, w, centers=cs, forces=False, atom_energy=True)
    assert np.all(e1[far] == e0[far])
    assert np.all(np.abs(e1[near] - e0[near]) > 0)


def test_dimer_vanishes_beyond_cutoff_and_is_smooth():
    desc = MAIN
    w = _weights(desc)
    box = 40.0
    z = np.array([1, 0])
    def E(d):
        pos = np.array([[10.0, 10.0, 10.0], [10.0 + d, 10.0, 10.0]])
        return oracle.energy_forces(pos, z, box, desc, w)
    e_out, f_out = E(desc.r_cut + 1e-9)
    assert e_out == 0.0 and np.all(f_out == 0.0)
    e1, _ = E(desc.r_cut - 1e-2)
    e2, _ = E(desc.r_cut - 2e-2)
    # E(d) ~ (r_c - d)^3 near the cutoff (u, u', u'' vanish there)
    assert abs(e1) < 1e-4 and abs(e2 / e1) > 6.0


def test_pair_potential_special_case():
    """With all environment weights zero, E is a sum of dimer energies."""
    desc = MAIN
    W = unpack_weights(desc, _weights(desc))
    for t in range(1, desc.n_layers + 1):
        W[f"layer{t}.env"] = np.zeros_like(W[f"layer{t}.env"])
    pos, z, box = _cluster(n_mol=2)
    E, _ = oracle.energy_forces(pos, z, box, desc, W)
    pair = 0.0
    for i in range(len(pos)):
        for j in range(i + 1, len(pos)):
            pair += oracle.energy_forces(pos[[i, j]], z[[i, j]], box, desc, W, forces=False)[0]
    assert abs(E - pair) < 1e-12 * abs(E)
    # and with the environment switched back on, E is no longer pair-additive
    E_env, _ = oracle.energy_forces(pos, z, box, desc, _weights(desc))
    W2 = unpack_weights(desc, _weights(desc))
    pair2 = sum(oracle.energy_forces(pos[[i, j]], z[[i, j]], box, desc, W2, forces=False)[0]
                for i in range(len(pos)) for j in range(i + 1, len(pos)))
    assert abs(E_env - pair2) > 1e-6


@pytest.mark.parametrize("desc", [SMALL, MAIN], ids=["l1", "l2"])
def test_scalar_paths_are_scaled_dot_products(desc):
    pos, z, box = _cluster(n_mol=3)
    tr = {}
    oracle.energy_forces(pos, z, box, desc, _weights(desc), forces=False, trace=tr)
    L, C = desc.lmax, desc.channels
    Y, w0, gam = tr["Y"], tr["w0"], tr["gamma1"]
    nE = len(tr["ei"])
    # Gamma_i gathered per edge: rows of gamma1 are per centre, reorder to edges
    centers = np.unique(tr["ei"])
    G = gam[np.searchsorted(centers, tr["ei"])]
    s = np.zeros((nE, (L + 1) * C))
    goff = 0
    for l in range(L + 1):
        nm = 2 * l + 1
        V = w0[:, l, :, None] * Y[:, l * l:l * l + nm][:, None, :]
        Gl = G[:, goff:goff + C * nm].reshape(nE, C, nm)
        s[:, l * C:(l + 1) * C] = (V * Gl).sum(2) / math.sqrt(nm)
        goff += C * nm
    np.testing.assert_allclose(tr["s1"], s, atol=1e-13)


def test_energy_scale_is_linear():
    cf = config("nh3_64_l1")
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    w = _weights(cf.model)
    E1, F1 = oracle.energy_forces(pos, z, L, cf.model, w)
    E2, F2 = oracle.energy_forces(pos, z, L, replace(cf.model, energy_scale=2.5), w)
    assert abs(E2 - 2.5 * E1) < 1e-12 * abs(E2)
    np.testing.assert_allclose(F2, 2.5 * F1, atol=1e-13)
