"""Pins of the oracle's radial basis and edge list (CPU).

Radial: closed-form values of the polynomial cutoff, the Bessel orthogonality
integral (scipy quadrature) and the d -> 0 limit. Edges: exact set equality
with scipy's periodic k-d tree (a library routine) on tiny random boxes with
atoms near faces and corners.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.spatial import cKDTree

from oracle.neighbors import edge_list
from oracle.radial import bessel, envelope
from synth import config, make_system


@pytest.mark.parametrize("p", [6, 5, 8])
def test_envelope_closed_form(p):
    u, du = envelope(np.array([0.0, 1.0, 1.3]), p)
    assert u[0] == 1.0 and u[1] == 0.0 and u[2] == 0.0
    assert abs(du[1]) < 1e-12 and du[2] == 0.0
    h = 1e-5
    um, _ = envelope(np.array([1.0 - h, 1.0 - 2 * h]), p)
    # second derivative at 1 vanishes: u(1-h) ~ h^3
    assert abs(um[0]) < 1e-10
    x = np.linspace(0.05, 0.95, 19)
    fd = (envelope(x + 1e-6, p)[0] - envelope(x - 1e-6, p)[0]) / 2e-6
    np.testing.assert_allclose(envelope(x, p)[1], fd, atol=1e-7)
    # p = 6 coefficients written out
    if p == 6:
        np.testing.assert_allclose(envelope(x, 6)[0], 1 - 28 * x ** 6 + 48 * x ** 7 - 21 * x ** 8, atol=1e-14)


def test_bessel_orthogonality_and_limit():
    rc, nb = 6.0, 8
    for n in range(nb):
        for m in range(nb):
            val, _ = quad(lambda d: bessel(np.array([d]), rc, nb)[0][0, n]
                          * bessel(np.array([d]), rc, nb)[0][0, m] * d * d, 0.0, rc, limit=200)
            assert abs(val - (2.0 / rc if n == m else 0.0)) < 1e-9
    B, _ = bessel(np.array([1e-7]), rc, nb)
    np.testing.assert_allclose(B[0], 2 * np.arange(1, nb + 1) * math.pi / rc ** 2, rtol=1e-9)
    d = np.linspace(0.3, 5.9, 30)
    fd = (bessel(d + 1e-6, rc, nb)[0] - bessel(d - 1e-6, rc, nb)[0]) / 2e-6
    np.testing.assert_allclose(bessel(d, rc, nb)[1], fd, atol=1e-7)


def _kdtree_edges(pos, L, rc):
    tree = cKDTree(np.mod(pos, L), boxsize=L)
    pairs = tree.query_pairs(rc, output_type="ndarray")
    e = np.concatenate([pairs, pairs[:, ::-1]], axis=0)
    e = e[np.lexsort((e[:, 1], e[:, 0]))]
    return e[:, 0], e[:, 1]


@pytest.mark.parametrize("seed", range(6))
def test_edges_match_periodic_kdtree(seed):
    rng = np.random.default_rng(seed)
    L = rng.uniform(9.0, 14.0)
    n = int(rng.integers(20, 200))
    pos = rng.uniform(0, L, size=(n, 3))
    # crowd some atoms against faces and corners
    k = n // 4
    pos[:k] = rng.choice([0.0, L - 1e-9], size=(k, 3)) + rng.uniform(-0.3, 0.3, size=(k, 3))
    pos = np.mod(pos, L)
    rc = 4.0
    ei, ej = edge_list(pos, L, rc)
    ki, kj = _kdtree_edges(pos, L, rc)
    np.testing.assert_array_equal(ei, ki)
    np.testing.assert_array_equal(ej, kj)


def test_edges_symmetric_and_dense_enough():
    cf = config("nh3_1024_l2")
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    ei, ej = edge_list(pos, L, cf.model.r_cut)
    fwd = set(zip(ei.tolist(), ej.tolist()))
    assert all((j, i) in fwd for i, j in fwd)
    # mean neighbour count close to 4/3 pi rc^3 rho
    assert abs(len(ei) / len(pos) - cf.model.avg_num_neighbors) < 0.05 * cf.model.avg_num_neighbors
