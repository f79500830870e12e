"""Pins of the oracle's spherical harmonics and coupling tables (CPU).

Each check is fixed by mathematics, not by the oracle itself: the addition
theorem against scipy's Legendre polynomials, orthonormality under a quadrature
in theta (the oracle's own tables use a rule in z = cos theta), parity,
orthogonal representation matrices under rotation, Schur orthogonality and the
closed forms of the (l,0,l), (0,l,l) and (l,l,0) couplings.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre

from oracle.sh import clebsch_gordan, real_sh, real_sh_grad, tp_paths
from synth.nh3 import random_rotation


def _unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _theta_rule(n=40):
    t, wt = np.polynomial.legendre.leggauss(n)
    theta = 0.5 * math.pi * (t + 1.0)
    wth = 0.5 * math.pi * wt * np.sin(theta)
    phi = 2 * math.pi * np.arange(2 * n) / (2 * n)
    TH, PH = np.meshgrid(theta, phi, indexing="ij")
    pts = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1).reshape(-1, 3)
    w = (wth[:, None] * np.full(2 * n, 2 * math.pi / (2 * n))[None, :]).reshape(-1) / (4 * math.pi)
    return pts, w


@pytest.mark.parametrize("l", [0, 1, 2])
def test_addition_theorem(l):
    rng = np.random.default_rng(1)
    a, b = _unit(rng, 200), _unit(rng, 200)
    lhs = (real_sh(l, a) * real_sh(l, b)).sum(1)
    rhs = (2 * l + 1) * eval_legendre(l, (a * b).sum(1))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_component_normalisation_and_orthonormality():
    rng = np.random.default_rng(2)
    r = _unit(rng, 100)
    for l in range(3):
        np.testing.assert_allclose((real_sh(l, r) ** 2).sum(1), 2 * l + 1, atol=1e-13)
    pts, w = _theta_rule()
    Y = np.concatenate([real_sh(l, pts) for l in range(3)], axis=1)
    gram = np.einsum("q,qa,qb->ab", w, Y, Y)
    np.testing.assert_allclose(gram, np.eye(9), atol=1e-13)


def test_parity():
    rng = np.random.default_rng(3)
    r = _unit(rng, 50)
    for l in range(3):
        np.testing.assert_allclose(real_sh(l, -r), (-1) ** l * real_sh(l, r), atol=1e-14)


def _wigner(l, R, rng):
    r = _unit(rng, 64)
    A, B = real_sh(l, r), real_sh(l, r @ R.T)
    D, res, *_ = np.linalg.lstsq(A, B, rcond=None)
    assert np.abs(A @ D - B).max() < 1e-12
    return D.T  # Y(R r) = D Y(r)


def test_rotation_representation_is_orthogonal():
    rng = np.random.default_rng(4)
    for s in range(3):
        R = random_rotation(40 + s)
        for l in range(3):
            D = _wigner(l, R, rng)
            np.testing.assert_allclose(D @ D.T, np.eye(2 * l + 1), atol=1e-12)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    r = rng.standard_normal((20, 3)) * 2.0
    h = 1e-6
    for l in range(3):
        d = np.linalg.norm(r, axis=1)
        rh = r / d[:, None]
        G = real_sh_grad(l, rh)
        P = (np.eye(3)[None] - rh[:, :, None] * rh[:, None, :]) / d[:, None, None]
        analytic = np.einsum("emk,ekj->emj", G, P)
        for j in range(3):
            dp, dm = r.copy(), r.copy()
            dp[:, j] += h
            dm[:, j] -= h
            fd = (real_sh(l, dp / np.linalg.norm(dp, axis=1, keepdims=True))
                  - real_sh(l, dm / np.linalg.norm(dm, axis=1, keepdims=True))) / (2 * h)
            np.testing.assert_allclose(analytic[:, :, j], fd, atol=1e-8)


def test_path_enumeration():
    assert tp_paths(1) == [(0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 0)]
    assert len(tp_paths(2)) == 11
    nnz = sum(int((np.abs(clebsch_gordan(*p)) > 1e-12).sum()) for p in tp_paths(2))
    assert nnz == 83


def test_cg_equivariance_under_rotations():
    rng = np.random.default_rng(6)
    R = random_rotation(77)
    D = [_wigner(l, R, rng) for l in range(3)]
    for (l1, l2, l3) in tp_paths(2):
        C = clebsch_gordan(l1, l2, l3)
        rot = np.einsum("abk,ax,by,kz->xyz", C, D[l1], D[l2], D[l3])
        np.testing.assert_allclose(rot, C, atol=1e-12)


def test_cg_schur_orthogonality_and_sign():
    for (l1, l2, l3) in tp_paths(2):
        C = clebsch_gordan(l1, l2, l3)
        M = np.einsum("abk,abq->kq", C, C)
        np.testing.assert_allclose(M, np.eye(2 * l3 + 1) / (2 * l3 + 1), atol=1e-13)
        flat = C.reshape(-1)
        assert flat[np.flatnonzero(np.abs(flat) > 1e-12)[0]] > 0


def test_cg_closed_forms():
    for l in range(3):
        eye = np.eye(2 * l + 1) / math.sqrt(2 * l + 1)
        np.testing.assert_allclose(clebsch_gordan(l, 0, l)[:, 0, :], eye, atol=1e-14)
        np.testing.assert_allclose(clebsch_gordan(0, l, l)[0, :, :], eye, atol=1e-14)
        np.testing.assert_allclose(clebsch_gordan(l, l, 0)[:, :, 0], eye, atol=1e-14)


def test_cg_matches_theta_quadrature():
    """Same Gaunt integrals under an unrelated quadrature rule (theta, not cos theta)."""
    pts, w = _theta_rule()
    for (l1, l2, l3) in tp_paths(2):
        g = np.einsum("q,qa,qb,qc->abc", w, real_sh(l1, pts), real_sh(l2, pts), real_sh(l3, pts))
        g /= np.linalg.norm(g)
        C = clebsch_gordan(l1, l2, l3)
        sign = np.sign((g * C).sum())
        np.testing.assert_allclose(sign * g, C, atol=1e-12)
