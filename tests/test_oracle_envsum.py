"""Closed-form pin of the environment sum (and the whole one-layer model) on
three atoms.

The model is the smallest one with an environment sum that carries direction:
l <= 1, one layer, one channel, widths 1, nu = 4 (so nu^-1 and nu^-1/2 differ).
Each atom has exactly two neighbours, so for the edge (i, j) the environment of
centre i is written out term by term,

    Gamma_i = nu^-1/2 (e_ij (x) Y(rhat_ij) + e_ik (x) Y(rhat_ik)),

and the energy is assembled from scalar expressions of the reading of Sec. 2.1
(radial basis and cutoff, two-body MLP, initial features V0 = w0 Y, the two
scalar coupling paths (0,0,0) -> V0_0 Gamma_0 and (1,1,0) -> V0_1 . Gamma_1 / sqrt 3,
latent MLP with residual, edge MLP). The oracle must give the same E to
rounding. Three plausible mistakes in the environment sum are shown to move
this closed form far outside that agreement: nu^-1 for nu^-1/2, leaving out
k = j, and pairing e_ik with Y(rhat_ij) instead of Y(rhat_ik); the first is also
planted in the oracle itself.
"""
import math
import types

import numpy as np
import pytest

import oracle
import oracle.model as om
from synth.configs import ModelDesc

DESC = ModelDesc(n_species=3, n_bessel=2, poly_p=6, lmax=1, n_layers=1, channels=1, twobody=[1], latent=[1],
                 edge=[1], r_cut=4.0, avg_num_neighbors=4.0, energy_scale=1.0)
BOX = 40.0
POS = np.array([[20.0, 20.0, 20.0], [22.1, 20.7, 19.4], [20.5, 22.6, 21.3]])
Z = np.array([1, 0, 2])


def _weights():
    rng = np.random.default_rng(17)
    segs = oracle.weight_segments(DESC)
    blob = np.concatenate([rng.uniform(0.4, 1.3, size=a * b) * rng.choice([-1.0, 1.0], size=a * b)
                           for _, a, b in segs])
    return blob, {name: blob_part for name, blob_part in zip(
        [s[0] for s in segs], np.split(blob, np.cumsum([a * b for _, a, b in segs])[:-1]))}


def _silu(a):
    return a / (1.0 + math.exp(-a))


def closed_form(W, nu_power=-0.5, include_self=True, y_of_own_edge=False):
    """E of the three-atom system from scalar expressions (see the module docstring)."""
    rc, p, nb = DESC.r_cut, DESC.poly_p, DESC.n_bessel
    nu = DESC.avg_num_neighbors

    def edge_geom(i, j):
        r = POS[j] - POS[i]
        d = math.sqrt(float(r @ r))
        x = d / rc
        u = 1 - (p + 1) * (p + 2) / 2 * x ** p + p * (p + 2) * x ** (p + 1) - p * (p + 1) / 2 * x ** (p + 2)
        b = [2 / rc * math.sin(n * math.pi * d / rc) / d * u for n in range(1, nb + 1)]
        return d, r / d, u, b

    def two_body(i, j):
        d, rhat, u, b = edge_geom(i, j)
        h = [1.0 if Z[i] == s else 0.0 for s in range(3)] + [1.0 if Z[j] == s else 0.0 for s in range(3)] + b
        a = sum(h[k] * W["twobody.0"][k] for k in range(8))
        return u * _silu(a), u, rhat

    E = 0.0
    for i in range(3):
        others = [j for j in range(3) if j != i]
        for j in others:
            x0, u, rhat_ij = two_body(i, j)
            w0_0, w0_1 = x0 * W["v0"][0], x0 * W["v0"][1]
            V0_0, V0_1 = w0_0, w0_1 * math.sqrt(3.0) * rhat_ij
            # Gamma_i as the sum over the centre's neighbours k (k = j included)
            G0, G1 = 0.0, np.zeros(3)
            for k in others:
                if k == j and not include_self:
                    continue
                x0k, _, rhat_ik = two_body(i, k)
                e0, e1 = x0k * W["layer1.env"][0], x0k * W["layer1.env"][1]
                Y1 = math.sqrt(3.0) * (rhat_ij if y_of_own_edge else rhat_ik)
                G0 += e0
                G1 = G1 + e1 * Y1
            G0 *= nu ** nu_power
            G1 = G1 * nu ** nu_power
            s0 = V0_0 * G0
            s1 = float(V0_1 @ G1) / math.sqrt(3.0)
            a = x0 * W["layer1.latent.0"][0] + s0 * W["layer1.latent.0"][1] + s1 * W["layer1.latent.0"][2]
            x1 = (x0 + u * _silu(a)) / math.sqrt(2.0)
            E += DESC.energy_scale * _silu(x1 * W["edge.0"][0]) * W["edge.out"][0]
    return E


def test_oracle_matches_closed_form():
    blob, W = _weights()
    E, F = oracle.energy_forces(POS, Z, BOX, DESC, blob)
    E_cf = closed_form(W)
    assert abs(E - E_cf) <= 1e-13 * max(1.0, abs(E_cf))
    assert abs(E_cf) > 1e-3


@pytest.mark.parametrize("mistake", [dict(nu_power=-1.0), dict(include_self=False), dict(y_of_own_edge=True)])
def test_closed_form_separates_each_mistake(mistake):
    """An oracle with one of these mistakes would miss the closed form by far
    more than rounding."""
    blob, W = _weights()
    E, _ = oracle.energy_forces(POS, Z, BOX, DESC, blob)
    E_bad = closed_form(W, **mistake)
    assert abs(E - E_bad) > 1e-4 * abs(E)


def test_planted_nu_power_mistake_fails_the_pin(monkeypatch):
    blob, W = _weights()
    # nu^-1 instead of nu^-1/2: the square root in the oracle's scale made the identity
    monkeypatch.setattr(om, "math", types.SimpleNamespace(sqrt=lambda v: v, fsum=math.fsum))
    E, _ = oracle.energy_forces(POS, Z, BOX, DESC, blob)
    assert abs(E - closed_form(W)) > 1e-4 * abs(E)
    assert abs(E - closed_form(W, nu_power=-1.0)) <= 1e-13 * max(1.0, abs(E))
