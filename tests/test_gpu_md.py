"""Velocity-Verlet MD step (Eq. 1) through nq_step, replayed from a HIP graph.

Checked against the oracle's FP64 velocity-Verlet driven by oracle forces for
the first steps (trajectories are chaotic, so only a short window is
comparable), for bitwise replay from the same state, for on-device neighbour
list rebuilds when atoms have moved more than half the skin, and for energy
conservation over a short NVE run.
"""
import numpy as np
import pytest
import torch

import oracle
from synth.nh3 import masses, maxwell_boltzmann
from tests.gpu_common import system

pytestmark = pytest.mark.gpu


def _state(pos, z, T=300.0, seed=200):
    v = maxwell_boltzmann(z, T, seed)
    m = masses(z)
    dev = "cuda"
    return (torch.tensor(pos, device=dev), torch.tensor(v, device=dev),
            torch.tensor(1.0 / m, device=dev), torch.tensor(z, dtype=torch.int32, device=dev), m, v)


def _run(pot, pos, z, L, dt, n, T=300.0):
    P, V, IM, Z, m, v0 = _state(pos, z, T)
    E, F = pot.energy_forces(P, Z, L)
    ep = torch.zeros(n, dtype=torch.float64, device="cuda")
    ek = torch.zeros(n, dtype=torch.float64, device="cuda")
    pot.step(P, V, IM, Z, L, dt, n, F, ep, ek)
    torch.cuda.synchronize()
    return P.cpu().numpy(), V.cpu().numpy(), ep.cpu().numpy(), ek.cpu().numpy(), E.item(), F.cpu().numpy()


def test_matches_oracle_velocity_verlet():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = Potential(cf.model, w, "fp32")
    n, dt = 20, 0.5
    P, V, ep, ek, _, _ = _run(pot, pos, z, L, dt, n)
    v0 = maxwell_boltzmann(z, 300.0, 200)
    rp, rv, rep, rek = oracle.velocity_verlet(pos, v0, masses(z), L, n, dt,
                                              lambda p: oracle.energy_forces(p, z, L, cf.model, w))
    d = P - rp
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-7
    assert np.abs(V - rv).max() < 1e-8
    np.testing.assert_allclose(ep, rep, rtol=1e-5)
    np.testing.assert_allclose(ek, rek, rtol=1e-6)
    pot.close()


def test_bitwise_replay_and_rebuilds():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = Potential(cf.model, w, "fp32")
    a = _run(pot, pos, z, L, 0.5, 60)
    _, rebuilds_a = pot.stats()
    b = _run(pot, pos, z, L, 0.5, 60)
    _, rebuilds_b = pot.stats()
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    assert rebuilds_b > rebuilds_a > 0  # atoms moved more than half the skin
    pot.close()


def test_short_nve_conserves_energy():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_1024_l2")
    pot = Potential(cf.model, w, "bf16x3")
    n = 40
    _, _, ep, ek, e0, _ = _run(pot, pos, z, L, 0.5, n)
    etot = ep + ek
    # per-atom drift far below the kinetic energy per atom (~0.04 eV)
    assert np.abs(etot - etot[0]).max() / len(pos) < 1e-5
    assert np.all(np.isfinite(etot))
    pot.close()
