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


def _run_nvt(pot, pos, z, L, dt, n, T_target, tau, T0=300.0):
    P, V, IM, Z, m, v0 = _state(pos, z, T0)
    E, F = pot.energy_forces(P, Z, L)
    th = torch.zeros(2, dtype=torch.float64, device="cuda")
    ep = torch.zeros(n, dtype=torch.float64, device="cuda")
    ek = torch.zeros(n, dtype=torch.float64, device="cuda")
    et = torch.zeros(n, dtype=torch.float64, device="cuda")
    pot.step_nvt(P, V, IM, Z, L, dt, n, T_target, tau, th, F, ep, ek, et)
    torch.cuda.synchronize()
    return (P.cpu().numpy(), V.cpu().numpy(), ep.cpu().numpy(), ek.cpu().numpy(), et.cpu().numpy(),
            th.cpu().numpy())


def test_nvt_matches_oracle_nose_hoover():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = Potential(cf.model, w, "fp32")
    n, dt, T, tau = 20, 0.5, 200.0, 20.0
    P, V, ep, ek, et, th = _run_nvt(pot, pos, z, L, dt, n, T, tau)
    v0 = maxwell_boltzmann(z, 300.0, 200)
    rp, rv, rep, rek, ret, xi, eta = oracle.nose_hoover(pos, v0, masses(z), L, n, dt,
                                                        lambda p: oracle.energy_forces(p, z, L, cf.model, w), T, tau)
    d = P - rp
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-7
    assert np.abs(V - rv).max() < 1e-8
    np.testing.assert_allclose(ek, rek, rtol=1e-6)
    np.testing.assert_allclose(et, ret, rtol=1e-6, atol=1e-9)
    assert abs(th[0] - xi) <= 1e-6 * abs(xi) and abs(th[1] - eta) <= 1e-6 * abs(eta)
    pot.close()


def test_nvt_extended_energy_conserved():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = Potential(cf.model, w, "fp32")
    P, V, ep, ek, et, th = _run_nvt(pot, pos, z, L, 0.25, 200, 200.0, 10.0)
    h = ep + ek + et
    assert np.abs(et).max() > 0.05 * ek.mean()  # the thermostat does work
    assert np.abs(h - h[0]).max() < 2e-3 * ek.mean()
    pot.close()


def test_force_outliers_by_injection():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = Potential(cf.model, w, "fp32")
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    _, F = pot.energy_forces(P, Z, L)
    torch.cuda.synchronize()

    f = F.cpu().numpy()
    assert pot.force_outliers(F, 5.0).item() == oracle.force_outliers(f, 5.0)
    assert pot.force_outliers(F, 1.0).item() == oracle.force_outliers(f, 1.0)
    G = F.clone()
    G[3, 1] = 50.0 * float(np.abs(f).max())
    G[17, 2] = -50.0 * float(np.abs(f).max())
    g = G.cpu().numpy()
    got = pot.force_outliers(G, 5.0).item()
    assert got == oracle.force_outliers(g, 5.0) and got >= 2
    # the constructed arrays of the oracle's pins: 11 of 300 components at a > 0 are
    # outliers, 12 are not
    for k, expected in ((11, 11), (12, 0)):
        H = torch.zeros(100, 3, dtype=torch.float64, device="cuda")
        H.view(-1)[:k] = 2.5
        assert pot.force_outliers(H, 5.0).item() == expected == oracle.force_outliers(H.cpu().numpy(), 5.0)
    pot.close()


def test_graph_recaptured_after_list_change():
    """A captured MD step bakes in the neighbour list's buffers, row capacity
    and list margin: rebuilding the list with another margin between two
    nq_step calls must capture the graph again, and the continued run must be
    bitwise the run of a fresh context that starts from the same state."""
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = Potential(cf.model, w, "fp32")
    P, V, IM, Z, m, _ = _state(pos, z)
    E, F = pot.energy_forces(P, Z, L)
    pot.step(P, V, IM, Z, L, 0.5, 5, F)
    torch.cuda.synchronize()
    assert pot.graph_captures() == 1
    P1, V1, F1 = P.clone(), V.clone(), F.clone()
    pot.neighbor_build(P, L, skin=0.2)
    pot.step(P, V, IM, Z, L, 0.5, 10, F)
    torch.cuda.synchronize()
    assert pot.graph_captures() == 2
    fresh = Potential(cf.model, w, "fp32")
    fresh.neighbor_build(P1, L, skin=0.2)
    fresh.step(P1, V1, IM, Z, L, 0.5, 10, F1)
    torch.cuda.synchronize()
    assert torch.equal(P, P1) and torch.equal(V, V1) and torch.equal(F, F1)
    # same pointers, step count and list: replayed, not captured again
    pot.step(P, V, IM, Z, L, 0.5, 10, F)
    torch.cuda.synchronize()
    assert pot.graph_captures() == 2
    pot.close()
    fresh.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_300K_run_collapses_like_the_oracle(prec):
    """NVE at 300 K on the 1,024-atom system, one step per call, against the
    FP64 oracle's own trajectory (tests/golden/c3_oracle_nve.json, written by
    c3_oracle_nve.py): with random weights the surface has no repulsive core,
    so both trajectories heat up as atoms fall together until a pair is closer
    than 0.1 A, where the library stops with NQ_ERR_NUMERIC. The kinetic
    energies agree step by step while the trajectories are close, and the
    library stops within a few steps of the oracle's collapse."""
    import json
    import os

    from paper_2303_08169_amd.binding import NQError
    from paper_2303_08169_amd.potential import Potential
    with open(os.path.join(os.path.dirname(__file__), "golden", "c3_oracle_nve.json")) as f:
        g = json.load(f)
    cf, pos, z, L, w = system("nh3_1024_l2")
    assert g["workload"] == "nh3_1024_l2" and g["velocity_seed"] == 200 and g["dt_fs"] == 0.5
    pot = Potential(cf.model, w, prec)
    P, V, IM, Z, m, v0 = _state(pos, z, g["temperature_K"], g["velocity_seed"])
    E, F = pot.energy_forces(P, Z, L)
    assert abs(E.item() - g["epot0"]) <= 1e-5 * abs(g["epot0"])
    ep = torch.zeros(1, dtype=torch.float64, device="cuda")
    ek = torch.zeros(1, dtype=torch.float64, device="cuda")
    stop, ekin = None, []
    for s in range(1, g["collapsed_at_step"] + 20):
        try:
            pot.step(P, V, IM, Z, L, g["dt_fs"], 1, F, ep, ek)
            torch.cuda.synchronize()
        except NQError as e:
            assert e.status == -4, str(e)  # NQ_ERR_NUMERIC: two atoms closer than 0.1 A
            stop = s
            break
        ekin.append(ek.item())
    pot.close()
    print(f"{prec}: stopped at step {stop}, oracle at {g['collapsed_at_step']}", flush=True)
    ref = np.array([st["ekin"] for st in g["steps"]])
    # the first 50 steps (25 fs): the trajectories have not separated yet
    np.testing.assert_allclose(ekin[:50], ref[:50], rtol=1e-3)
    assert stop is not None and abs(stop - g["collapsed_at_step"]) <= 5
