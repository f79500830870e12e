"""Replica-batched evaluation (the path-integral application: many replicas of
one box evaluated together) and the ring-polymer coupling.

Each replica's energy, forces and atom energies from one batched call must be
bitwise those of evaluating that replica alone (only same-replica atoms
interact and every per-replica reduction keeps its order); the ring-polymer
springs are compared with the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import TOL, rel_rms, system

pytestmark = pytest.mark.gpu


def _replicas(pos, L, R, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    return np.stack([(pos + rng.normal(scale=scale, size=pos.shape)) % L for _ in range(R)])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_replicas_match_single_evaluations(prec):
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_1024_l2")
    R = 3
    reps = _replicas(pos, L, R, 17)
    pot = Potential(cf.model, w, prec)
    P = torch.tensor(reps, device="cuda")
    Z = torch.tensor(np.tile(z, (R, 1)), dtype=torch.int32, device="cuda")
    E, F, Ei = pot.energy_forces_replicas(P, Z, L, atom_energy=True)
    torch.cuda.synchronize()
    E, F, Ei = E.clone(), F.clone(), Ei.clone()
    one = Potential(cf.model, w, prec)
    for r in range(R):
        e1, f1, ei1 = one.energy_forces(P[r].contiguous(), Z[r].contiguous(), L, atom_energy=True)
        torch.cuda.synchronize()
        assert E[r].item() == e1.item(), r
        assert torch.equal(F[r], f1), r
        assert torch.equal(Ei[r], ei1), r
    pot.close()
    one.close()


def test_replicas_match_oracle_small():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    R = 4
    reps = _replicas(pos, L, R, 23, scale=0.03)
    pot = Potential(cf.model, w, "fp32")
    E, F = pot.energy_forces_replicas(torch.tensor(reps, device="cuda"),
                                      torch.tensor(np.tile(z, (R, 1)), dtype=torch.int32, device="cuda"), L)
    E, F = E.cpu().numpy(), F.cpu().numpy()
    for r in range(R):
        E0, F0 = oracle.energy_forces(reps[r], z, L, cf.model, w)
        assert abs(E[r] - E0) <= TOL["fp32"]["energy"] * abs(E0)
        assert rel_rms(F[r], F0) <= TOL["fp32"]["force"]
    pot.close()


@pytest.mark.parametrize("R", [1, 2, 32])
def test_ring_polymer_matches_oracle(R):
    from paper_2303_08169_amd.potential import Potential
    from synth.nh3 import masses
    cf, pos, z, L, w = system("nh3_64_l1")
    reps = _replicas(pos, L, R, 31, scale=0.2)
    m = masses(z)
    pot = Potential(cf.model, w, "fp32")
    P = torch.tensor(reps, device="cuda")
    F0 = torch.tensor(np.random.default_rng(5).normal(size=reps.shape), device="cuda")
    F = F0.clone()
    E = pot.ring_polymer(P, torch.tensor(1.0 / m, device="cuda"), L, 250.0, F)
    torch.cuda.synchronize()
    Eo, Fo = oracle.ring_polymer(reps, m, L, 250.0)
    assert abs(E.item() - Eo) <= 1e-12 * max(1.0, abs(Eo))
    np.testing.assert_allclose((F - F0).cpu().numpy(), Fo, rtol=1e-10, atol=1e-10 * max(1.0, np.abs(Fo).max()))
    pot.close()


def test_replica_arguments_rejected():
    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = Potential(cf.model, w, "fp32")
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    F = torch.empty_like(P)
    import ctypes as C
    cell = (C.c_double * 3)(L, L, L)
    st = pot.lib.nq_energy_forces_replicas(pot._ctx, pot._model, C.c_void_p(P.data_ptr()), C.c_void_p(Z.data_ptr()),
                                          len(pos), 0, cell, C.c_void_p(E.data_ptr()), C.c_void_p(F.data_ptr()), None)
    assert B.STATUS[st] == "NQ_ERR_ARG"
    st = pot.lib.nq_ring_polymer(pot._ctx, C.c_void_p(P.data_ptr()), None, len(pos), 1, cell, 300.0,
                                 C.c_void_p(F.data_ptr()), C.c_void_p(E.data_ptr()))
    assert B.STATUS[st] == "NQ_ERR_ARG"
    pot.close()
