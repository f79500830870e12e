"""Chunked evaluation: centres processed in chunks of consecutive atoms must give
exactly the single-chunk result (every per-edge computation and every per-centre
reduction is independent of the chunking), and the 262,144-atom, three-layer,
64-channel model (which only fits in chunks) must match the oracle on sampled
centres and atoms."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import TOL, assert_forces_close, rel_rms, system

pytestmark = pytest.mark.gpu


def _dev(pos, z):
    return torch.tensor(pos, device="cuda"), torch.tensor(np.asarray(z), dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_chunking_is_exact(prec):
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_1024_l2")
    P, Z = _dev(pos, z)
    one = Potential(cf.model, w, prec)
    E1, F1, A1 = one.energy_forces(P, Z, L, atom_energy=True)
    torch.cuda.synchronize()
    many = Potential(cf.model, w, prec)
    many.set_workspace_budget(256 << 20)  # forces several chunks
    E2, F2, A2 = many.energy_forces(P, Z, L, atom_energy=True)
    torch.cuda.synchronize()
    ne, _ = many.stats()
    assert ne == one.stats()[0]
    assert torch.equal(A1, A2)
    assert torch.equal(F1, F2)
    assert E1.item() == E2.item()
    one.close()
    many.close()


def test_big_model_sampled():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_262144_l2_big")
    pot = Potential(cf.model, w, "bf16x3")
    P, Z = _dev(pos, z)
    E, F, Ei = pot.energy_forces(P, Z, L, atom_energy=True)
    torch.cuda.synchronize()
    ne, _ = pot.stats()
    F, Ei = F.cpu().numpy(), Ei.cpu().numpy()
    rng = np.random.default_rng(11)
    centres = rng.choice(len(pos), 6, replace=False)
    _, _, E0 = oracle.energy_forces(pos, z, L, cf.model, w, centers=centres, forces=False, atom_energy=True)
    assert rel_rms(Ei[centres], E0[centres]) <= 10 * TOL["bf16x3"]["energy"]
    # exact forces on three atoms: every centre within r_c of them contributes
    atoms = centres[:3]
    cs = np.unique(np.concatenate([atoms] + [oracle.edge_list(pos, L, cf.model.r_cut, centers=[a])[1]
                                            for a in atoms]))
    _, F0 = oracle.energy_forces(pos, z, L, cf.model, w, centers=cs)
    assert_forces_close(F[atoms], F0[atoms], TOL["bf16x3"]["force"])
    assert abs(E.item() - Ei.sum()) <= 1e-9 * np.abs(Ei).sum()
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-6 * np.abs(F).sum())
    assert abs(ne / len(pos) - cf.model.avg_num_neighbors) < 0.05 * cf.model.avg_num_neighbors
    pot.close()


def test_autotune_keeps_results_bitwise():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_1024_l2")
    pot = Potential(cf.model, w, "bf16x3")
    pot.set_path("layered")  # the tuned products are the layered kernels'
    P, Z = _dev(pos, z)
    E1, F1 = pot.energy_forces(P, Z, L)
    torch.cuda.synchronize()
    E1, F1 = E1.clone(), F1.clone()
    rep = pot.autotune(P, Z, L, reps=1)
    assert rep["sites"] and all(0 <= s["chosen"] < len(s["ms"]) for s in rep["sites"])
    E2, F2 = pot.energy_forces(P, Z, L)
    torch.cuda.synchronize()
    assert E1.item() == E2.item()
    assert torch.equal(F1, F2)
    pot.close()


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
def test_kernel_variants_bitwise(prec):
    """Every kernel choice of every matrix-core product (all tile shapes of the
    tiled kernel, both epilogue forms of the weight-stationary kernel) gives
    the same bits. Variant v selects v modulo each product's count, so
    v = 0 .. max count - 1 visits every variant of every product; -2 / -3 are
    the two weight-stationary forms where compiled. (The 27,648-atom test
    repeats this for the tuned choice at a ragged edge count.)"""
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_1024_l2")
    pot = Potential(cf.model, w, prec)
    pot.set_path("layered")
    P, Z = _dev(pos, z)
    rep = pot.autotune(P, Z, L, reps=1)
    nmax = max(len(site["ms"]) for site in rep["sites"])
    assert nmax >= 4
    ref = None
    for v in list(range(nmax)) + [-2, -3, -1]:
        pot.set_variant(v)
        E, F, Ei = pot.energy_forces(P, Z, L, atom_energy=True)
        torch.cuda.synchronize()
        got = (E.item(), F.cpu().numpy(), Ei.cpu().numpy())
        if ref is None:
            ref = got
        else:
            assert got[0] == ref[0], v
            assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2]), v
    from paper_2303_08169_amd.binding import NQError
    with pytest.raises(NQError):
        pot.set_variant(-4)
    pot.close()
