"""Per-product precision overrides (nq_model_set_product_precision) through
the C ABI.

Every product keeps FP32 inputs and outputs in memory, so a model whose
products are all overridden to another precision runs exactly the kernels of
a model built in that precision: the results must be bitwise equal. A single
override changes only that product's arithmetic and stays within the plain
BF16 error of the FP64 oracle; the fused path refuses overrides; an MD graph
captured before an override is captured again."""
import numpy as np
import pytest
import torch

from tests.gpu_common import TOL, assert_forces_close, golden, system

pytestmark = pytest.mark.gpu


def _pot(cf, w, prec, path="layered"):
    from paper_2303_08169_amd.potential import Potential
    p = Potential(cf.model, w, prec)
    p.set_path(path)
    return p


def _sites(pot, P, Z, L, T):
    names = [s["name"] for s in pot.autotune(P, Z, L, reps=1)["sites"]]
    return names + [f"tp_{d}{t}" for t in range(1, T) for d in ("fwd", "bwd")]


def _eval(pot, P, Z, L):
    E, F, Ei = pot.energy_forces(P, Z, L, atom_energy=True)
    torch.cuda.synchronize()
    return E.item(), F.cpu().numpy(), Ei.cpu().numpy()


@pytest.mark.parametrize("base,target", [("bf16", "bf16x3"), ("bf16x3", "bf16"), ("bf16x3", "fp32")])
def test_all_sites_overridden_equal_the_other_model(base, target):
    cf, pos, z, L, w = system("nh3_1024_l2")
    print(f"precision overrides {base} -> {target}", flush=True)
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    ref = _pot(cf, w, target)
    Er, Fr, Eir = _eval(ref, P, Z, L)
    ref.close()
    pot = _pot(cf, w, base)
    sites = _sites(pot, P, Z, L, cf.model.n_layers)
    assert len(sites) >= 18
    pot.set_product_precision({s: target for s in sites})
    E, F, Ei = _eval(pot, P, Z, L)
    assert E == Er and np.array_equal(F, Fr) and np.array_equal(Ei, Eir)
    # dropping the overrides gives the base model back
    pot.set_product_precision({s: None for s in sites})
    E2, F2, _ = _eval(pot, P, Z, L)
    base_pot = _pot(cf, w, base)
    E3, F3, _ = _eval(base_pot, P, Z, L)
    base_pot.close()
    pot.close()
    assert E2 == E3 and np.array_equal(F2, F3)


def test_single_override_changes_only_within_bf16_error():
    cf, pos, z, L, w = system("nh3_1024_l2")
    g = golden("nh3_1024_l2")
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    pot = _pot(cf, w, "bf16x3")
    E0, F0, _ = _eval(pot, P, Z, L)
    pot.set_product_precision({"fwd.latent1.0": "bf16"})
    E1, F1, _ = _eval(pot, P, Z, L)
    pot.close()
    assert not np.array_equal(F0, F1)   # the override took effect
    assert abs(E1 - g["energy"]) <= TOL["bf16"]["energy"] * abs(g["energy"])
    assert_forces_close(F1, g["forces"], TOL["bf16"]["force"], "one product in bf16")


def test_fused_path_refuses_overrides():
    from paper_2303_08169_amd.binding import NQError
    cf, pos, z, L, w = system("nh3_1024_l2")
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    pot = _pot(cf, w, "bf16x3", "fused")
    pot.set_product_precision({"fwd.latent1.0": "bf16"})
    with pytest.raises(NQError):
        _eval(pot, P, Z, L)
    pot.set_product_precision({"fwd.latent1.0": None})
    E, F, _ = _eval(pot, P, Z, L)
    assert np.isfinite(E) and np.isfinite(F).all()
    pot.close()


def test_md_graph_recaptured_after_override():
    from synth.nh3 import masses, maxwell_boltzmann
    cf, pos, z, L, w = system("nh3_1024_l2")
    pot = _pot(cf, w, "bf16x3")
    P = torch.tensor(pos, device="cuda")
    V = torch.tensor(maxwell_boltzmann(z, 300.0, 200) * 0.01, device="cuda")
    IM = torch.tensor(1.0 / masses(z), device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    E, F = pot.energy_forces(P, Z, L)
    pot.step(P, V, IM, Z, L, 0.5, 2, F)
    pot.step(P, V, IM, Z, L, 0.5, 2, F)
    torch.cuda.synchronize()
    n0 = pot.graph_captures()
    pot.set_product_precision({"fwd.latent1.0": "bf16"})
    pot.step(P, V, IM, Z, L, 0.5, 2, F)
    torch.cuda.synchronize()
    assert pot.graph_captures() == n0 + 1
    # the replayed step uses the override: its forces are those of a direct call
    Fg = F.clone()
    E2, F2 = pot.energy_forces(P, Z, L)
    torch.cuda.synchronize()
    assert torch.equal(Fg, F2)
    pot.close()


def test_mixed_precision_meets_targets():
    """The "mixed" precision (split BF16 with the least sensitive products in
    plain BF16) against the FP64 oracle on 1,024 atoms: 1e-3 forces, 1e-5 energy."""
    from paper_2303_08169_amd.potential import MIXED_BF16
    cf, pos, z, L, w = system("nh3_1024_l2")
    g = golden("nh3_1024_l2")
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    pot = _pot(cf, w, "mixed")
    E, F, Ei = _eval(pot, P, Z, L)
    pot.close()
    ref = _pot(cf, w, "bf16x3")
    E3, F3, _ = _eval(ref, P, Z, L)
    ref.close()
    assert len(MIXED_BF16) > 0 and not np.array_equal(F, F3)
    assert abs(E - g["energy"]) <= TOL["bf16x3"]["energy"] * abs(g["energy"])
    assert_forces_close(F, g["forces"], TOL["bf16x3"]["force"], "mixed")
