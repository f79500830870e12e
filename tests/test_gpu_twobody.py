"""The two-body MLP as one kernel per direction (the automatic path on the
benchmark model) against the per-layer products (the layered path), through
the C ABI.

The fused kernels form the same BF16 splits, the same K steps and the same
product order as the per-layer kernels, recompute the first two layers'
pre-activations from the same inputs in the adjoint, and add the dE/du row
sums in the same order, so energies, per-atom energies and forces must be
bitwise equal. Cases: 1,024 and 27,648 atoms (the latter leaves a ragged last
32-row tile), both BF16 kinds, a dilute system with fewer tiles than
workgroups (one-tile workgroups and idle ones), a system without edges, and an
evaluation split into centre chunks."""
import ctypes as C
import json

import numpy as np
import pytest
import torch

from tests.gpu_common import system

pytestmark = pytest.mark.gpu


def _pot(cf, w, prec, path):
    from paper_2303_08169_amd.potential import Potential
    p = Potential(cf.model, w, prec)
    p.set_path(path)
    return p


def _eval(pot, P, Z, L):
    E, F, Ei = pot.energy_forces(P, Z, L, atom_energy=True)
    torch.cuda.synchronize()
    return E.item(), F.cpu().numpy(), Ei.cpu().numpy()


def _spans(pot, P, Z, L):
    """Names of the timed stages of one evaluation."""
    from paper_2303_08169_amd import binding as B
    B.check(pot.lib.nq_timing(pot._ctx, 1), pot._ctx)
    pot.energy_forces(P, Z, L)
    torch.cuda.synchronize()
    B.check(pot.lib.nq_timing(pot._ctx, 0), pot._ctx)
    buf = C.create_string_buffer(1 << 20)
    n = C.c_int64(0)
    B.check(pot.lib.nq_timing_report(pot._ctx, buf, len(buf), C.byref(n)), pot._ctx)
    return {k["name"] for k in json.loads(buf.value.decode())["kernels"]}


@pytest.mark.parametrize("name,prec", [("nh3_1024_l2", "bf16x3"), ("nh3_1024_l2", "bf16"),
                                       ("nh3_27648_l2", "bf16x3")])
def test_fused_two_body_is_bitwise_the_per_layer_path(name, prec):
    cf, pos, z, L, w = system(name)
    print(f"two-body fused vs per-layer: {name} {prec}", flush=True)
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    lay = _pot(cf, w, prec, "layered")
    El, Fl, Eil = _eval(lay, P, Z, L)
    ne, _ = lay.stats()
    assert "fwd.twobody.0" in _spans(lay, P, Z, L)
    lay.close()
    auto = _pot(cf, w, prec, "auto")
    Ea, Fa, Eia = _eval(auto, P, Z, L)
    sp = _spans(auto, P, Z, L)
    assert {"fwd.twobody", "bwd.twobody"} <= sp and "fwd.twobody.0" not in sp and "bwd.twobody.2" not in sp
    # a second call reuses dE/du and the activations' buffers: same bits again
    Ea2, Fa2, _ = _eval(auto, P, Z, L)
    auto.close()
    print(f"{ne} edges, last 32-row tile {ne % 32 or 32} rows", flush=True)
    assert Ea == El and np.array_equal(Fa, Fl) and np.array_equal(Eia, Eil)
    assert Ea2 == Ea and np.array_equal(Fa2, Fa)


def test_fp32_and_layered_keep_the_per_layer_products():
    cf, pos, z, L, w = system("nh3_1024_l2")
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    p = _pot(cf, w, "fp32", "auto")
    assert "fwd.twobody.2" in _spans(p, P, Z, L)
    p.close()
    # an override of one two-body product keeps the per-layer kernels
    p = _pot(cf, w, "bf16x3", "auto")
    p.set_product_precision({"bwd.twobody.1": "bf16"})
    sp = _spans(p, P, Z, L)
    p.close()
    assert "bwd.twobody.1" in sp and "fwd.twobody" not in sp


def test_no_edges_and_chunks():
    cf, pos, z, L, w = system("nh3_1024_l2")
    # three atoms beyond each other's cutoff: no edges, zero forces
    pos3 = np.array([[0.0, 0.0, 0.0], [7.0, 0.0, 0.0], [0.0, 7.5, 0.0]])
    z3 = np.array([0, 1, 2], dtype=np.int32)
    L3 = 30.0
    P3 = torch.tensor(pos3, device="cuda")
    Z3 = torch.tensor(z3, dtype=torch.int32, device="cuda")
    res = {}
    for path in ("layered", "auto"):
        p = _pot(cf, w, "bf16x3", path)
        res[path] = _eval(p, P3, Z3, L3)
        p.close()
    assert res["auto"][0] == res["layered"][0]
    assert np.array_equal(res["auto"][1], res["layered"][1]) and not res["auto"][1].any()
    # the evaluation split into centre chunks by a small workspace budget
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    out = {}
    for path in ("layered", "auto"):
        p = _pot(cf, w, "bf16x3", path)
        p.set_workspace_budget(256 << 20)  # several chunks
        out[path] = _eval(p, P, Z, L)
        p.close()
    assert out["auto"][0] == out["layered"][0] and np.array_equal(out["auto"][1], out["layered"][1])


def test_few_tiles():
    """200 atoms in a 30 A box: about 40 edge tiles, fewer than the persistent
    workgroups, so most workgroups have no tile and the others exactly one."""
    cf, _, _, _, w = system("nh3_1024_l2")
    rng = np.random.default_rng(5)
    pos = []
    while len(pos) < 200:  # no pair closer than 1.5 A
        p = rng.uniform(0.0, 30.0, 3)
        if all(np.linalg.norm((p - q + 15.0) % 30.0 - 15.0) > 1.5 for q in pos):
            pos.append(p)
    pos = np.array(pos)
    z = rng.integers(0, 3, len(pos)).astype(np.int32)
    P = torch.tensor(pos, device="cuda")
    Z = torch.tensor(z, device="cuda")
    res = {}
    for path in ("layered", "auto"):
        p = _pot(cf, w, "bf16x3", path)
        res[path] = _eval(p, P, Z, 30.0)
        ne, _ = p.stats()
        p.close()
    print(f"{ne} edges, {(ne + 31) // 32} tiles", flush=True)
    assert 0 < ne < 32 * 256
    assert res["auto"][0] == res["layered"][0]
    assert np.array_equal(res["auto"][1], res["layered"][1]) and np.array_equal(res["auto"][2], res["layered"][2])
