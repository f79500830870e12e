"""GPU parity of the fused per-centre kernel against the FP64 oracle and the
layered kernels, through the C ABI.

The fused kernel evaluates one centre per workgroup in blocks of 64 edges, so
the cases cover centres with fewer than 16, between 16 and 64, between 64 and
128 and more than 128 edges (one, two and three blocks, ragged last row
tiles), isolated atoms (no edges), the liquid-ammonia systems of the
benchmark model, and the spatial-domain and replica entry points that share
the kernel.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import TOL, assert_forces_close, golden, rel_rms, system

pytestmark = pytest.mark.gpu


def _pot(cf, w, prec, path):
    from paper_2303_08169_amd.potential import Potential
    p = Potential(cf.model, w, prec)
    p.set_path(path)
    return p


def _dev(pos, z):
    return (torch.tensor(pos, device="cuda"), torch.tensor(np.asarray(z), dtype=torch.int32, device="cuda"))


def _run(pot, pos, z, L):
    P, Z = _dev(pos, z)
    E, F, Ei = pot.energy_forces(P, Z, L, atom_energy=True)
    torch.cuda.synchronize()
    return E.item(), F.cpu().numpy(), Ei.cpu().numpy()


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
def test_fused_matches_oracle_1024(prec):
    cf, pos, z, L, w = system("nh3_1024_l2")
    g = golden("nh3_1024_l2")
    print(f"fused 1024 atoms {prec}", flush=True)
    pot = _pot(cf, w, prec, "fused")
    E, F, Ei = _run(pot, pos, z, L)
    assert abs(E - g["energy"]) <= TOL[prec]["energy"] * abs(g["energy"])
    assert_forces_close(F, g["forces"], TOL[prec]["force"], "fused " + prec)
    assert rel_rms(Ei, g["atom_energy"]) <= 10 * TOL[prec]["energy"]
    fd, got = g["fd_forces"], F[g["fd_atoms"]]
    assert np.abs(got - fd).max() <= TOL[prec]["force"] * 10 * np.abs(fd).max()
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-5 * np.abs(F).sum())
    # a second call gives the same bits (every sum runs in a fixed order)
    E2, F2, Ei2 = _run(pot, pos, z, L)
    assert E2 == E and np.array_equal(F2, F) and np.array_equal(Ei2, Ei)
    pot.close()


def test_fused_agrees_with_layered_1024():
    cf, pos, z, L, w = system("nh3_1024_l2")
    print("fused vs layered 1024 atoms bf16x3", flush=True)
    pf = _pot(cf, w, "bf16x3", "fused")
    Ef, Ff, Eif = _run(pf, pos, z, L)
    pf.close()
    pl = _pot(cf, w, "bf16x3", "layered")
    El, Fl, Eil = _run(pl, pos, z, L)
    pl.close()
    # both paths are within the BF16X3 error of the oracle; they differ by less
    assert abs(Ef - El) <= 1e-5 * abs(El)
    assert_forces_close(Ff, Fl, 1e-4, "fused vs layered")
    assert rel_rms(Eif, Eil) <= 1e-4


def _dense_box(seed, n, L, dmin):
    """n atoms, uniformly random in a cube of side L, no pair closer than dmin."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0, L, 3)
        if pts:
            d = np.asarray(pts) - p
            d -= L * np.round(d / L)
            if np.min(np.linalg.norm(d, axis=1)) < dmin:
                continue
        pts.append(p)
    return np.asarray(pts), rng.integers(0, 2, size=n).astype(np.int32)


@pytest.mark.parametrize("case", ["dense", "sparse"])
def test_fused_block_edges(case):
    """Centres of 0 to ~170 edges: one to three blocks of 64, ragged tiles."""
    cf, _, _, _, w = system("nh3_1024_l2")
    if case == "dense":
        L = 13.0
        pos, z = _dense_box(11, 360, L, 0.85)   # 122 to 169 neighbours per atom
    else:
        # a cluster in one corner of a 20 A box plus one atom with no neighbour
        L = 20.0
        pos, z = _dense_box(12, 40, 6.0, 1.2)
        pos = np.vstack([pos, [12.5, 12.5, 12.5]])
        z = np.append(z, 1).astype(np.int32)
    ei, _ = oracle.edge_list(pos, L, cf.model.r_cut)
    cnt = np.bincount(ei, minlength=len(pos))
    print(f"fused {case}: edges per centre {cnt.min()}..{cnt.max()}", flush=True)
    E0, F0, Ei0 = oracle.energy_forces(pos, z, L, cf.model, w, atom_energy=True)
    pot = _pot(cf, w, "bf16x3", "fused")
    E, F, Ei = _run(pot, pos, z, L)
    pot.close()
    assert abs(E - E0) <= 1e-5 * np.abs(Ei0).sum()
    assert_forces_close(F, F0, 1e-3, "fused " + case)
    assert np.abs(Ei - Ei0).max() <= 1e-4 * np.abs(Ei0).max()
    if case == "dense":
        assert cnt.max() > 128 and cnt.min() > 64
    else:
        assert cnt.min() == 0 and cnt.max() > 16


def test_fused_unsupported_model_is_an_error():
    from paper_2303_08169_amd.binding import NQError
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = _pot(cf, w, "bf16x3", "fused")
    with pytest.raises(NQError):
        _run(pot, pos, z, L)
    pot.set_path("auto")  # the layered kernels serve this model
    E, F, _ = _run(pot, pos, z, L)
    assert np.isfinite(E) and np.isfinite(F).all()
    pot.close()


def test_fused_replicas_bitwise_single():
    """Replica-batched evaluation through the fused kernel: each replica's
    results are bitwise those of evaluating it alone (centres never mix)."""
    from tests.test_gpu_replicas import _replicas
    cf, pos, z, L, w = system("nh3_1024_l2")
    R = 3
    reps = _replicas(pos, L, R, 17)
    print("fused replicas", flush=True)
    pot = _pot(cf, w, "bf16x3", "fused")
    P = torch.tensor(reps, device="cuda")
    Z = torch.tensor(np.tile(z, (R, 1)), dtype=torch.int32, device="cuda")
    E, F, Ei = pot.energy_forces_replicas(P, Z, L, atom_energy=True)
    torch.cuda.synchronize()
    E, F, Ei = E.clone(), F.clone(), Ei.clone()
    one = _pot(cf, w, "bf16x3", "fused")
    for r in range(R):
        e1, f1, ei1 = one.energy_forces(P[r].contiguous(), Z[r].contiguous(), L, atom_energy=True)
        torch.cuda.synchronize()
        assert E[r].item() == e1.item() and torch.equal(F[r], f1) and torch.equal(Ei[r], ei1), r
    pot.close()
    one.close()


def test_fused_domain_matches_oracle():
    """One spatial domain (owned atoms + ghost images in an open frame) through
    the fused kernel against the oracle with the owned atoms as the only centres."""
    from tests.test_gpu_domain import _domain
    cf, pos, z, L, w = system("nh3_1024_l2")
    q, orig, n_own, frame = _domain(pos, L, 0.0, L / 2, cf.model.r_cut, margin=8.0)
    print(f"fused domain: {n_own} owned, {len(q) - n_own} ghosts", flush=True)
    Eo, Fo = oracle.energy_forces(q, z[orig], frame, cf.model, w, centers=np.arange(n_own))
    pot = _pot(cf, w, "bf16x3", "fused")
    Ed, Fd, Ad = pot.energy_forces_domain(torch.tensor(q, device="cuda"),
                                          torch.tensor(z[orig], dtype=torch.int32, device="cuda"), n_own, frame,
                                          atom_energy=True)
    Fd, Ad = Fd.cpu().numpy(), Ad.cpu().numpy()
    pot.close()
    assert abs(Ed.item() - Eo) <= TOL["bf16x3"]["energy"] * abs(Eo)
    assert_forces_close(Fd[:n_own], Fo[:n_own], TOL["bf16x3"]["force"], "owned")
    assert_forces_close(Fd[n_own:], Fo[n_own:], TOL["bf16x3"]["force"], "ghosts")
    assert np.all(Ad[n_own:] == 0.0)


def test_fused_md_steps_match_layered():
    """Velocity-Verlet through the captured MD step with the fused kernel
    against the same steps with the layered kernels (10 steps of 0.5 fs)."""
    from synth.nh3 import masses, maxwell_boltzmann
    cf, pos, z, L, w = system("nh3_1024_l2")
    out = {}
    for path in ("fused", "layered"):
        print(f"md steps {path}", flush=True)
        pot = _pot(cf, w, "bf16x3", path)
        P = torch.tensor(pos, device="cuda")
        V = torch.tensor(maxwell_boltzmann(z, 300.0, 200) * 0.01, device="cuda")
        IM = torch.tensor(1.0 / masses(z), device="cuda")
        Z = torch.tensor(z, dtype=torch.int32, device="cuda")
        E, F = pot.energy_forces(P, Z, L)
        ep = torch.zeros(10, dtype=torch.float64, device="cuda")
        ek = torch.zeros(10, dtype=torch.float64, device="cuda")
        pot.step(P, V, IM, Z, L, 0.5, 10, F, ep, ek)
        torch.cuda.synchronize()
        out[path] = (P.cpu().numpy(), ep.cpu().numpy())
        pot.close()
    d = out["fused"][0] - out["layered"][0]
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-6
    np.testing.assert_allclose(out["fused"][1], out["layered"][1], rtol=1e-5)


def test_fused_full_size_sampled():
    """27,648 atoms through the fused kernel: exact oracle forces on sampled
    atoms and per-centre energies around them."""
    cf, pos, z, L, w = system("nh3_27648_l2")
    print("fused 27,648 atoms", flush=True)
    pot = _pot(cf, w, "bf16x3", "fused")
    E, F, Ei = _run(pot, pos, z, L)
    pot.close()
    rng = np.random.default_rng(7)
    atoms = rng.choice(len(pos), 4, replace=False)
    cs = [atoms] + [oracle.edge_list(pos, L, cf.model.r_cut, centers=[a])[1] for a in atoms]
    centers = np.unique(np.concatenate(cs))
    _, F0, E0 = oracle.energy_forces(pos, z, L, cf.model, w, centers=centers, atom_energy=True)
    assert_forces_close(F[atoms], F0[atoms], TOL["bf16x3"]["force"], "fused full size")
    assert rel_rms(Ei[centers], E0[centers]) <= 10 * TOL["bf16x3"]["energy"]
    assert abs(E - Ei.sum()) <= 1e-9 * np.abs(Ei).sum()
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-6 * np.abs(F).sum())
