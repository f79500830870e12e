"""The ring-polymer entry point that allocates no device memory
(nq_ring_polymer_noalloc, for callers that cannot allocate) against the
allocating nq_ring_polymer, through the C ABI.

Both run the same kernels on the same inputs, so energies and forces must be
bitwise equal; the oracle bounds both. Two calls in a row, the second with a
smaller input, show that what the fixed array keeps from the first call does
not leak into the second; an oversize request is rejected before anything is
launched."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_common import system

pytestmark = pytest.mark.gpu


def _beads(pos, L, R, seed):
    rng = np.random.default_rng(seed)
    return np.stack([(pos + rng.normal(scale=0.2, size=pos.shape)) % L for _ in range(R)])


def _call(lib, ctx, name, P, IM, L, T, F, E):
    cell = (C.c_double * 3)(L, L, L)
    return getattr(lib, name)(ctx, C.c_void_p(P.data_ptr()), C.c_void_p(IM.data_ptr()), P.shape[1], P.shape[0],
                              cell, T, C.c_void_p(F.data_ptr()), C.c_void_p(E.data_ptr()))


def test_noalloc_matches_allocating_entry_point():
    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.potential import Potential
    from synth.nh3 import masses
    cf, pos, z, L, w = system("nh3_1024_l2")
    m = masses(z)
    pot = Potential(cf.model, w, "fp32")
    IM = torch.tensor(1.0 / m, device="cuda")
    # first call: 32 beads x 1024 atoms; second: 8 beads x 1000 atoms
    for R, n, T, seed in ((32, len(pos), 300.0, 3), (8, 1000, 150.0, 4)):
        print(f"ring polymer noalloc: {R} beads x {n} atoms", flush=True)
        reps = _beads(pos[:n], L, R, seed)
        P = torch.tensor(reps, device="cuda")
        F0 = torch.tensor(np.random.default_rng(seed).normal(size=reps.shape), device="cuda")
        out = {}
        for name in ("nq_ring_polymer_noalloc", "nq_ring_polymer"):
            F = F0.clone()
            E = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            assert B.STATUS[_call(pot.lib, pot._ctx, name, P, IM[:n], L, T, F, E)] == "NQ_OK", name
            torch.cuda.synchronize()
            out[name] = (E.item(), (F - F0).cpu().numpy())
        Ea, Fa = out["nq_ring_polymer_noalloc"]
        Eb, Fb = out["nq_ring_polymer"]
        assert Ea == Eb and np.array_equal(Fa, Fb)
        Eo, Fo = oracle.ring_polymer(reps, m[:n], L, T)
        assert abs(Ea - Eo) <= 1e-12 * max(1.0, abs(Eo))
        np.testing.assert_allclose(Fa, Fo, rtol=1e-10, atol=1e-10 * max(1.0, np.abs(Fo).max()))
    pot.close()


def test_noalloc_rejects_oversize():
    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    pot = Potential(cf.model, w, "fp32")
    n = 64
    R = (1 << 20) // n + 1                     # one bead more than the array holds
    P = torch.zeros((R, n, 3), dtype=torch.float64, device="cuda")
    F = torch.zeros_like(P)
    E = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    IM = torch.ones(n, dtype=torch.float64, device="cuda")
    st = _call(pot.lib, pot._ctx, "nq_ring_polymer_noalloc", P, IM, L, 300.0, F, E)
    assert B.STATUS[st] == "NQ_ERR_CAPACITY"
    assert "NQ_RING_POLYMER_NOALLOC_MAX" in pot.lib.nq_last_error(pot._ctx).decode()
    torch.cuda.synchronize()
    assert E.item() == 7.0 and not F.any()   # nothing was launched
    # the largest size it accepts works
    P = P[: R - 1].contiguous()
    F = torch.zeros_like(P)
    assert B.STATUS[_call(pot.lib, pot._ctx, "nq_ring_polymer_noalloc", P, IM, L, 300.0, F, E)] == "NQ_OK"
    torch.cuda.synchronize()
    assert E.item() == 0.0 and not F.any()   # coincident beads: no spring stretched
    pot.close()
