"""Error paths of the C ABI on the GPU. Every condition is produced from the host
inputs (no kernel is made to fault): each call must return its documented
status, and the context must stay usable afterwards."""
import numpy as np
import pytest
import torch

from paper_2303_08169_amd.binding import NQError
from tests.gpu_common import system

pytestmark = pytest.mark.gpu


def _setup():
    from paper_2303_08169_amd.potential import Potential
    cf, pos, z, L, w = system("nh3_64_l1")
    return Potential(cf.model, w, "fp32"), pos, z, L


def _dev(pos, z):
    return torch.tensor(pos, device="cuda"), torch.tensor(np.asarray(z), dtype=torch.int32, device="cuda")


def test_status_codes_and_recovery():
    pot, pos, z, L = _setup()
    P, Z = _dev(pos, z)
    E0, F0 = pot.energy_forces(P, Z, L)
    E0 = E0.item()
    # cutoff larger than half the box: rejected before any launch
    with pytest.raises(NQError) as e:
        pot.energy_forces(P, Z, 7.0)
    assert e.value.status == -1
    # a non-finite coordinate
    bad = pos.copy()
    bad[5, 1] = np.nan
    with pytest.raises(NQError) as e:
        pot.energy_forces(*_dev(bad, z), L)
        pot.stats()
    assert e.value.status == -4
    # two atoms 0.05 A apart
    close = pos.copy()
    close[1] = close[0] + np.array([0.05, 0.0, 0.0])
    with pytest.raises(NQError) as e:
        pot.energy_forces(*_dev(close, z), L)
        pot.stats()
    assert e.value.status == -4
    # species outside [0, n_species)
    zz = np.array(z).copy()
    zz[3] = 7
    with pytest.raises(NQError) as e:
        pot.energy_forces(*_dev(pos, zz), L)
        pot.stats()
    assert e.value.status == -1
    # the context still works
    E1, F1 = pot.energy_forces(P, Z, L)
    torch.cuda.synchronize()
    assert E1.item() == E0
    pot.stats()
    pot.close()


def test_argument_checks():
    pot, pos, z, L = _setup()
    P, Z = _dev(pos, z)
    with pytest.raises(TypeError):
        pot.energy_forces(P.float(), Z, L)
    with pytest.raises(ValueError):
        pot.energy_forces(P[:, :2].contiguous(), Z, L)
    pot.close()


def _compressed_1024():
    """The 1,024-atom system with 343 atoms moved onto a 7x7x7 grid of spacing
    0.55 A (rows of > 340 list entries, beyond the 256 the list was sized for;
    no pair closer than 0.55 A)."""
    cf, pos, z, L, w = system("nh3_1024_l2")
    q = pos.copy()
    g = np.stack(np.meshgrid(*[np.arange(7) * 0.55] * 3, indexing="ij"), -1).reshape(-1, 3)
    # every atom within 0.7 A of the grid's box moves onto it, then others until 343
    c = 5.0 + 1.65
    inside = np.abs(((q - c + L / 2) % L) - L / 2).max(axis=1) <= 1.65 + 0.7
    idx = np.concatenate([np.where(inside)[0], np.where(~inside)[0]])[:343]
    assert inside.sum() < 343
    q[idx] = 5.0 + g
    return cf, pos, q, z, L, w


def test_device_detected_overflow_poisons_outputs():
    """An on-device list rebuild whose rows overflow truncates them: the outputs
    of that evaluation are NaN without any synchronising call, the next
    nq_stats reports NQ_ERR_CAPACITY, and the next evaluation rebuilds the list
    on the host with a grown capacity and gives the result of a fresh context."""
    from paper_2303_08169_amd.potential import Potential
    cf, pos, q, z, L, w = _compressed_1024()
    pot = Potential(cf.model, w, "fp32")
    Z = torch.tensor(z, dtype=torch.int32, device="cuda")
    pot.energy_forces(torch.tensor(pos, device="cuda"), Z, L)
    Q = torch.tensor(q, device="cuda")
    E, F = pot.energy_forces(Q, Z, L)  # moved atoms: rebuilt on the device, rows overflow
    torch.cuda.synchronize()
    assert np.isnan(E.item()) and torch.isnan(F).all()
    with pytest.raises(NQError) as e:
        pot.stats()
    assert e.value.status == -3
    E2, F2 = pot.energy_forces(Q, Z, L)
    torch.cuda.synchronize()
    pot.stats()
    fresh = Potential(cf.model, w, "fp32")
    E3, F3 = fresh.energy_forces(Q, Z, L)
    torch.cuda.synchronize()
    assert np.isfinite(E2.item()) and E2.item() == E3.item() and torch.equal(F2, F3)
    pot.close()
    fresh.close()


def test_row_capacity_growth_and_limit():
    """A host-side list build whose rows overflow grows the row capacity once and
    succeeds (checked against the oracle); rows beyond the largest capacity
    (2,048) give NQ_ERR_CAPACITY, after which the context still works."""
    import oracle
    from paper_2303_08169_amd.potential import Potential
    cf, _, _, _, w = system("nh3_64_l1")
    rng = np.random.default_rng(5)
    L = 20.0
    # 100 atoms spread out (at least 1 A apart) and a 5x5x4 block of spacing 0.6 A
    spread = [rng.uniform(0, L, 3)]
    while len(spread) < 100:
        p = rng.uniform(0, L, 3)
        d = np.array(spread) - p
        d -= L * np.round(d / L)
        e = p - 2.2
        e -= L * np.round(e / L)
        if np.linalg.norm(d, axis=1).min() > 1.0 and np.linalg.norm(e) > 3.5:
            spread.append(p)
    block = 1.0 + 0.6 * np.stack(np.meshgrid(np.arange(5), np.arange(5), np.arange(4), indexing="ij"), -1).reshape(-1, 3)
    pos = np.concatenate([np.array(spread), block])
    z = rng.integers(0, 2, len(pos)).astype(np.int32)
    pot = Potential(cf.model, w, "fp32")
    P, Z = _dev(pos, z)
    E, F = pot.energy_forces(P, Z, L)  # rows of ~100 entries against a capacity sized for ~13
    torch.cuda.synchronize()
    pot.stats()
    E0, F0 = oracle.energy_forces(pos, z, L, cf.model, w)
    assert abs(E.item() - E0) <= 1e-5 * abs(E0)
    assert float(np.abs(F.cpu().numpy() - F0).max()) <= 1e-5 * float(np.abs(F0).max())
    # 2,100 atoms within 2.4 A of one point: rows of 2,099 entries
    ball = rng.normal(size=(2100, 3))
    ball = 10.0 + 2.4 * ball / np.linalg.norm(ball, axis=1, keepdims=True) * rng.uniform(0, 1, (2100, 1)) ** (1 / 3)
    with pytest.raises(NQError) as e:
        pot.energy_forces(*_dev(ball, np.zeros(2100, np.int32)), L)
    assert e.value.status == -3
    E2, F2 = pot.energy_forces(P, Z, L)
    torch.cuda.synchronize()
    assert E2.item() == E.item() and torch.equal(F2, F)
    pot.close()
