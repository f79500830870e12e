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
