"""The five workloads of the energy+force path, as plain data.

Sizes follow the liquid-ammonia systems of the paper's scaling runs (Sec. 3.3:
6,912 atoms per GPU; single-node runs of 1,728 to 13,824 atoms) at a number
density of 0.0965 atoms per cubic Angstrom, with the cutoff r_max = 6.0 A and
the equivariant rank l of the model table (Sec. 4.1, Table 2; Sec. 4.5, Table 5).
The model widths are this project's choice (the paper does not state them).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List

DENSITY = 0.0965  # atoms per A^3


@dataclass(frozen=True)
class ModelDesc:
    """Hyper-parameters of the Allegro-style edge model (mirrors nq_model_desc)."""
    n_species: int = 3
    n_bessel: int = 8
    poly_p: int = 6
    lmax: int = 2
    n_layers: int = 2
    channels: int = 32
    twobody: List[int] = field(default_factory=lambda: [64, 128, 256])
    latent: List[int] = field(default_factory=lambda: [256])
    edge: List[int] = field(default_factory=lambda: [128])
    r_cut: float = 6.0
    avg_num_neighbors: float = 4.0 / 3.0 * math.pi * 6.0 ** 3 * DENSITY
    energy_scale: float = 1.0

    @property
    def latent_dim(self) -> int:
        return self.twobody[-1]

    def as_dict(self):
        return asdict(self)


@dataclass(frozen=True)
class SystemSpec:
    name: str
    n_atoms: int
    seed: int
    model: ModelDesc
    skin: float = 1.0
    weight_seed: int = 0

    @property
    def n_molecules(self) -> int:
        return self.n_atoms // 4

    @property
    def box(self) -> float:
        return (self.n_atoms / DENSITY) ** (1.0 / 3.0)


def _nu(rc: float) -> float:
    return 4.0 / 3.0 * math.pi * rc ** 3 * DENSITY


SMALL_MODEL = ModelDesc(lmax=1, n_layers=1, channels=8, twobody=[32, 32], latent=[32],
                        edge=[16], r_cut=4.0, avg_num_neighbors=_nu(4.0))
MAIN_MODEL = ModelDesc()
SCALE_MODEL = ModelDesc(lmax=2, n_layers=3, channels=64, twobody=[128, 256, 512],
                        latent=[512], edge=[128])

CONFIGS = {
    # 64 atoms (16 NH3), box ~8.7 A, cutoff 4 A, l<=1, one layer, 8 channels
    "nh3_64_l1": SystemSpec("nh3_64_l1", 64, 100, SMALL_MODEL, skin=0.3),
    # 1,024 atoms (256 NH3), box ~22 A, cutoff 6 A, l<=2, two layers, 32 channels
    "nh3_1024_l2": SystemSpec("nh3_1024_l2", 1024, 101, MAIN_MODEL),
    # 27,648 atoms (6,912 NH3), box ~65.9 A, same model
    "nh3_27648_l2": SystemSpec("nh3_27648_l2", 27648, 102, MAIN_MODEL),
    # 262,144 atoms (65,536 NH3), box ~140 A, three layers, 64 channels
    "nh3_262144_l2_big": SystemSpec("nh3_262144_l2_big", 262144, 104, SCALE_MODEL),
}


def config(name: str) -> SystemSpec:
    return CONFIGS[name]
