"""FP64 CPU oracle of the Allegro-style energy and force evaluation.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
definition that the GPU path is checked against. Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it. It shares no code with the
GPU library (paper_2303_08169_amd) and never imports it.

What it computes follows the paper's problem statement: Newton's equations with
forces f = -dE/dr (Sec. 2.1, Eq. 1), an energy assembled from pairwise
embedding energies E_ij of atom pairs within a finite cutoff that is invariant
under rotation, inversion and translation and is built from tensors up to rank l
combined by tensor products of irreducible representations (Sec. 2.1). The
paper does not print Allegro's equations; the concrete model (Bessel radial
basis with a polynomial cutoff, component-normalised real spherical harmonics,
two-body / latent / edge MLPs with SiLU, environment sums over neighbours,
channel-wise Clebsch-Gordan products, per-edge energies) is this project's
reading of that summary and is written out step by step in oracle.model.

Every function states its pin (closed form, invariance, brute force or finite
differences) in the tests under tests/test_oracle_*.py.
"""
from .sh import real_sh, real_sh_grad, tp_paths, clebsch_gordan
from .radial import envelope, bessel
from .neighbors import edge_list
from .model import weight_segments, unpack_weights, energy_forces, EdgeTrace
from .md import velocity_verlet, nose_hoover
from .pimd import ring_polymer, omega_p
from .robustness import force_outliers

__all__ = ["real_sh", "real_sh_grad", "tp_paths", "clebsch_gordan", "envelope", "bessel",
           "edge_list", "weight_segments", "unpack_weights", "energy_forces", "EdgeTrace",
           "velocity_verlet", "nose_hoover", "ring_polymer", "omega_p", "force_outliers"]
