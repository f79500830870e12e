"""PyTorch-facing wrapper of the HIP library.

PyTorch provides device memory and the stream; every step of the energy/force
path runs in libnnqmd.so. `Potential.energy_forces` returns E and F = -dE/dr
(paper Sec. 2.1, Eq. 1); `EnergyForces` exposes E to autograd with the
library's forces as its gradient; `Potential.step` runs velocity-Verlet steps
replayed from a HIP graph.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as B


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _cell(box):
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)).copy()
    return (C.c_double * 3)(*b.tolist())


# Products of the split-BF16 model that run in plain BF16 in the "mixed"
# precision: the channel mixing of the tensor product (both directions), the
# environment embeddings of the second layer and the adjoint of the first
# layer's tensor-feature/environment embedding. Chosen by a per-product study
# on the 1,024-atom system against the FP64 oracle (bench.py --sensitivity):
# each alone in plain BF16 moves the force error by less than 1e-4 relative
# and the energy error by less than 3e-6, and all together keep both below
# half the 1e-3 / 1e-5 targets. The two-body, latent and edge-energy MLPs stay
# split (each alone in plain BF16 moves the force error by 5e-4 to 5e-3).
MIXED_BF16 = ("bwd.env2", "tp_bwd1", "tp_fwd1", "fwd.env2", "bwd.v0env1")


class Potential:
    """One context + one model on a GPU.

    model: an object with the hyper-parameters (n_species, n_bessel, poly_p, lmax,
    n_layers, channels, twobody, latent, edge, r_cut, avg_num_neighbors,
    energy_scale); weights: flat FP64 host array in the library's layout.
    """

    def __init__(self, model, weights, precision: str = "fp32", device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required")
        self.lib = B.lib()
        self.device = torch.device("cuda", device)
        self.desc = B.make_desc(model, precision)
        self.precision = precision
        segs, ntot = B.weight_layout(self.desc)
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        if w.size != ntot:
            raise ValueError(f"weights have {w.size} values, the model needs {ntot}")
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            B.check(self.lib.nq_ctx_create(device, C.c_void_p(stream), C.byref(self._ctx)))
            self._model = C.c_void_p()
            B.check(self.lib.nq_model_create(self._ctx, C.byref(self.desc),
                                             w.ctypes.data_as(C.POINTER(C.c_double)), w.size,
                                             C.byref(self._model)), self._ctx)
        self._energy = torch.zeros(1, dtype=torch.float64, device=self.device)
        if precision == "mixed":
            self.set_product_precision({site: "bf16" for site in MIXED_BF16})

    def close(self):
        if getattr(self, "_model", None):
            self.lib.nq_model_destroy(self._model)
            self._model = None
        if getattr(self, "_ctx", None):
            self.lib.nq_ctx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        B.check(self.lib.nq_ctx_set_stream(self._ctx, C.c_void_p(s)), self._ctx)

    def _check_inputs(self, pos, species):
        if pos.device != self.device or species.device != self.device:
            raise ValueError("positions and species must live on the potential's device")
        if pos.dtype != torch.float64 or species.dtype != torch.int32:
            raise TypeError("positions must be float64 and species int32")
        if pos.dim() != 2 or pos.shape[1] != 3 or species.shape != (pos.shape[0],):
            raise ValueError("positions [n, 3], species [n]")
        if not (pos.is_contiguous() and species.is_contiguous()):
            raise ValueError("inputs must be contiguous")

    def neighbor_build(self, pos, box, r_cut=None, skin=1.0):
        self._sync_stream()
        rc = float(self.desc.r_cut if r_cut is None else r_cut)
        B.check(self.lib.nq_neighbor_build(self._ctx, _ptr(pos), pos.shape[0], _cell(box), rc, float(skin)),
                self._ctx)

    def energy_forces(self, pos, species, box, forces=None, energy=None, atom_energy=False):
        """(E [1] f64, F [n,3] f64[, E_i [n] f64]) on the device, queued on the current stream."""
        self._check_inputs(pos, species)
        n = pos.shape[0]
        F = forces if forces is not None else torch.empty((n, 3), dtype=torch.float64, device=self.device)
        E = energy if energy is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        Ei = torch.empty(n, dtype=torch.float64, device=self.device) if atom_energy else None
        self._sync_stream()
        B.check(self.lib.nq_energy_forces(self._ctx, self._model, _ptr(pos), _ptr(species), n, _cell(box),
                                          _ptr(E), _ptr(F), _ptr(Ei)), self._ctx)
        return (E, F, Ei) if atom_energy else (E, F)

    def energy_forces_replicas(self, pos, species, box, atom_energy=False):
        """Replicas of one box in one evaluation: pos [R, n, 3] f64, species
        [R, n] int32 -> (E [R] f64, F [R, n, 3] f64[, E_i [R, n] f64])."""
        if pos.dim() != 3 or pos.shape[2] != 3 or species.shape != pos.shape[:2]:
            raise ValueError("positions [R, n, 3], species [R, n]")
        R, n = pos.shape[0], pos.shape[1]
        self._check_inputs(pos.reshape(R * n, 3), species.reshape(R * n))
        F = torch.empty_like(pos)
        E = torch.empty(R, dtype=torch.float64, device=self.device)
        Ei = torch.empty((R, n), dtype=torch.float64, device=self.device) if atom_energy else None
        self._sync_stream()
        B.check(self.lib.nq_energy_forces_replicas(self._ctx, self._model, _ptr(pos), _ptr(species), n, R,
                                                   _cell(box), _ptr(E), _ptr(F), _ptr(Ei)), self._ctx)
        return (E, F, Ei) if atom_energy else (E, F)

    def energy_forces_domain(self, pos, species, n_local, box, atom_energy=False):
        """One spatial domain: pos [n, 3] with the n_local owned atoms first and
        ghosts after -> (E of the owned centres [1], F of all n atoms [n, 3][,
        E_i [n]]); box must leave r_c + skin of empty space around the atoms."""
        self._check_inputs(pos, species)
        n = pos.shape[0]
        F = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        E = torch.empty(1, dtype=torch.float64, device=self.device)
        Ei = torch.empty(n, dtype=torch.float64, device=self.device) if atom_energy else None
        self._sync_stream()
        B.check(self.lib.nq_energy_forces_domain(self._ctx, self._model, _ptr(pos), _ptr(species), int(n_local), n,
                                                 _cell(box), _ptr(E), _ptr(F), _ptr(Ei)), self._ctx)
        return (E, F, Ei) if atom_energy else (E, F)

    def ring_polymer(self, pos, inv_mass, box, temperature, forces, energy=None, noalloc=False):
        """Adds the ring-polymer spring forces of the beads pos [R, n, 3] to
        forces [R, n, 3] and returns the spring energy [1] (eV). noalloc uses
        the entry point that allocates no device memory (at most 2^20 beads x
        atoms; pass `energy` too, so that nothing here allocates either)."""
        if pos.dim() != 3 or forces.shape != pos.shape or inv_mass.shape != (pos.shape[1],):
            raise ValueError("positions and forces [R, n, 3], inv_mass [n]")
        for t in (pos, inv_mass, forces):
            if t.device != self.device or t.dtype != torch.float64 or not t.is_contiguous():
                raise TypeError("ring-polymer arrays must be contiguous float64 on the potential's device")
        E = energy if energy is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        self._sync_stream()
        fn = self.lib.nq_ring_polymer_noalloc if noalloc else self.lib.nq_ring_polymer
        B.check(fn(self._ctx, _ptr(pos), _ptr(inv_mass), pos.shape[1], pos.shape[0], _cell(box), float(temperature),
                   _ptr(forces), _ptr(E)), self._ctx)
        return E

    def step(self, pos, vel, inv_mass, species, box, dt_fs, n_steps, forces, epot=None, ekin=None):
        """n_steps velocity-Verlet steps in place; forces must hold F(pos) on entry."""
        self._check_inputs(pos, species)
        self._sync_stream()
        B.check(self.lib.nq_step(self._ctx, self._model, _ptr(pos), _ptr(vel), _ptr(inv_mass), _ptr(species),
                                 pos.shape[0], _cell(box), float(dt_fs), int(n_steps), _ptr(forces),
                                 _ptr(epot), _ptr(ekin)), self._ctx)

    def step_nvt(self, pos, vel, inv_mass, species, box, dt_fs, n_steps, temperature, tau_fs, thermostat, forces,
                 epot=None, ekin=None, ethermo=None):
        """n_steps Nose-Hoover NVT steps in place; thermostat: device float64 [2]
        (xi, eta), zero to start; forces must hold F(pos) on entry."""
        self._check_inputs(pos, species)
        self._sync_stream()
        B.check(self.lib.nq_step_nvt(self._ctx, self._model, _ptr(pos), _ptr(vel), _ptr(inv_mass), _ptr(species),
                                     pos.shape[0], _cell(box), float(dt_fs), int(n_steps), float(temperature),
                                     float(tau_fs), _ptr(thermostat), _ptr(forces), _ptr(epot), _ptr(ekin),
                                     _ptr(ethermo)), self._ctx)

    def force_outliers(self, forces, nsigma=5.0):
        """Number of force components beyond nsigma standard deviations (device int32 [1])."""
        count = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._sync_stream()
        B.check(self.lib.nq_force_outliers(self._ctx, _ptr(forces), forces.shape[0], float(nsigma), _ptr(count)),
                self._ctx)
        return count

    def autotune(self, pos, species, box, reps: int = 3):
        """Time every tile-shape candidate of every matrix-core product on this
        system and keep the fastest; returns the library's JSON report."""
        import json
        self._check_inputs(pos, species)
        self._sync_stream()
        buf = C.create_string_buffer(1 << 20)
        n = C.c_int64(0)
        B.check(self.lib.nq_autotune(self._ctx, self._model, _ptr(pos), _ptr(species), pos.shape[0], _cell(box),
                                     int(reps), buf, len(buf), C.byref(n)), self._ctx)
        return json.loads(buf.value.decode())

    def set_choice(self, choices):
        """Kernel variant per matrix-core product ({name: variant}, as in the
        "chosen" entries of autotune()'s report), e.g. replayed from a file."""
        for name, v in choices.items():
            B.check(self.lib.nq_model_set_choice(self._model, name.encode(), int(v)), self._ctx)

    def set_product_precision(self, precisions):
        """Arithmetic per product ({site: "fp32" | "bf16" | "bf16x3" | None}),
        overriding the model's precision; sites are the matrix-core product
        names of autotune()'s report and "tp_fwd<t>" / "tp_bwd<t>" (channel
        mixing of layer t). None drops an override."""
        for name, p in precisions.items():
            v = -1 if p is None else B.PRECISION[p]
            B.check(self.lib.nq_model_set_product_precision(self._model, name.encode(), v), self._ctx)

    def set_variant(self, variant: int):
        """Kernel choice of the matrix-core products: -1 tuned (default), -2 / -3
        the last / second-to-last variant of each product (the two epilogue forms
        of the weight-stationary kernel where compiled), v >= 0 variant v of
        each. Results are bitwise identical for every choice."""
        B.check(self.lib.nq_ctx_set_variant(self._ctx, int(variant)), self._ctx)

    PATHS = {"auto": 0, "layered": 1, "fused": 2}

    def set_path(self, path: str):
        """Evaluation path of later calls: "auto" or "layered" (the layered
        kernels) or "fused" (the persistent per-centre kernel; an error at the
        next evaluation if the model does not fit it)."""
        B.check(self.lib.nq_ctx_set_path(self._ctx, self.PATHS[path]), self._ctx)

    def set_workspace_budget(self, nbytes: int):
        """Cap the per-edge activation memory; larger systems run in chunks of centres."""
        B.check(self.lib.nq_ctx_set_workspace_budget(self._ctx, int(nbytes)), self._ctx)

    def stats(self):
        ne, nr = C.c_int64(0), C.c_int64(0)
        B.check(self.lib.nq_stats(self._ctx, C.byref(ne), C.byref(nr)), self._ctx)
        return ne.value, nr.value

    def graph_captures(self) -> int:
        """How many times nq_step / nq_step_nvt captured their HIP graph on this context."""
        n = C.c_int64(0)
        B.check(self.lib.nq_ctx_graph_captures(self._ctx, C.byref(n)), self._ctx)
        return n.value

    def edges(self):
        ne, _ = self.stats()
        cap = max(ne, 1)
        ei = torch.empty(cap, dtype=torch.int32, device=self.device)
        ej = torch.empty(cap, dtype=torch.int32, device=self.device)
        n = C.c_int64(0)
        B.check(self.lib.nq_edges_export(self._ctx, _ptr(ei), _ptr(ej), cap, C.byref(n)), self._ctx)
        return ei[:n.value], ej[:n.value]

    def debug(self, name: str, cap: int):
        out = torch.empty(cap, dtype=torch.float32, device=self.device)
        rows, width = C.c_int64(0), C.c_int64(0)
        B.check(self.lib.nq_debug_export(self._ctx, self._model, name.encode(), _ptr(out), cap,
                                         C.byref(rows), C.byref(width)), self._ctx)
        return out[:rows.value * width.value].view(rows.value, width.value)


class EnergyForces(torch.autograd.Function):
    """E(pos) with dE/dpos = -F from the library's hand-written adjoint."""

    @staticmethod
    def forward(ctx, pos, potential: Potential, species, box):
        E, F = potential.energy_forces(pos.detach(), species, box)
        ctx.save_for_backward(F)
        return E

    @staticmethod
    def backward(ctx, gE):
        (F,) = ctx.saved_tensors
        return -gE * F, None, None, None
