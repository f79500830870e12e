"""ctypes binding of libnnqmd.so: argument marshalling only.

Every function here maps one-to-one onto an entry point of include/nnqmd.h; all
arithmetic runs in the HIP library. Loading fails loudly if the library has not
been built (python -m paper_2303_08169_amd.build).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnnqmd.so")

NQ_OK = 0
STATUS = {0: "NQ_OK", -1: "NQ_ERR_ARG", -2: "NQ_ERR_UNSUPPORTED", -3: "NQ_ERR_CAPACITY",
          -4: "NQ_ERR_NUMERIC", -5: "NQ_ERR_DEVICE", -6: "NQ_ERR_OOM"}
PRECISION = {"fp32": 0, "bf16": 1, "bf16x3": 2}

EXPORTS = ["nq_ctx_create", "nq_ctx_set_stream", "nq_ctx_destroy", "nq_model_weight_layout",
           "nq_model_create", "nq_model_destroy", "nq_neighbor_build", "nq_energy_forces",
           "nq_energy_forces_replicas", "nq_energy_forces_domain", "nq_ring_polymer", "nq_ring_polymer_noalloc", "nq_step",
           "nq_step_nvt", "nq_force_outliers",
           "nq_stats", "nq_ctx_graph_captures", "nq_edges_export", "nq_debug_export", "nq_ctx_set_workspace_budget", "nq_ctx_set_variant", "nq_ctx_set_path", "nq_autotune", "nq_model_set_choice", "nq_model_set_product_precision", "nq_timing",
           "nq_timing_report",
           "nq_status_str", "nq_last_error"]


class NQError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class ModelDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_bessel", C.c_int32), ("poly_p", C.c_int32),
                ("lmax", C.c_int32), ("n_layers", C.c_int32), ("channels", C.c_int32),
                ("n_twobody", C.c_int32), ("twobody", C.c_int32 * 4),
                ("n_latent", C.c_int32), ("latent", C.c_int32 * 4),
                ("n_edge", C.c_int32), ("edge", C.c_int32 * 4),
                ("r_cut", C.c_double), ("avg_num_neighbors", C.c_double), ("energy_scale", C.c_double),
                ("precision", C.c_int32)]


def make_desc(model, precision: str = "fp32") -> ModelDesc:
    """Fill the C description from any object with the model's attributes."""
    d = ModelDesc()
    for name in ("n_species", "n_bessel", "poly_p", "lmax", "n_layers", "channels"):
        setattr(d, name, int(getattr(model, name)))
    for name in ("twobody", "latent", "edge"):
        widths = list(getattr(model, name))
        if len(widths) > 4:
            raise ValueError(f"at most 4 {name} layers")
        setattr(d, "n_" + name, len(widths))
        arr = getattr(d, name)
        for k, w in enumerate(widths):
            arr[k] = int(w)
    d.r_cut = float(model.r_cut)
    d.avg_num_neighbors = float(model.avg_num_neighbors)
    d.energy_scale = float(model.energy_scale)
    # "mixed" is the split-BF16 model with some products overridden to plain
    # BF16 after creation (Potential does that)
    d.precision = PRECISION["bf16x3" if precision == "mixed" else precision]
    return d


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2303_08169_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    P = C.POINTER
    sig = {
        "nq_ctx_create": (C.c_int, [C.c_int, vp, P(vp)]),
        "nq_ctx_set_stream": (C.c_int, [vp, vp]),
        "nq_ctx_destroy": (None, [vp]),
        "nq_model_weight_layout": (C.c_int, [P(ModelDesc), P(i64), i32, P(i32), P(i64)]),
        "nq_model_create": (C.c_int, [vp, P(ModelDesc), P(dbl), i64, P(vp)]),
        "nq_model_destroy": (None, [vp]),
        "nq_neighbor_build": (C.c_int, [vp, vp, i64, P(dbl), dbl, dbl]),
        "nq_energy_forces": (C.c_int, [vp, vp, vp, vp, i64, P(dbl), vp, vp, vp]),
        "nq_energy_forces_replicas": (C.c_int, [vp, vp, vp, vp, i64, i64, P(dbl), vp, vp, vp]),
        "nq_energy_forces_domain": (C.c_int, [vp, vp, vp, vp, i64, i64, P(dbl), vp, vp, vp]),
        "nq_ring_polymer": (C.c_int, [vp, vp, vp, i64, i64, P(dbl), dbl, vp, vp]),
        "nq_ring_polymer_noalloc": (C.c_int, [vp, vp, vp, i64, i64, P(dbl), dbl, vp, vp]),
        "nq_step": (C.c_int, [vp, vp, vp, vp, vp, vp, i64, P(dbl), dbl, i32, vp, vp, vp]),
        "nq_step_nvt": (C.c_int, [vp, vp, vp, vp, vp, vp, i64, P(dbl), dbl, i32, dbl, dbl, vp, vp, vp, vp, vp]),
        "nq_force_outliers": (C.c_int, [vp, vp, i64, dbl, vp]),
        "nq_stats": (C.c_int, [vp, P(i64), P(i64)]),
        "nq_ctx_graph_captures": (C.c_int, [vp, P(i64)]),
        "nq_edges_export": (C.c_int, [vp, vp, vp, i64, P(i64)]),
        "nq_debug_export": (C.c_int, [vp, vp, C.c_char_p, vp, i64, P(i64), P(i64)]),
        "nq_ctx_set_workspace_budget": (C.c_int, [vp, i64]),
        "nq_ctx_set_variant": (C.c_int, [vp, C.c_int32]),
        "nq_ctx_set_path": (C.c_int, [vp, C.c_int32]),
        "nq_model_set_choice": (C.c_int, [vp, C.c_char_p, C.c_int32]),
        "nq_model_set_product_precision": (C.c_int, [vp, C.c_char_p, C.c_int32]),
        "nq_autotune": (C.c_int, [vp, vp, vp, vp, i64, P(dbl), i32, C.c_char_p, i64, P(i64)]),
        "nq_timing": (C.c_int, [vp, C.c_int]),
        "nq_timing_report": (C.c_int, [vp, C.c_char_p, i64, P(i64)]),
        "nq_status_str": (C.c_char_p, [C.c_int]),
        "nq_last_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status: int, ctx=None):
    if status != NQ_OK:
        msg = lib().nq_last_error(ctx).decode()
        raise NQError(status, msg)


def weight_layout(desc: ModelDesc):
    """[(fan_in, fan_out), ...] the library expects, and the total count."""
    L = lib()
    nseg, ntot = C.c_int32(0), C.c_int64(0)
    check(L.nq_model_weight_layout(C.byref(desc), None, 0, C.byref(nseg), C.byref(ntot)))
    buf = (C.c_int64 * (2 * nseg.value))()
    check(L.nq_model_weight_layout(C.byref(desc), buf, nseg.value, C.byref(nseg), C.byref(ntot)))
    return [(buf[2 * k], buf[2 * k + 1]) for k in range(nseg.value)], ntot.value
