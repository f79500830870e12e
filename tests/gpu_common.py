"""Shared helpers of the GPU tests (inputs come from synth/, references from oracle/)."""
import json
import os

import numpy as np

import oracle
from synth import config, make_system, weight_blob

HERE = os.path.dirname(os.path.abspath(__file__))

# Tolerances. BF16X3 and BF16 follow the stated target for the BF16 path:
# forces within 1e-3 relative RMS and energies within 1e-5 relative of the FP64
# oracle (plain BF16 misses it and is only checked loosely). FP32: the products
# and sums run in FP32 (unit roundoff 6e-8) through ~10 chained stages with
# sums of up to ~100 terms, so 1e-5 relative is a safe bound for both.
TOL = {
    "fp32": {"energy": 1e-5, "force": 1e-5},
    "bf16x3": {"energy": 1e-5, "force": 1e-3},
    "bf16": {"energy": 1e-2, "force": 3e-2},
}


def system(name):
    cf = config(name)
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    w = weight_blob(cf.weight_seed, [(a, b) for _, a, b in oracle.weight_segments(cf.model)])
    return cf, pos, z, L, w


def golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as f:
        g = json.load(f)
    g["forces"] = np.asarray(g["forces"])
    g["atom_energy"] = np.asarray(g["atom_energy"])
    if "fd_forces" in g:
        g["fd_forces"] = np.asarray(g["fd_forces"])
    return g


def checksum(pos):
    return float(np.sum(pos * np.arange(1, pos.size + 1).reshape(pos.shape)))


def rel_rms(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def assert_forces_close(F, F_ref, tol, what=""):
    """Forces within tol of the reference: relative RMS over all components, and
    per atom max_a |F_a - F_ref,a| <= tol * RMS_a |F_ref,a| (one wrong atom cannot
    hide in the norm of a large system)."""
    F, F_ref = np.asarray(F).reshape(-1, 3), np.asarray(F_ref).reshape(-1, 3)
    rr = rel_rms(F, F_ref)
    assert rr <= tol, f"{what} force rel-RMS {rr:.3e} > {tol:.1e}"
    rms_ref = float(np.sqrt((F_ref * F_ref).sum(1).mean()))
    worst = float(np.linalg.norm(F - F_ref, axis=1).max())
    assert worst <= tol * rms_ref, f"{what} worst atom {worst:.3e} > {tol:.1e} * RMS|F| {rms_ref:.3e}"
