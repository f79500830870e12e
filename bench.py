#!/usr/bin/env python3
"""Throughput of one energy+force evaluation (one MD step's force call) on one MI355X.

Workload: 27,648-atom synthetic liquid NH3 (6,912 molecules, box 65.9 A), the
l <= 2 model with 2 layers and 32 channels, cutoff 6 A (about 2.4 M directed
edges). A step is one call of nq_energy_forces: edge list from the neighbour
list, the equivariant edge model forward and its hand-written adjoint, force
gather and compensated FP64 energy. Inputs are resident in HBM before timing.
The reported mode is split BF16 on the automatic path (the layered kernels
with the two-body MLP as one kernel per direction).

Passes over the reported mode, in this order:
  1. headline: W warm-up calls, then K calls timed back to back between two
     device synchronisations (no per-kernel events inside);
  2. median: the median of --median-calls calls, each between two HIP events;
  3. breakdown: --breakdown-steps calls with the library's per-kernel HIP
     events, for the roofline position of the dominant kernel.
The other modes (--compare) are timed as in pass 1 with fewer calls. The FP64
oracle is timed on the host cores on a bounded sample of the same system and
on the whole 1,024-atom system (all threads and one thread), and gives the
energy/force error of every mode.

Prints ONE JSON line. --profile-evals runs only the reported mode between two
marker kernels, for rocprofv3 (see paper_2303_08169_amd/profile_summary.py).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s (E+F) at 27,648-atom NH3, lmax=2; force RMS err vs FP64 oracle"
# MI355X published dense peaks (TFLOP/s) and HBM bandwidth (GB/s)
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}
VALU_FP32_TFLOPS = 157.3
HBM_GBS = 8000.0
DTYPE = {"fp32": "fp32", "bf16": "bf16", "bf16x3": "bf16x3", "mixed": "bf16x3+bf16"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Work per edge of the method (paper Sec. 2.1; input gradients only)
# ---------------------------------------------------------------------------

def tp_paths(lmax):
    """Coupling paths (l1, l2 -> l3) of the tensor product that keep even
    parity, the number of output components and the number of scalar outputs."""
    paths = [(a, b, c) for a in range(lmax + 1) for b in range(lmax + 1) for c in range(abs(a - b), min(a + b, lmax) + 1)
             if (a + b + c) % 2 == 0]
    return paths, sum(2 * c + 1 for _, _, c in paths), sum(1 for *_, c in paths if c == 0)


def method_mac_per_edge(model):
    """Multiply-adds per edge of the forward matrix products, the channel
    mixing included: two-body MLP, tensor-feature and environment embeddings,
    latent MLPs, mixing of the tensor-product outputs (every layer but the
    last) and the edge-energy MLP."""
    def mlp(dims):
        return sum(a * b for a, b in zip(dims[:-1], dims[1:]))

    D, C, T = model.twobody[-1], model.channels, model.n_layers
    _, nt, nscal = tp_paths(model.lmax)
    nw = C * (model.lmax + 1)
    mac = mlp([2 * model.n_species + model.n_bessel] + list(model.twobody))
    mac += D * nw * (1 + T)
    mac += T * mlp([D + nscal * C] + list(model.latent))
    mac += (T - 1) * nt * C * C
    mac += mlp([D] + list(model.edge) + [1])
    return mac


def algorithmic_bytes(n_atoms, n_edges, n_weights, precision):
    """HBM bytes one evaluation cannot avoid: positions read, forces written
    (FP64), species, the neighbour list and its reverse table (4 B each per
    edge) and the weights once (BF16 hi+lo for bf16x3)."""
    wbytes = {"fp32": 4, "bf16": 2, "bf16x3": 4, "mixed": 4}[precision]
    return n_atoms * (24 + 24 + 4) + 8 * n_edges + wbytes * n_weights


# ---------------------------------------------------------------------------
# Timing passes
# ---------------------------------------------------------------------------

def timed_calls(pot, P, Z, box, steps, warmup):
    """Mean wall time of `steps` back-to-back calls between two synchronisations."""
    import torch

    E = torch.empty(1, dtype=torch.float64, device=P.device)
    F = torch.empty_like(P)
    for _ in range(warmup):
        pot.energy_forces(P, Z, box, forces=F, energy=E)
    torch.cuda.synchronize()
    pot.stats()  # raises on capacity or numeric flags
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pot.energy_forces(P, Z, box, forces=F, energy=E)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ne, _ = pot.stats()
    return (t1 - t0) / steps, ne, E, F


def median_call(pot, P, Z, box, calls):
    """Median device time of one call, each between two HIP events on the stream."""
    import torch

    E = torch.empty(1, dtype=torch.float64, device=P.device)
    F = torch.empty_like(P)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        pot.energy_forces(P, Z, box, forces=F, energy=E)
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return ms[len(ms) // 2] if calls % 2 else 0.5 * (ms[calls // 2 - 1] + ms[calls // 2])


def breakdown(pot, P, Z, box, steps):
    """The library's per-kernel HIP-event report over `steps` calls."""
    import ctypes as C

    import torch
    from paper_2303_08169_amd import binding as B

    E = torch.empty(1, dtype=torch.float64, device=P.device)
    F = torch.empty_like(P)
    torch.cuda.synchronize()
    B.check(pot.lib.nq_timing(pot._ctx, 1), pot._ctx)
    for _ in range(steps):
        pot.energy_forces(P, Z, box, forces=F, energy=E)
    torch.cuda.synchronize()
    B.check(pot.lib.nq_timing(pot._ctx, 0), pot._ctx)
    buf = C.create_string_buffer(1 << 20)
    n = C.c_int64(0)
    B.check(pot.lib.nq_timing_report(pot._ctx, buf, len(buf), C.byref(n)), pot._ctx)
    return json.loads(buf.value.decode())


# ---------------------------------------------------------------------------
# Roofline
# ---------------------------------------------------------------------------

def source_digest():
    """SHA-256 over the library sources: counter figures recorded for one
    state of the kernels are used only while the sources are unchanged."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_08169_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def recorded_counters(precision, path, workload):
    """The committed counter summary for this mode and workload
    (profiles/counters_<workload>_<precision>_<path>.json), or None when there
    is none or the sources changed since it was taken."""
    f = os.path.join(ROOT, "profiles", f"counters_{workload}_{precision}_{path}.json")
    try:
        with open(f) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    return rec if rec.get("source_sha256") == source_digest() else None


def roofline(report, steps, precision, path, workload, n_atoms, n_edges, n_weights, model, ms_step):
    """Roofline position of the kernel with the largest share of the step.

    The method's work is dense per-edge matrix products, so the bound is the
    matrix cores at the peak of the contraction dtype (BF16 for bf16 and
    bf16x3, FP32 for fp32). `achieved` counts the method's FLOPs (the products
    of the model, input gradients only: a split-BF16 product is one product,
    not three). Also reported: the matrix-core fraction counting the three
    split products, the vector-ALU fraction of the kernel's non-matrix FLOPs,
    the HBM fraction of its counter bytes, and the step as a whole against the
    matrix-core floor of the method's FLOPs."""
    import re

    ks = report["kernels"]
    # launches of one kernel on the same shape in different layers count as
    # one kernel (the latent products of layers 1 and 2 run the same code on
    # the same sizes)
    groups = {}
    for k in ks:
        key = (re.sub(r"\d+", "#", k["name"]), round(k["flop_per_launch"]), round(k["bytes_per_launch"]))
        g = groups.setdefault(key, {"names": [], "ms_total": 0.0, "count": 0, "flop_per_launch": k["flop_per_launch"],
                                    "mfma_flop_per_launch": k.get("mfma_flop_per_launch", 0.0)})
        g["names"].append(k["name"])
        g["ms_total"] += k["ms_total"]
        g["count"] += k["count"]
    dom = max(groups.values(), key=lambda g: g["ms_total"])
    dom["name"] = "+".join(dom["names"])
    avg_s = dom["ms_total"] / dom["count"] * 1e-3
    mfma = dom["mfma_flop_per_launch"]
    valu = dom["flop_per_launch"] - mfma
    cdt = "fp32" if precision == "fp32" else "bf16"
    peak = MFMA_PEAK_TFLOPS[cdt]
    from paper_2303_08169_amd.potential import MIXED_BF16
    passes = 3 if precision == "bf16x3" or (precision == "mixed" and dom["names"][0] not in MIXED_BF16) else 1
    out = {"bound": "mfma", "achieved": mfma / avg_s / 1e12, "peak": peak, "unit": "TFLOP/s"}
    out["frac"] = out["achieved"] / peak
    rec = recorded_counters(precision, path, workload)
    members = [rec.get("spans", {}).get(n) for n in dom["names"]] if rec else [None]
    kc = None
    if all(m and "hbm_bytes_per_launch" in m for m in members):
        kc = {f: sum(m[f] for m in members) / len(members)
              for f in ("hbm_bytes_per_launch", "avg_ms_trace", "mfma_busy", "valu_busy", "wait_any",
                        "lds_bank_conflict_per_lds_inst") if all(f in m for m in members)}
    out["traffic"] = kc["hbm_bytes_per_launch"] if kc else None
    out["kernel"] = dom["name"]
    out["avg_launch_ms"] = avg_s * 1e3
    out["launches_per_step"] = dom["count"] / steps
    out["share_of_step"] = dom["ms_total"] / sum(k["ms_total"] for k in ks)
    out["method_flop_per_launch"] = mfma
    out["fractions"] = {
        "mfma_method": out["frac"],
        "mfma_issued": out["frac"] * passes,
        "valu": valu / avg_s / 1e12 / VALU_FP32_TFLOPS,
        "hbm_counters": (kc["hbm_bytes_per_launch"] / avg_s / 1e9 / HBM_GBS) if kc else None,
    }
    if kc:
        out["counters"] = {k: kc[k] for k in ("mfma_busy", "valu_busy", "wait_any", "lds_bank_conflict_per_lds_inst",
                                              "avg_ms_trace") if k in kc}
        out["counters_source"] = "profiles/" + rec["source_file"]
    flop_edge = 4.0 * method_mac_per_edge(model)
    step_flop = flop_edge * n_edges
    alg = algorithmic_bytes(n_atoms, n_edges, n_weights, precision)
    floor_ms = step_flop / (peak * 1e12) * 1e3
    out["step"] = {
        "method_flop_per_edge": flop_edge,
        "method_flop": step_flop,
        "mfma_floor_ms": floor_ms,
        "frac_mfma": floor_ms / ms_step,
        "algorithmic_bytes": alg,
        "hbm_counter_bytes": rec["hbm_bytes_per_step"] if rec else None,
        "counter_over_algorithmic": (rec["hbm_bytes_per_step"] / alg) if rec else None,
        "valu_frac_sum": sum(k["flop_per_launch"] - k.get("mfma_flop_per_launch", 0.0) for k in ks)
        / steps / (ms_step * 1e-3) / 1e12 / VALU_FP32_TFLOPS,
    }
    return out


# ---------------------------------------------------------------------------
# Oracle on the host cores
# ---------------------------------------------------------------------------

def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        return os.cpu_count()


def cpu_sample(pos, z, box, model, w, n_atoms_sample, seed=300):
    """Oracle on the centres within the cutoff of a few random atoms: exact
    forces on those atoms and exact E_i of every evaluated centre."""
    import numpy as np

    import oracle

    rng = np.random.default_rng(seed)
    atoms = rng.choice(len(pos), n_atoms_sample, replace=False)
    cs = [atoms]
    for a in atoms:
        _, nb = oracle.edge_list(pos, box, model.r_cut, centers=[a])
        cs.append(nb)
    centers = np.unique(np.concatenate(cs))
    oracle.energy_forces(pos, z, box, model, w, centers=centers[:8])  # warm-up
    t0 = time.perf_counter()
    E, F, Ei = oracle.energy_forces(pos, z, box, model, w, centers=centers, atom_energy=True)
    dt = time.perf_counter() - t0
    return dict(atoms=atoms, centers=centers, F=F, Ei=Ei, seconds=dt, cores=_threads())


def cpu_full_c1(precision):
    """The oracle on the whole 1,024-atom system (same model): all threads,
    then one thread. Returns atom-steps/s for both."""
    from threadpoolctl import threadpool_limits

    import oracle
    from paper_2303_08169_amd import binding as B
    from synth import config, make_system, weight_blob

    cf = config("nh3_1024_l2")
    pos, z, box = make_system(cf.n_atoms, cf.seed)
    segs, _ = B.weight_layout(B.make_desc(cf.model, precision))
    w = weight_blob(cf.weight_seed, segs)
    out = {}
    for name, lim in (("all_threads", None), ("one_thread", 1)):
        if lim is None:
            cores = _threads()
            t0 = time.perf_counter()
            oracle.energy_forces(pos, z, box, cf.model, w)
            dt = time.perf_counter() - t0
        else:
            with threadpool_limits(limits=1):
                cores = 1
                t0 = time.perf_counter()
                oracle.energy_forces(pos, z, box, cf.model, w)
                dt = time.perf_counter() - t0
        out[name] = {"value": cf.n_atoms / dt, "seconds": dt, "cores": cores}
        log(f"oracle 1,024 atoms ({name}): {dt:.1f} s")
    return out


def errors(sample, F_gpu, Ei_gpu):
    import numpy as np

    a, c = sample["atoms"], sample["centers"]
    dF = F_gpu[a] - sample["F"][a]
    f_err = float(np.linalg.norm(dF) / np.linalg.norm(sample["F"][a]))
    e_err = float(np.linalg.norm(Ei_gpu[c] - sample["Ei"][c]) / np.linalg.norm(sample["Ei"][c]))
    e_sum = float(abs(Ei_gpu[c].sum() - sample["Ei"][c].sum()) / abs(sample["Ei"][c].sum()))
    return {"force_rel_rms": f_err, "atom_energy_rel_rms": e_err, "energy_rel_sampled": e_sum,
            "sample_atoms": int(len(a)), "sample_centres": int(len(c))}


# ---------------------------------------------------------------------------
# Other workloads
# ---------------------------------------------------------------------------

def md_run(args, cf, pos, z, box, dt_fs=0.5, chunk=50):
    """NVE run through nq_step in chunks of `chunk` graph-replayed steps; stops at
    the first chunk that reports an error (e.g. two atoms closer than 0.1 A)."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.binding import NQError
    from paper_2303_08169_amd.potential import Potential
    from synth import weight_blob
    from synth.nh3 import masses, maxwell_boltzmann

    prec = args.precision
    model = dataclasses.replace(cf.model, energy_scale=cf.model.energy_scale * args.md_energy_scale)
    segs, _ = B.weight_layout(B.make_desc(model, prec))
    w = weight_blob(cf.weight_seed, segs)
    pot = Potential(model, w, prec)
    pot.set_path(args.path)
    dev = torch.device("cuda", 0)
    P = torch.tensor(pos, device=dev)
    V = torch.tensor(maxwell_boltzmann(z, args.md_temp, 200), device=dev)
    IM = torch.tensor(1.0 / masses(z), device=dev)
    Z = torch.tensor(z, dtype=torch.int32, device=dev)
    pot.neighbor_build(P, box, skin=args.md_skin)
    E, F = pot.energy_forces(P, Z, box)
    if not args.no_autotune and args.path != "fused":
        # the captured step replays the tuned kernel choice
        pot.autotune(P, Z, box, reps=5)
    ep = torch.zeros(chunk, dtype=torch.float64, device=dev)
    ek = torch.zeros(chunk, dtype=torch.float64, device=dev)
    epot, ekin, err = [], [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < args.md:
        n = min(chunk, args.md - done)
        try:
            pot.step(P, V, IM, Z, box, dt_fs, n, F, ep, ek)
        except NQError as e:
            err = str(e)
            break
        epot.extend(ep[:n].cpu().tolist())
        ekin.extend(ek[:n].cpu().tolist())
        done += n
        log(f"md: {done} steps, E_tot/N = {(epot[-1] + ekin[-1]) / cf.n_atoms:.6f} eV")
    t1 = time.perf_counter()
    _, rebuilds = pot.stats() if err is None else (0, -1)
    etot = np.array(epot) + np.array(ekin)
    out = {"md_steps_requested": args.md, "md_steps_done": done, "dt_fs": dt_fs, "precision": prec,
           "path": args.path, "workload": args.workload, "atoms": cf.n_atoms, "T0_K": args.md_temp,
           "energy_scale_factor": args.md_energy_scale, "skin_A": args.md_skin, "error": err,
           "rebuilds": rebuilds}
    if done:
        t = np.arange(1, done + 1) * dt_fs * 1e-3  # ps
        slope = np.polyfit(t, (etot - etot[0]) / cf.n_atoms * 1e3, 1)[0] if done > 2 else 0.0
        out.update({"atom_steps_per_s": cf.n_atoms * done / (t1 - t0), "ms_per_step": (t1 - t0) / done * 1e3,
                    "drift_meV_per_atom_per_ps": float(slope),
                    "max_abs_dE_per_atom_meV": float(np.abs(etot - etot[0]).max() / cf.n_atoms * 1e3),
                    "T_final_K": float(2 * ekin[-1] / (3 * cf.n_atoms - 3) / 8.617333262e-5)})
    print(json.dumps(out), flush=True)
    pot.close()


def replicas_run(args, cf, pos, z, box, temperature=300.0):
    """Path-integral workload: args.replicas perturbed replicas (beads) of the
    system evaluated in one nq_energy_forces_replicas call plus the ring-polymer
    springs, against the same replicas evaluated one call each."""
    import numpy as np
    import torch

    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.potential import Potential
    from synth import weight_blob
    from synth.nh3 import masses

    R = args.replicas
    segs, _ = B.weight_layout(B.make_desc(cf.model, args.precision))
    w = weight_blob(cf.weight_seed, segs)
    pot = Potential(cf.model, w, args.precision)
    pot.set_path(args.path)
    rng = np.random.default_rng(400)
    reps = np.stack([(pos + rng.normal(scale=0.02, size=pos.shape)) % box for _ in range(R)])
    dev = torch.device("cuda", 0)
    P = torch.tensor(reps, device=dev)
    Z = torch.tensor(np.tile(z, (R, 1)), dtype=torch.int32, device=dev)
    IM = torch.tensor(1.0 / masses(z), device=dev)

    def batched():
        E, F = pot.energy_forces_replicas(P, Z, box)
        return pot.ring_polymer(P, IM, box, temperature, F)

    singles = [(P[r].contiguous(), Z[r].contiguous()) for r in range(R)]

    def one_by_one():
        for p_, z_ in singles:
            pot.energy_forces(p_, z_, box)

    out = {"metric": "atom-steps/s (E+F of all replicas + ring-polymer springs)", "workload": args.workload,
           "replicas": R, "atoms_per_replica": cf.n_atoms, "precision": args.precision, "path": args.path,
           "data": "synthetic"}
    for name, fn in (("batched", batched), ("one_call_per_replica", one_by_one)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        out[name] = {"ms_per_step": dt * 1e3, "atom_steps_per_s": R * cf.n_atoms / dt}
        log(f"{name}: {dt * 1e3:.3f} ms per step of {R} replicas")
    print(json.dumps(out), flush=True)
    pot.close()


def sensitivity_run(args):
    """Error of the energy and forces of the 1,024-atom system against the
    FP64 oracle when single products run in plain BF16 inside the split-BF16
    model (and in split-BF16 inside the plain-BF16 model), then a greedy
    mixture: products move to plain BF16 in order of their error while the
    force error stays under --mix-force and the energy error under --mix-energy."""
    import numpy as np
    import torch

    import oracle  # noqa: F401  (test infrastructure: the oracle comparison of this mode)
    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.potential import Potential
    from synth import config, make_system, weight_blob

    cf = config("nh3_1024_l2")
    pos, z, box = make_system(cf.n_atoms, cf.seed)
    segs, _ = B.weight_layout(B.make_desc(cf.model, "bf16x3"))
    w = weight_blob(cf.weight_seed, segs)
    log("oracle on 1,024 atoms ...")
    E0, F0 = oracle.energy_forces(pos, z, box, cf.model, w)
    dev = torch.device("cuda", 0)
    P = torch.tensor(pos, device=dev)
    Z = torch.tensor(z, dtype=torch.int32, device=dev)
    pot = Potential(cf.model, w, "bf16x3")
    pot.set_path("layered")
    sites = [s["name"] for s in pot.autotune(P, Z, box, reps=1)["sites"]]
    sites += [f"tp_{d}{t}" for t in range(1, cf.model.n_layers) for d in ("fwd", "bwd")]

    def err(over):
        pot.set_product_precision({s: None for s in sites})
        pot.set_product_precision(over)
        E, F = pot.energy_forces(P, Z, box)
        torch.cuda.synchronize()
        F = F.cpu().numpy()
        return {"force_rel_rms": float(np.linalg.norm(F - F0) / np.linalg.norm(F0)),
                "energy_rel": float(abs(E.item() - E0) / abs(E0))}

    out = {"workload": "nh3_1024_l2", "sites": sites, "bf16x3": err({}),
           "bf16": err({s: "bf16" for s in sites}), "one_bf16": {}, "one_bf16x3_in_bf16": {}}
    for s in sites:
        out["one_bf16"][s] = err({s: "bf16"})
        out["one_bf16x3_in_bf16"][s] = err({**{t: "bf16" for t in sites}, s: "bf16x3"})
        log(f"{s:<16} alone in bf16: {out['one_bf16'][s]}   alone in bf16x3: {out['one_bf16x3_in_bf16'][s]}")
    order = sorted(sites, key=lambda s: out["one_bf16"][s]["force_rel_rms"])
    chosen, steps = [], []
    for s in order:
        e = err({t: "bf16" for t in chosen + [s]})
        ok = e["force_rel_rms"] <= args.mix_force and e["energy_rel"] <= args.mix_energy
        steps.append({"site": s, "accepted": ok, **e})
        if ok:
            chosen.append(s)
    out["greedy"] = steps
    out["mix_bf16_sites"] = chosen
    out["mix"] = err({t: "bf16" for t in chosen})
    pot.close()
    print(json.dumps(out), flush=True)


def profile_run(args, pot, P, Z, box):
    """Calls for rocprofv3: two warm-ups, a marker kernel, --profile-evals
    calls with the library's span events on, a marker kernel. Writes the span
    order and sizes (what profile_summary.py needs to name the dispatches)."""
    import torch

    E = torch.empty(1, dtype=torch.float64, device=P.device)
    F = torch.empty_like(P)
    for _ in range(2):
        pot.energy_forces(P, Z, box, forces=F, energy=E)
    torch.cuda.synchronize()
    torch.cuda._sleep(1000)  # marker: the evaluations start after it
    rep = breakdown(pot, P, Z, box, args.profile_evals)
    torch.cuda._sleep(1000)  # marker: the evaluations end before it
    torch.cuda.synchronize()
    ne, _ = pot.stats()
    out = {"workload": args.workload, "precision": args.precision, "path": args.path, "evals": args.profile_evals,
           "edges": ne, "spans": [k["name"] for k in rep["kernels"]],
           "span_counts": [k["count"] for k in rep["kernels"]], "source_sha256": source_digest()}
    if args.profile_out:
        with open(args.profile_out, "w") as fh:
            json.dump(out, fh)
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--median-calls", type=int, default=100)
    ap.add_argument("--breakdown-steps", type=int, default=10)
    ap.add_argument("--workload", default="nh3_27648_l2")
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16", "bf16x3", "mixed"])
    ap.add_argument("--path", default="auto", choices=["auto", "fused", "layered"],
                    help="evaluation path of the reported mode")
    ap.add_argument("--compare", default="mixed,bf16x3:layered,bf16x3:fused,fp32,bf16",
                    help="other modes timed alongside: precision[:path], comma separated")
    ap.add_argument("--cpu-sample-atoms", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="skip the tile-shape autotuner")
    ap.add_argument("--save-tuned", default="", metavar="FILE", help="write the autotuned kernel variants here")
    ap.add_argument("--load-tuned", default="", metavar="FILE",
                    help="use the kernel variants of a --save-tuned file instead of autotuning")
    ap.add_argument("--profile-evals", type=int, default=0, metavar="K",
                    help="instead: K calls of the reported mode between marker kernels, for rocprofv3")
    ap.add_argument("--profile-out", default="", help="with --profile-evals: write the span order here")
    ap.add_argument("--sensitivity", action="store_true",
                    help="instead: per-product precision study on the 1,024-atom system against the oracle")
    ap.add_argument("--mix-force", type=float, default=5e-4, help="force error bound of --sensitivity's mixture")
    ap.add_argument("--mix-energy", type=float, default=8e-6, help="energy error bound of --sensitivity's mixture")
    ap.add_argument("--md", type=int, default=0, metavar="STEPS",
                    help="instead: NVE velocity-Verlet run of STEPS steps (dt 0.5 fs) through nq_step")
    ap.add_argument("--md-temp", type=float, default=300.0, help="initial temperature (K) of --md")
    ap.add_argument("--md-energy-scale", type=float, default=1.0,
                    help="factor on the model's energy scale for --md (random weights have no repulsive core)")
    ap.add_argument("--md-skin", type=float, default=1.0, help="neighbour-list skin (A) for --md")
    ap.add_argument("--replicas", type=int, default=0, metavar="R",
                    help="instead: R path-integral replicas of the workload in one call (with ring-polymer springs)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calib:
        import torch
        src = torch.ones(args.copy_calib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": src.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; no multi-GPU path is built "
                                   "(spatial decomposition is a design note only)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.potential import Potential
    from synth import config, make_system, weight_blob

    if args.sensitivity:
        return sensitivity_run(args)
    cf = config(args.workload)
    pos, z, box = make_system(cf.n_atoms, cf.seed)
    if args.md:
        return md_run(args, cf, pos, z, box)
    if args.replicas:
        return replicas_run(args, cf, pos, z, box)
    dev = torch.device("cuda", 0)
    P = torch.tensor(pos, device=dev)
    Z = torch.tensor(z, dtype=torch.int32, device=dev)
    log(f"workload {args.workload}: {cf.n_atoms} atoms, box {box:.3f} A")

    loaded = {}
    if args.load_tuned:
        with open(args.load_tuned) as fh:
            loaded = json.load(fh)
    saved = {}

    def make(prec, path):
        segs, nw = B.weight_layout(B.make_desc(cf.model, prec))
        pot = Potential(cf.model, weight_blob(cf.weight_seed, segs), prec)
        pot.set_path(path)
        tuned, mode = None, f"{prec}:{path}"
        if mode in loaded:
            tuned = loaded[mode]
            pot.set_choice(tuned)
            log(f"{mode}: kernel variants from {args.load_tuned}")
        elif not args.no_autotune and path != "fused":
            rep = pot.autotune(P, Z, box, reps=5)
            tuned = {s["name"]: s["chosen"] for s in rep["sites"]}
            log(f"{mode}: autotuned kernel variants {tuned}")
        if tuned is not None and args.save_tuned:
            saved[mode] = tuned
            with open(args.save_tuned, "w") as fh:
                json.dump(saved, fh)
        return pot, nw, tuned

    if args.profile_evals:
        pot, _, _ = make(args.precision, args.path)
        profile_run(args, pot, P, Z, box)
        pot.close()
        return

    main_mode = f"{args.precision}:{args.path}"
    modes = [main_mode]
    for m in args.compare.split(","):
        if m:
            m = m if ":" in m else m + ":auto"
            if m not in modes:
                modes.append(m)
    results, main_extra = {}, {}
    w_main = None
    for mode in modes:
        prec, path = mode.split(":")
        pot, nw, tuned = make(prec, path)
        if mode == main_mode:
            dt, ne, E, F = timed_calls(pot, P, Z, box, args.steps, args.warmup)
            log(f"{mode}: {dt * 1e3:.3f} ms/step over {args.steps} calls")
            med = median_call(pot, P, Z, box, args.median_calls)
            log(f"{mode}: median {med:.3f} ms over {args.median_calls} calls")
            rep = breakdown(pot, P, Z, box, args.breakdown_steps)
            main_extra = dict(median_ms=med, report=rep, n_weights=nw, tuned=tuned)
            w_main = weight_blob(cf.weight_seed, B.weight_layout(B.make_desc(cf.model, prec))[0])
            steps = args.steps
        else:
            steps = max(3, min(args.steps, 10))
            dt, ne, E, F = timed_calls(pot, P, Z, box, steps, 3)
        _, _, Ei = pot.energy_forces(P, Z, box, atom_energy=True)
        torch.cuda.synchronize()
        results[mode] = dict(dt=dt, edges=ne, E=E.item(), F=F.cpu().numpy(), Ei=Ei.cpu().numpy(), steps=steps)
        log(f"{mode}: {dt * 1e3:.3f} ms/step, {cf.n_atoms / dt:.4g} atom-steps/s, {ne} edges, E={E.item():.6f}")
        pot.close()
        del pot
        torch.cuda.empty_cache()

    r0 = results[main_mode]
    line = {
        "metric": METRIC,
        "value": cf.n_atoms / r0["dt"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": r0["steps"],
        "warmup": args.warmup,
        "ms_per_step": r0["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "atoms": cf.n_atoms, "edges": r0["edges"],
                   "lmax": cf.model.lmax, "layers": cf.model.n_layers, "channels": cf.model.channels,
                   "r_cut": cf.model.r_cut, "precision": args.precision, "path": args.path,
                   "parallelism": "single GPU (one spatial domain)"},
        "median": {"calls": args.median_calls, "ms_per_call": main_extra["median_ms"],
                   "value": cf.n_atoms / (main_extra["median_ms"] * 1e-3)},
        "roofline": roofline(main_extra["report"], args.breakdown_steps, args.precision, args.path, args.workload,
                             cf.n_atoms, r0["edges"], main_extra["n_weights"], cf.model, r0["dt"] * 1e3),
    }
    modes_out = {m: {"ms_per_step": r["dt"] * 1e3, "value": cf.n_atoms / r["dt"]} for m, r in results.items()}
    if not args.no_cpu_baseline:
        import oracle  # noqa: F401  (test infrastructure: only this leg touches it)
        log("oracle sample on host cores ...")
        smp = cpu_sample(pos, z, box, cf.model, w_main, args.cpu_sample_atoms)
        line["cpu_baseline"] = {
            "value": len(smp["centers"]) / smp["seconds"], "unit": "atom-steps/s", "cores": smp["cores"],
            "kind": "oracle",
            "sample": f"E+F of the {len(smp['centers'])} centres within r_c of {len(smp['atoms'])} random atoms "
                      f"(seed 300) of the same 27,648-atom system, FP64 NumPy, {smp['seconds']:.1f} s after a "
                      f"warm-up on 8 centres"}
        line["cpu_baseline"]["full_1024_atoms"] = cpu_full_c1(args.precision)
        for mode, r in results.items():
            modes_out[mode].update(errors(smp, r["F"], r["Ei"]))
    line["modes"] = modes_out
    if main_extra["tuned"]:
        line["autotune"] = main_extra["tuned"]
    rep = main_extra["report"]
    line["kernels_top"] = sorted(
        [{"name": k["name"], "ms_per_step": k["ms_total"] / args.breakdown_steps,
          "launches_per_step": k["count"] / args.breakdown_steps,
          "method_tflops": k.get("mfma_flop_per_launch", 0.0) / (k["ms_total"] / k["count"] * 1e-3) / 1e12}
         for k in rep["kernels"]], key=lambda k: -k["ms_per_step"])
    line["breakdown_ms_per_step"] = sum(k["ms_total"] for k in rep["kernels"]) / args.breakdown_steps
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
