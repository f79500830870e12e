#!/usr/bin/env python3
"""Throughput of one energy+force evaluation (one MD step's force call) on one MI355X.

Workload: 27,648-atom synthetic liquid NH3 (6,912 molecules, box 65.9 A), the
l <= 2 model with 2 layers and 32 channels, cutoff 6 A (about 2.4 M directed
edges). A step is one call of nq_energy_forces: edge list from the neighbour
list, the equivariant edge model forward and its hand-written adjoint, force
gather and compensated FP64 energy. Inputs are resident in HBM before timing.

Prints ONE JSON line with atom-steps/s (N atoms / time per step), the roofline
position of the dominant kernel (per-kernel HIP-event timings over the timed
region), the FP64 oracle timed on a bounded sample on the host cores, and the
energy/force error of each precision mode against that oracle sample.
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
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}  # dense MFMA, MI355X
VALU_FP32_TFLOPS = 157.3
HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_run(pot, P, Z, box, steps, warmup, timing=True):
    import ctypes as C

    import torch
    from paper_2303_08169_amd import binding as B

    E = torch.empty(1, dtype=torch.float64, device=P.device)
    F = torch.empty_like(P)
    for _ in range(warmup):
        pot.energy_forces(P, Z, box, forces=F, energy=E)
    torch.cuda.synchronize()
    pot.stats()  # raises on capacity or numeric flags
    if timing:
        B.check(pot.lib.nq_timing(pot._ctx, 1), pot._ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pot.energy_forces(P, Z, box, forces=F, energy=E)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    report = None
    if timing:
        B.check(pot.lib.nq_timing(pot._ctx, 0), pot._ctx)
        buf = C.create_string_buffer(1 << 20)
        n = C.c_int64(0)
        B.check(pot.lib.nq_timing_report(pot._ctx, buf, len(buf), C.byref(n)), pot._ctx)
        report = json.loads(buf.value.decode())
    ne, _ = pot.stats()
    return (t1 - t0) / steps, report, ne, E, F


def source_digest():
    """SHA-256 over the library sources: HBM counter figures recorded for one
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


def recorded_traffic(kernel, precision, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy-kernel calibration), or None
    when there is none for this kernel and configuration or the sources have
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    for k in rec.get("kernels", []):
        if (k.get("kernel") == kernel and rec.get("precision") == precision and rec.get("workload") == workload
                and rec.get("source_sha256") == source_digest()):
            return k.get("traffic_bytes")
    return None


def roofline(report, steps, precision, workload):
    """Roofline position of the kernel with the largest share of the step.

    The bound is whichever floor is highest for its algorithmic work: HBM
    bytes at 8 TB/s, matrix-core FLOPs at the dense peak of the precision
    (split-BF16 counts its three BF16 products), or FP32 vector FLOPs."""
    ks = report["kernels"]
    dom = max(ks, key=lambda k: k["ms_total"])
    avg_s = dom["ms_total"] / dom["count"] * 1e-3
    mfma = dom.get("mfma_flop_per_launch", 0.0)
    valu = dom["flop_per_launch"] - mfma
    passes = 3 if precision == "bf16x3" else 1
    floors = {
        "hbm": dom["bytes_per_launch"] / (HBM_GBS * 1e9),
        "mfma": mfma * passes / (PEAK_TFLOPS[precision] * 1e12),
        "alu": valu / (VALU_FP32_TFLOPS * 1e12),
    }
    bound = max(floors, key=floors.get)
    if bound == "hbm":
        out = {"bound": "hbm", "achieved": dom["bytes_per_launch"] / avg_s / 1e9, "peak": HBM_GBS, "unit": "GB/s"}
    elif bound == "mfma":
        out = {"bound": "mfma", "achieved": mfma * passes / avg_s / 1e12, "peak": PEAK_TFLOPS[precision],
               "unit": "TFLOP/s"}
    else:
        out = {"bound": "alu", "achieved": valu / avg_s / 1e12, "peak": VALU_FP32_TFLOPS, "unit": "TFLOP/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["traffic"] = recorded_traffic(dom["name"], precision, workload)
    out["kernel"] = dom["name"]
    out["avg_launch_ms"] = avg_s * 1e3
    out["algorithmic_bytes"] = dom["bytes_per_launch"]
    out["floors_ms"] = {k: v * 1e3 for k, v in floors.items()}
    out["launches_per_step"] = dom["count"] / steps
    out["share_of_step"] = dom["ms_total"] / sum(k["ms_total"] for k in ks)
    return out


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
    t0 = time.perf_counter()
    E, F, Ei = oracle.energy_forces(pos, z, box, model, w, centers=centers, atom_energy=True)
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    return dict(atoms=atoms, centers=centers, F=F, Ei=Ei, seconds=dt, cores=cores)


def errors(sample, F_gpu, Ei_gpu):
    import numpy as np

    a, c = sample["atoms"], sample["centers"]
    dF = F_gpu[a] - sample["F"][a]
    f_err = float(np.linalg.norm(dF) / np.linalg.norm(sample["F"][a]))
    e_err = float(np.linalg.norm(Ei_gpu[c] - sample["Ei"][c]) / np.linalg.norm(sample["Ei"][c]))
    e_sum = float(abs(Ei_gpu[c].sum() - sample["Ei"][c].sum()) / abs(sample["Ei"][c].sum()))
    return {"force_rel_rms": f_err, "atom_energy_rel_rms": e_err, "energy_rel_sampled": e_sum,
            "sample_atoms": int(len(a)), "sample_centres": int(len(c))}


def md_run(args, cf, pos, z, box, dt_fs=0.5, chunk=50):
    """NVE run through nq_step in chunks of `chunk` graph-replayed steps; stops at
    the first chunk that reports an error (e.g. two atoms closer than 0.1 A)."""
    import numpy as np
    import torch

    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.binding import NQError
    from paper_2303_08169_amd.potential import Potential
    from synth import weight_blob
    from synth.nh3 import masses, maxwell_boltzmann

    import dataclasses

    model = dataclasses.replace(cf.model, energy_scale=cf.model.energy_scale * args.md_energy_scale)
    segs, _ = B.weight_layout(B.make_desc(model, args.precision))
    w = weight_blob(cf.weight_seed, segs)
    pot = Potential(model, w, args.precision)
    dev = torch.device("cuda", 0)
    P = torch.tensor(pos, device=dev)
    V = torch.tensor(maxwell_boltzmann(z, args.md_temp, 200), device=dev)
    IM = torch.tensor(1.0 / masses(z), device=dev)
    Z = torch.tensor(z, dtype=torch.int32, device=dev)
    pot.neighbor_build(P, box, skin=args.md_skin)
    E, F = pot.energy_forces(P, Z, box)
    if not args.no_autotune:
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
    out = {"md_steps_requested": args.md, "md_steps_done": done, "dt_fs": dt_fs, "precision": args.precision,
           "workload": args.workload, "atoms": cf.n_atoms, "T0_K": args.md_temp,
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
           "replicas": R, "atoms_per_replica": cf.n_atoms, "precision": args.precision, "data": "synthetic"}
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="nh3_27648_l2")
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16", "bf16x3"])
    ap.add_argument("--path", default="auto", choices=["auto", "fused", "layered"],
                    help="evaluation path of the reported mode (auto: the fused kernel where compiled)")
    ap.add_argument("--compare", default="bf16x3:layered,fp32,bf16",
                    help="other modes timed alongside: precision[:path], comma separated")
    ap.add_argument("--cpu-sample-atoms", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="skip the tile-shape autotuner")
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

    import numpy as np
    import torch

    from paper_2303_08169_amd import binding as B
    from paper_2303_08169_amd.potential import Potential
    from synth import config, make_system, weight_blob

    cf = config(args.workload)
    pos, z, box = make_system(cf.n_atoms, cf.seed)
    if args.md:
        return md_run(args, cf, pos, z, box)
    if args.replicas:
        return replicas_run(args, cf, pos, z, box)
    desc = B.make_desc(cf.model, args.precision)
    segs, _ = B.weight_layout(desc)
    w = weight_blob(cf.weight_seed, segs)
    dev = torch.device("cuda", 0)
    P = torch.tensor(pos, device=dev)
    Z = torch.tensor(z, dtype=torch.int32, device=dev)
    log(f"workload {args.workload}: {cf.n_atoms} atoms, box {box:.3f} A")

    results = {}
    main_mode = args.precision + ("" if args.path == "auto" else ":" + args.path)
    modes = [main_mode] + [m for m in args.compare.split(",") if m and m != main_mode]
    tuned = {}
    for mode in modes:
        prec, _, path = mode.partition(":")
        pot = Potential(cf.model, w, prec)
        pot.set_path(path or "auto")
        if not args.no_autotune and (path == "layered" or prec == "fp32"):
            rep = pot.autotune(P, Z, box, reps=5)
            tuned[mode] = {s["name"]: s["chosen"] for s in rep["sites"]}
            log(f"{mode}: autotuned kernel variants {tuned[mode]}")
            for s_ in rep["sites"]:
                log(f"   {s_['name']:<16} " + " ".join(f"{t:.3f}" for t in s_["ms"]))
        steps = args.steps if mode == main_mode else max(3, min(args.steps, 10))
        dt, report, ne, E, F = timed_run(pot, P, Z, box, steps, args.warmup if mode == main_mode else 2)
        _, _, Ei = pot.energy_forces(P, Z, box, atom_energy=True)
        torch.cuda.synchronize()
        results[mode] = dict(dt=dt, report=report, edges=ne, E=E.item(), F=F.cpu().numpy(),
                             Ei=Ei.cpu().numpy(), steps=steps)
        log(f"{mode}: {dt * 1e3:.3f} ms/step, {cf.n_atoms / dt:.4g} atom-steps/s, {ne} edges, E={E.item():.6f}")
        pot.close()
        del pot
        torch.cuda.empty_cache()

    main_res = results[main_mode]
    line = {
        "metric": METRIC,
        "value": cf.n_atoms / main_res["dt"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": main_res["steps"],
        "warmup": args.warmup,
        "ms_per_step": main_res["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if args.precision.startswith("bf16") else "fp32",
        "data": "synthetic",
        "config": {"workload": args.workload, "atoms": cf.n_atoms, "edges": main_res["edges"],
                   "lmax": cf.model.lmax, "layers": cf.model.n_layers, "channels": cf.model.channels,
                   "r_cut": cf.model.r_cut, "precision": args.precision,
                   "parallelism": "single GPU (one spatial domain)"},
        "roofline": roofline(main_res["report"], main_res["steps"], args.precision, args.workload),
    }
    modes_out = {}
    for mode, r in results.items():
        modes_out[mode] = {"ms_per_step": r["dt"] * 1e3, "value": cf.n_atoms / r["dt"]}
    if not args.no_cpu_baseline:
        import oracle  # noqa: F401  (test infrastructure: only this leg touches it)
        log("oracle sample on host cores ...")
        smp = cpu_sample(pos, z, box, cf.model, w, args.cpu_sample_atoms)
        line["cpu_baseline"] = {
            "value": len(smp["centers"]) / smp["seconds"], "unit": "atom-steps/s", "cores": smp["cores"],
            "kind": "oracle",
            "sample": f"E+F of the {len(smp['centers'])} centres within r_c of {len(smp['atoms'])} random atoms "
                      f"(seed 300) of the same system, FP64 NumPy, {smp['seconds']:.1f} s"}
        for mode, r in results.items():
            modes_out[mode].update(errors(smp, r["F"], r["Ei"]))
    line["modes"] = modes_out
    if tuned:
        line["autotune"] = tuned.get(main_mode)
    line["kernels_top"] = sorted(
        [{"name": k["name"], "ms_per_step": k["ms_total"] / main_res["steps"], "launches": k["count"]}
         for k in main_res["report"]["kernels"]], key=lambda k: -k["ms_per_step"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
