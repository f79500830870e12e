"""FP64 oracle NVE run of the 1,024-atom liquid-NH3 system at 300 K (writes c3_oracle_nve.json).

Evidence for the reading of the batched-MD workload: with random weights the
model has no repulsive core, so a velocity-Verlet run started from
Maxwell-Boltzmann velocities at 300 K brings atom pairs together until one pair
is closer than 0.1 A (the library's coincident-atom guard). This script shows
that the FP64 oracle's own trajectory does this (no GPU code involved): it
integrates with oracle.velocity_verlet one step at a time, oracle forces, and
records the closest pair distance, the temperature and the total energy per
step. Calls only oracle/ and synth/.

Usage: python tests/golden/c3_oracle_nve.py [max_steps]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import config, make_system, weight_blob  # noqa: E402
from synth.nh3 import masses, maxwell_boltzmann  # noqa: E402

KB = 8.617333262e-5


def closest_pair(pos, L):
    ei, ej = oracle.edge_list(pos, L, 1.5)
    if len(ei) == 0:
        return 1.5
    d = pos[ej] - pos[ei]
    d -= L * np.round(d / L)
    return float(np.sqrt((d * d).sum(1)).min())


def main(max_steps=120, dt=0.5, temperature=300.0):
    cf = config("nh3_1024_l2")
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    w = weight_blob(cf.weight_seed, [(a, b) for _, a, b in oracle.weight_segments(cf.model)])
    vel = maxwell_boltzmann(z, temperature, 200)
    m = masses(z)
    ndof = 3 * len(pos) - 3

    last = {}

    def ff(p):
        # velocity_verlet starts each call with F(pos) of the position the
        # previous call ended at: reuse it instead of evaluating it twice
        if "pos" in last and np.array_equal(last["pos"], p):
            return last["ef"]
        ef = oracle.energy_forces(p, z, L, cf.model, w)
        last["pos"], last["ef"] = p.copy(), ef
        return ef

    rec = {"workload": "nh3_1024_l2", "dt_fs": dt, "temperature_K": temperature,
           "velocity_seed": 200, "steps": [], "collapsed_at_step": None}
    E0, F0 = ff(pos)
    rec["epot0"] = E0
    rec["rms_force0"] = float(np.sqrt((F0 * F0).mean() * 3))
    rec["closest0"] = closest_pair(pos, L)
    t0 = time.time()
    for s in range(1, max_steps + 1):
        pos, vel, ep, ek = oracle.velocity_verlet(pos, vel, m, L, 1, dt, ff)
        dmin = closest_pair(pos, L)
        T = 2.0 * ek[0] / (ndof * KB)
        rec["steps"].append({"step": s, "closest": dmin, "temperature": T, "epot": ep[0], "ekin": ek[0]})
        print(f"step {s}: closest {dmin:.4f} A, T {T:.1f} K, Etot {ep[0] + ek[0]:.4f} eV ({time.time() - t0:.0f} s)",
              flush=True)
        if dmin < 0.1:
            rec["collapsed_at_step"] = s
            break
    with open(os.path.join(HERE, "c3_oracle_nve.json"), "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 120)
