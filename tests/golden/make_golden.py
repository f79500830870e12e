"""Writes the oracle reference values stored next to this script.

Calls only the FP64 oracle (oracle/) on the seeded synthetic systems of synth/:
  nh3_64_l1.json    64 atoms, l<=1 model: E, E_i, F
  nh3_1024_l2.json  1,024 atoms, l<=2 model: E, E_i, F, and central finite
                    differences (h = 1e-4 A) of the oracle energy for 32 atoms
                    chosen with seed 300 (only the centres within the cutoff of
                    an atom change when it moves, so E is summed over those).
The stored positions let a test detect a change of the input generator.
Run: python tests/golden/make_golden.py  (about ten minutes on 8 cores)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import config, make_system, weight_blob  # noqa: E402


def write(name, fd_atoms=0, h=1e-4):
    cf = config(name)
    pos, z, L = make_system(cf.n_atoms, cf.seed)
    w = weight_blob(cf.weight_seed, [(a, b) for _, a, b in oracle.weight_segments(cf.model)])
    E, F, Ei = oracle.energy_forces(pos, z, L, cf.model, w, atom_energy=True)
    out = {"config": name, "box": L, "pos_checksum": float(np.sum(pos * np.arange(1, pos.size + 1).reshape(pos.shape))),
           "energy": E, "atom_energy": Ei.tolist(), "forces": F.tolist()}
    if fd_atoms:
        rng = np.random.default_rng(300)
        atoms = rng.choice(len(pos), fd_atoms, replace=False)
        fd = []
        for a in atoms:
            _, nb = oracle.edge_list(pos, L, cf.model.r_cut, centers=[a])
            cs = np.concatenate([[a], nb])
            row = []
            for k in range(3):
                pp, pm = pos.copy(), pos.copy()
                pp[a, k] += h
                pm[a, k] -= h
                ep, _ = oracle.energy_forces(pp, z, L, cf.model, w, centers=cs, forces=False)
                em, _ = oracle.energy_forces(pm, z, L, cf.model, w, centers=cs, forces=False)
                row.append(-(ep - em) / (2 * h))
            fd.append(row)
            print(name, "fd atom", int(a), row, flush=True)
        out["fd_atoms"] = [int(a) for a in atoms]
        out["fd_forces"] = fd
        out["fd_step"] = h
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)
    print("wrote", name, E, flush=True)


if __name__ == "__main__":
    write("nh3_64_l1")
    write("nh3_1024_l2", fd_atoms=32)
