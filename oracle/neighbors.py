"""Directed edge list by brute force (FP64, test oracle).

An edge is an ordered pair (i, j), i != j, whose minimum-image distance is below
the cutoff (pair energies live within a finite cutoff, Sec. 2.1; the paper's
linked-cell neighbour list of Sec. 2.4 is an O(N) way to find the same set).
The minimum image needs r_c < L/2 on every axis. Edges are sorted by (i, j).
"""
from __future__ import annotations

import numpy as np


def minimum_image(r: np.ndarray, box) -> np.ndarray:
    box = np.asarray(box, dtype=np.float64)
    return r - box * np.round(r / box)


def edge_list(pos: np.ndarray, box, r_cut: float, centers=None, block: int = 256):
    """Return (ei, ej) int64 arrays of all edges whose centre is in `centers`."""
    pos = np.asarray(pos, dtype=np.float64)
    box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    if not np.all(r_cut < box / 2):
        raise ValueError("minimum image needs r_cut < L/2")
    n = len(pos)
    centers = np.arange(n) if centers is None else np.asarray(centers, dtype=np.int64)
    ei_all, ej_all = [], []
    r2 = r_cut * r_cut
    for s in range(0, len(centers), block):
        c = centers[s:s + block]
        dr = minimum_image(pos[None, :, :] - pos[c][:, None, :], box)
        d2 = (dr * dr).sum(-1)
        d2[np.arange(len(c)), c] = np.inf
        ii, jj = np.nonzero(d2 < r2)
        ei_all.append(c[ii])
        ej_all.append(jj)
    ei = np.concatenate(ei_all) if ei_all else np.zeros(0, np.int64)
    ej = np.concatenate(ej_all) if ej_all else np.zeros(0, np.int64)
    order = np.lexsort((ej, ei))
    return ei[order].astype(np.int64), ej[order].astype(np.int64)
