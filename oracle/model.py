"""Allegro-style energy E and forces F = -dE/dr in FP64 (test oracle).

Test infrastructure only (see the package docstring). The paper summarises the
model (Sec. 2.1): E is a sum of pairwise embedding energies E_ij of pairs within
a cutoff, built E(3)-equivariantly from tensors up to rank l and their tensor
products; forces are f = -dE/dr (Eq. 1). Allegro's own equations are not in the
paper; the steps below are this project's reading, in order:

  O1 edges       (i, j), i != j, minimum-image distance d < r_c, sorted by (i, j)
  O2 geometry    r_ij = mic(r_j - r_i), d = |r_ij|, rhat = r_ij / d
  O3 radial      u = envelope(d/r_c), b_n = B_n(d) u
  O4 angular     Y_l(rhat), l <= lmax
  O6 two-body    h = [onehot(z_i) | onehot(z_j) | b]; h <- SiLU(h W_k) per layer;
                 x0 = u h
  O7 features    w0 = x0 W_V0 laid out [l][c];  V0[c,l,m] = w0[l,c] Y_lm
  O8 layer t     e = x W_env^t ([l][c]);
                 Gamma_i[c,l,m] = nu^-1/2 sum_{k: (i,k) edge} e_ik[l,c] Y_lm(rhat_ik)
                 T_pi[c,m3] = sum_{m1,m2} C^pi[m1,m2,m3] V[c,l1,m1] Gamma_i[c,l2,m2]
                 s = (T_pi[c,0] for the l3 = 0 paths, path-major then channel)
                 h = [x | s]; h <- SiLU(h W) per latent layer; x <- (x + u h)/sqrt2
                 if t < T:  V[c',l3,m] = sum_{pi: l3} sum_c T_pi[c,m] W_mix^t_l3[(p,c), c']
  O9 edge        h = x; h <- SiLU(h W_k) per hidden layer; E_ij = sigma_E (h w_out)
  O10 totals     E_i = sum_j E_ij, E = sum_i E_i (math.fsum)
  O11 forces     hand-written reverse mode gives g_ij = dE/dr_ij; F_i += g_ij, F_j -= g_ij

All linear maps are y = x W with W [fan_in, fan_out] and no biases. Centres are
processed in chunks: E_i depends only on the edges of i, so chunking is exact.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from .neighbors import edge_list, minimum_image
from .radial import bessel, envelope
from .sh import clebsch_gordan, real_sh, real_sh_grad, tp_paths

SQRT2 = math.sqrt(2.0)


# --------------------------------------------------------------------------- weights

def weight_segments(desc):
    """Blob order: list of (name, fan_in, fan_out); every segment is row-major."""
    S, nb, L, T, C = desc.n_species, desc.n_bessel, desc.lmax, desc.n_layers, desc.channels
    D = desc.twobody[-1]
    paths = tp_paths(L)
    nscal = sum(1 for p in paths if p[2] == 0)
    if desc.latent[-1] != D:
        raise ValueError("the last latent width must equal the two-body output width")
    segs = []
    fin = 2 * S + nb
    for k, w in enumerate(desc.twobody):
        segs.append((f"twobody.{k}", fin, w))
        fin = w
    segs.append(("v0", D, (L + 1) * C))
    for t in range(1, T + 1):
        segs.append((f"layer{t}.env", D, (L + 1) * C))
        fin = D + nscal * C
        for k, w in enumerate(desc.latent):
            segs.append((f"layer{t}.latent.{k}", fin, w))
            fin = w
        if t < T:
            for l3 in range(L + 1):
                npath = sum(1 for p in paths if p[2] == l3)
                segs.append((f"layer{t}.mix.{l3}", npath * C, C))
    fin = D
    for k, w in enumerate(desc.edge):
        segs.append((f"edge.{k}", fin, w))
        fin = w
    segs.append(("edge.out", fin, 1))
    return segs


def unpack_weights(desc, blob: np.ndarray) -> Dict[str, np.ndarray]:
    blob = np.asarray(blob, dtype=np.float64)
    out, off = {}, 0
    for name, fi, fo in weight_segments(desc):
        out[name] = blob[off:off + fi * fo].reshape(fi, fo)
        off += fi * fo
    if off != blob.size:
        raise ValueError(f"weight blob has {blob.size} values, layout needs {off}")
    return out


# --------------------------------------------------------------------------- helpers

def _sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def _silu(a):
    return a * _sigmoid(a)


def _dsilu(a):
    s = _sigmoid(a)
    return s * (1.0 + a * (1.0 - s))


def _segment_sum(x: np.ndarray, starts: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """Sum rows of x over consecutive segments (sequential order inside each)."""
    out = np.zeros((len(counts),) + x.shape[1:])
    nz = counts > 0
    if nz.any():
        out[nz] = np.add.reduceat(x, starts[nz], axis=0)
    return out


def _tp(C, V, G):
    """T[e,c,k] = sum_{a,b} C[a,b,k] V[e,c,a] G[e,c,b]."""
    E, Ch, A = V.shape
    B = G.shape[2]
    outer = (V[:, :, :, None] * G[:, :, None, :]).reshape(E * Ch, A * B)
    return (outer @ C.reshape(A * B, -1)).reshape(E, Ch, -1)


def _tp_grad_v(C, G, gT):
    """dT/dV contracted with gT: [e,c,a] = sum_{b,k} C[a,b,k] G[e,c,b] gT[e,c,k]."""
    E, Ch, B = G.shape
    K = gT.shape[2]
    outer = (G[:, :, :, None] * gT[:, :, None, :]).reshape(E * Ch, B * K)
    return (outer @ C.transpose(1, 2, 0).reshape(B * K, -1)).reshape(E, Ch, -1)


def _tp_grad_g(C, V, gT):
    """dT/dGamma contracted with gT: [e,c,b] = sum_{a,k} C[a,b,k] V[e,c,a] gT[e,c,k]."""
    E, Ch, A = V.shape
    K = gT.shape[2]
    outer = (V[:, :, :, None] * gT[:, :, None, :]).reshape(E * Ch, A * K)
    return (outer @ C.transpose(0, 2, 1).reshape(A * K, -1)).reshape(E, Ch, -1)


@dataclass
class EdgeTrace:
    """Per-edge intermediates of one evaluation (for stage-level comparisons)."""
    ei: np.ndarray
    ej: np.ndarray
    values: Dict[str, np.ndarray] = field(default_factory=dict)


# --------------------------------------------------------------------------- core

def _evaluate_chunk(desc, W, pos, species, box, ei, ej, centers, forces, trace):
    S, nb, p, L, T, C = (desc.n_species, desc.n_bessel, desc.poly_p, desc.lmax,
                         desc.n_layers, desc.channels)
    D = desc.twobody[-1]
    rc = float(desc.r_cut)
    inv_sqrt_nu = 1.0 / math.sqrt(float(desc.avg_num_neighbors))
    sigma_e = float(desc.energy_scale)
    paths = tp_paths(L)
    cg = {pi: clebsch_gordan(*pi) for pi in paths}
    scal = [pi for pi in paths if pi[2] == 0]
    nE = len(ei)

    # local centre index of every edge; edges are sorted by centre
    local = np.searchsorted(centers, ei)
    counts = np.bincount(local, minlength=len(centers))
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])

    # O2 geometry
    r = minimum_image(pos[ej] - pos[ei], box)
    d = np.sqrt((r * r).sum(1))
    if np.any(d <= 0.0):
        raise ValueError("coincident atoms")
    rhat = r / d[:, None]
    # O3 radial
    u, dudx = envelope(d / rc, p)
    dudd = dudx / rc
    B, dB = bessel(d, rc, nb)
    b = B * u[:, None]
    # O4 angular
    Y = [real_sh(l, rhat) for l in range(L + 1)]

    # O6 two-body MLP
    onehot = np.eye(S)
    h = np.concatenate([onehot[species[ei]], onehot[species[ej]], b], axis=1)
    tb_cache = []
    for k in range(len(desc.twobody)):
        a = h @ W[f"twobody.{k}"]
        tb_cache.append(a)
        h = _silu(a)
    h2b = h
    x = u[:, None] * h2b
    # O7 initial tensor features
    w0 = (x @ W["v0"]).reshape(nE, L + 1, C)
    V = [w0[:, l, :, None] * Y[l][:, None, :] for l in range(L + 1)]
    if trace is not None:
        trace.update(d=d, u=u, b=b, Y=np.concatenate(Y, axis=1), x0=x.copy(), w0=w0.copy())

    layers = []
    for t in range(1, T + 1):
        last = t == T
        e = (x @ W[f"layer{t}.env"]).reshape(nE, L + 1, C)
        gam_c = [_segment_sum(e[:, l, :, None] * Y[l][:, None, :], starts, counts) * inv_sqrt_nu
                 for l in range(L + 1)]
        G = [g[local] for g in gam_c]
        need = scal if last else paths
        Tp = {pi: _tp(cg[pi], V[pi[0]], G[pi[1]]) for pi in need}
        s = np.concatenate([Tp[pi][:, :, 0] for pi in scal], axis=1)
        hh = np.concatenate([x, s], axis=1)
        lat_cache = []
        for k in range(len(desc.latent)):
            a = hh @ W[f"layer{t}.latent.{k}"]
            lat_cache.append(a)
            hh = _silu(a)
        x_new = (x + u[:, None] * hh) / SQRT2
        V_new = None
        if not last:
            V_new = []
            for l3 in range(L + 1):
                grp = [pi for pi in paths if pi[2] == l3]
                X = np.concatenate([Tp[pi] for pi in grp], axis=1)      # [E, P*C, 2l3+1]
                Vl = (X.transpose(0, 2, 1) @ W[f"layer{t}.mix.{l3}"]).transpose(0, 2, 1)
                V_new.append(Vl)
        layers.append(dict(x=x, e=e, G=G, V=V, Tp=Tp, need=need, hh=hh, lat=lat_cache))
        if trace is not None:
            trace[f"gamma{t}"] = np.concatenate(gam_c_flat(gam_c), axis=1)
            trace[f"s{t}"] = s
            trace[f"x{t}"] = x_new.copy()
            if V_new is not None:
                trace[f"V{t}"] = np.concatenate([v.reshape(nE, -1) for v in V_new], axis=1)
        x, V = x_new, V_new

    # O9 edge energy MLP
    hh = x
    e_cache = []
    for k in range(len(desc.edge)):
        a = hh @ W[f"edge.{k}"]
        e_cache.append(a)
        hh = _silu(a)
    wout = W["edge.out"][:, 0]
    Eij = sigma_e * (hh @ wout)
    if trace is not None:
        trace["Eij"] = Eij

    if forces is None:
        return Eij, None

    # ---------------------------------------------------------------- reverse mode
    gh = sigma_e * np.ones(nE)[:, None] * wout[None, :]
    for k in reversed(range(len(desc.edge))):
        ga = gh * _dsilu(e_cache[k])
        gh = ga @ W[f"edge.{k}"].T
    gx = gh
    gu = np.zeros(nE)
    gY = [np.zeros_like(y) for y in Y]
    gV = None
    for t in range(T, 0, -1):
        st = layers[t - 1]
        gx_prev = gx / SQRT2
        ghh = gx * u[:, None] / SQRT2
        gu += (gx * st["hh"]).sum(1) / SQRT2
        for k in reversed(range(len(desc.latent))):
            ga = ghh * _dsilu(st["lat"][k])
            ghh = ga @ W[f"layer{t}.latent.{k}"].T
        gx_prev = gx_prev + ghh[:, :D]
        gs = ghh[:, D:]
        gT = {pi: np.zeros_like(st["Tp"][pi]) for pi in st["need"]}
        for q, pi in enumerate(scal):
            gT[pi][:, :, 0] += gs[:, q * C:(q + 1) * C]
        if gV is not None:
            for l3 in range(L + 1):
                grp = [pi for pi in paths if pi[2] == l3]
                gX = (gV[l3].transpose(0, 2, 1) @ W[f"layer{t}.mix.{l3}"].T).transpose(0, 2, 1)
                for q, pi in enumerate(grp):
                    gT[pi] += gX[:, q * C:(q + 1) * C, :]
        gVprev = [np.zeros_like(v) for v in st["V"]]
        gG = [np.zeros_like(g) for g in st["G"]]
        for pi in st["need"]:
            l1, l2, _ = pi
            gVprev[l1] += _tp_grad_v(cg[pi], st["G"][l2], gT[pi])
            gG[l2] += _tp_grad_g(cg[pi], st["V"][l1], gT[pi])
        ge = np.zeros_like(st["e"])
        for l in range(L + 1):
            gGam = _segment_sum(gG[l], starts, counts)[local] * inv_sqrt_nu
            ge[:, l, :] = (gGam * Y[l][:, None, :]).sum(2)
            gY[l] += (st["e"][:, l, :, None] * gGam).sum(1)
        gx_prev = gx_prev + ge.reshape(nE, -1) @ W[f"layer{t}.env"].T
        gx, gV = gx_prev, gVprev
    # V0 = w0 (x) Y
    gw0 = np.stack([(gV[l] * Y[l][:, None, :]).sum(2) for l in range(L + 1)], axis=1)
    for l in range(L + 1):
        gY[l] += (w0[:, l, :, None] * gV[l]).sum(1)
    gx = gx + gw0.reshape(nE, -1) @ W["v0"].T
    # x0 = u h2b
    gu += (gx * h2b).sum(1)
    gh = gx * u[:, None]
    for k in reversed(range(len(desc.twobody))):
        ga = gh * _dsilu(tb_cache[k])
        gh = ga @ W[f"twobody.{k}"].T
    gb = gh[:, 2 * S:]
    gB = gb * u[:, None]
    gu += (gb * B).sum(1)
    gd = (gB * dB).sum(1) + gu * dudd
    grhat = np.zeros((nE, 3))
    for l in range(L + 1):
        grhat += np.einsum("em,emk->ek", gY[l], real_sh_grad(l, rhat))
    radial = (grhat * rhat).sum(1)
    g = gd[:, None] * rhat + (grhat - radial[:, None] * rhat) / d[:, None]
    if trace is not None:
        trace["g"] = g
    np.add.at(forces, ei, g)
    np.add.at(forces, ej, -g)
    return Eij, g


def gam_c_flat(gam_c):
    return [g.reshape(g.shape[0], -1) for g in gam_c]


def energy_forces(pos, species, box, desc, weights, centers=None, forces=True,
                  chunk: int = 512, atom_energy: bool = False, trace: Optional[dict] = None):
    """Energy (sum of E_i over `centers`, default all) and F = -dE/dr for all atoms.

    weights: the flat FP64 blob or the dict from unpack_weights. Returns
    (E, F or None[, E_i per centre]). With `trace` (a dict), per-edge
    intermediates of all evaluated edges are stored in it (small systems only).
    """
    pos = np.asarray(pos, dtype=np.float64)
    species = np.asarray(species, dtype=np.int64)
    box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)).copy()
    W = weights if isinstance(weights, dict) else unpack_weights(desc, weights)
    n = len(pos)
    if species.min() < 0 or species.max() >= desc.n_species:
        raise ValueError("species out of range")
    centers = np.arange(n) if centers is None else np.unique(np.asarray(centers, np.int64))
    F = np.zeros((n, 3)) if forces else None
    e_parts: List[np.ndarray] = []
    e_atom = np.zeros(n)
    traces = []
    for s in range(0, len(centers), chunk):
        cs = centers[s:s + chunk]
        ei, ej = edge_list(pos, box, desc.r_cut, centers=cs)
        if len(ei) == 0:
            continue
        tr = {} if trace is not None else None
        Eij, _ = _evaluate_chunk(desc, W, pos, species, box, ei, ej, cs, F, tr)
        e_parts.append(Eij)
        np.add.at(e_atom, ei, Eij)
        if tr is not None:
            tr["ei"], tr["ej"] = ei, ej
            traces.append(tr)
    E = math.fsum(np.concatenate(e_parts)) if e_parts else 0.0
    if trace is not None:
        for key in traces[0] if traces else []:
            trace[key] = np.concatenate([t[key] for t in traces], axis=0)
    out = (E, F)
    if atom_energy:
        out = out + (e_atom,)
    return out
