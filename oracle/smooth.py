"""Smooth (sigmoid) relaxation of the WECT and its gradients: float64 oracle.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU baseline may use it.

The paper names differentiable forms of its transforms as future work (Section
"Discussion") and points to the differentiable ECT of Roell and Rieck among
related software (Section "Related Work").  The relaxation evaluated here
replaces the step [f^max(c) <= t] of the lower-star filtration by a logistic
sigmoid of sharpness lam >= 0:

    S[p][q] = sum over cells c of (-1)^dim(c) w(c) sig(lam (thr[q] - f_p^max(c))),
    sig(x) = 1 / (1 + exp(-x)),

with f_p^max(c) the maximum of the float32 vertex heights of c exactly as in
the WECT (``oracle.heights``).  As lam grows, S tends to the WECT at every
threshold that differs from all cell values (and to the mean of the two
one-sided limits at a threshold equal to a cell value); at lam = 0 every entry
is half the weighted Euler characteristic.

Gradients of L = sum g[p][q] S[p][q] follow from the chain rule, in float64:
  dL/dw(c)      = (-1)^dim(c) sum_{p,q} g[p][q] sig_pq(c)
  dL/df_p^max(c) = -(-1)^dim(c) w(c) lam sum_q g[p][q] sig_pq(c) (1 - sig_pq(c))
and f_p^max(c) = <l(a), s_p> for the vertex a of c attaining the maximum
height (the lowest vertex id among equal maxima), so that value passes
s_p to the coordinates of a and l(a) to the direction s_p.  Vertex-max weights
pass dL/dw(c) to the lowest-numbered vertex of maximum weight.

Pins (tests marked "not gpu"): a hand-computed triangle (values and every
gradient from the sigmoid's textbook values), lam = 0 (half the Euler
characteristic), large lam against the step WECT of ``oracle.wect`` away from
the cell values, and float64 central finite differences of ``smooth_wect`` for
every gradient.
"""
from __future__ import annotations

from typing import Dict, List

import numpy as np

from . import heights, owner_vertex, simplicial_cells

__all__ = ["sigmoid", "smooth_wect", "smooth_wect_vjp", "fd_smooth"]

_CHUNK = 1 << 16   # simplices per block of the dense [simplices, T] evaluation


def sigmoid(x):
    """1 / (1 + exp(-x)) in float64, without overflow for large |x|."""
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def _argmax_vertex(h: np.ndarray, v: np.ndarray):
    """(max height, vertex attaining it with the lowest id) of every row of v."""
    hv = h[v]                                   # [k, m]
    hm = hv.max(axis=1)
    ids = np.where(hv == hm[:, None], v, np.iinfo(np.int64).max)
    return hm, ids.min(axis=1)


def smooth_wect(K, dirs, thr, lam, absolute: bool = False) -> np.ndarray:
    """S [d, T] float64 for one simplicial complex.  ``absolute`` sums |w| in
    place of the signed weights (a magnitude used for error bounds)."""
    cells = simplicial_cells(K, weight_dtype=np.float64)
    dirs = np.asarray(dirs, dtype=np.float32)
    t = np.asarray(thr, dtype=np.float32).astype(np.float64)
    lam = float(np.float32(lam))
    d, T = dirs.shape[0], t.shape[0]
    out = np.zeros((d, T), dtype=np.float64)
    for p in range(d):
        h = heights(cells.coords, dirs[p:p + 1])[0].astype(np.float64)
        for dim, v in enumerate(cells.verts):
            if v.shape[0] == 0:
                continue
            hm = h[v].max(axis=1)
            c = np.abs(cells.weights[dim]) if absolute else cells.signed(dim)
            for i in range(0, hm.shape[0], _CHUNK):   # rows in chunks: bounded memory
                out[p] += c[i:i + _CHUNK] @ sigmoid(lam * (t[None, :] - hm[i:i + _CHUNK, None]))
    return out


def smooth_wect_vjp(K, dirs, thr, lam, g, absolute: bool = False) -> Dict[str, object]:
    """Gradients of L = <g, S> (g [d, T]) with respect to the weights, the
    vertex coordinates [V, n] and the directions [d, n], float64.

    Returns {"weights": list per dimension (explicit weights) or [V] array
    (vertex-max weights) or None (unit weights), "coords": [V, n],
    "dirs": [d, n]}.  ``absolute`` takes the absolute value of every factor
    (weights, g, coordinates, directions), giving the sum of the magnitudes
    of the terms of each gradient entry (for error bounds)."""
    cells = simplicial_cells(K, weight_dtype=np.float64)
    coords32 = np.asarray(cells.coords, dtype=np.float32)
    X = coords32.astype(np.float64)
    dirs32 = np.asarray(dirs, dtype=np.float32)
    D = dirs32.astype(np.float64)
    t = np.asarray(thr, dtype=np.float32).astype(np.float64)
    lam = float(np.float32(lam))
    G = np.asarray(g, dtype=np.float64)
    if absolute:
        G, X, D = np.abs(G), np.abs(X), np.abs(D)
    d = D.shape[0]
    V, n = X.shape
    gx = np.zeros((V, n))
    gd = np.zeros((d, n))
    gw: List[np.ndarray] = [np.zeros(v.shape[0]) for v in cells.verts]
    for p in range(d):
        h = heights(coords32, dirs32[p:p + 1])[0].astype(np.float64)
        for dim, v in enumerate(cells.verts):
            if v.shape[0] == 0:
                continue
            hm, a = _argmax_vertex(h, v)
            sign = -1.0 if dim % 2 else 1.0
            w = cells.weights[dim]
            if absolute:
                sign, w = 1.0, np.abs(w)
            for i in range(0, hm.shape[0], _CHUNK):
                r = slice(i, i + _CHUNK)
                sg = sigmoid(lam * (t[None, :] - hm[r, None]))          # [rows, T]
                gw[dim][r] += sign * (sg @ G[p])
                # d sig(lam (t - h)) / d h = -lam sig (1 - sig)
                dh = -(sign * w[r]) * lam * ((sg * (1.0 - sg)) @ G[p])
                if absolute:
                    dh = np.abs(dh)
                np.add.at(gx, a[r], dh[:, None] * D[p][None, :])
                gd[p] += (dh[:, None] * X[a[r]]).sum(axis=0)
    if K.wmode == "vertex_max":
        gv = np.zeros(V)
        for dim, own in enumerate(owner_vertex(K)):
            np.add.at(gv, own, gw[dim])
        wres: object = gv
    elif K.wmode == "explicit":
        wres = gw
    else:
        wres = None
    return {"weights": wres, "coords": gx, "dirs": gd}


def fd_smooth(K, dirs, thr, lam, g, what: str, index, eps: float = 1e-6) -> float:
    """Central finite difference in float64 of L = <g, S> with respect to one
    input entry: what = "coords" (index (v, k)), "dirs" ((p, k)), "vweight"
    (v, vertex-max weights) or ("weight", dim) with index = simplex row.

    Heights are taken in float64 here (coordinates and directions perturbed
    by eps are not float32 values), so the complex must have no equal maxima
    and eps must be small against the gaps between heights."""
    from copy import deepcopy

    G = np.asarray(g, np.float64)
    t = np.asarray(thr, np.float32).astype(np.float64)
    lam = float(np.float32(lam))

    def value(coords, D, Kc):
        cells = simplicial_cells(Kc, weight_dtype=np.float64)
        tot = 0.0
        for p in range(D.shape[0]):
            h = coords @ D[p]
            for dim, v in enumerate(cells.verts):
                if v.shape[0] == 0:
                    continue
                hm = h[v].max(axis=1)
                tot += float(G[p] @ (cells.signed(dim) @ sigmoid(lam * (t[None, :] - hm[:, None]))))
        return tot

    X0 = np.asarray(K.coords, np.float32).astype(np.float64)
    D0 = np.asarray(dirs, np.float32).astype(np.float64)
    vals = []
    for sgn in (1.0, -1.0):
        X, D, Kc = X0.copy(), D0.copy(), K
        if what == "coords":
            X[index] += sgn * eps
        elif what == "dirs":
            D[index] += sgn * eps
        elif what == "vweight":
            Kc = deepcopy(K)
            w = np.asarray(K.weights[0], np.float64).copy()
            w[index] += sgn * eps
            Kc.weights = [w]
        else:
            dim = what[1]
            Kc = deepcopy(K)
            ws = [np.asarray(x, np.float64).copy() for x in K.weights]
            ws[dim][index] += sgn * eps
            Kc.weights = ws
        vals.append(value(X, D, Kc))
    return (vals[0] - vals[1]) / (2 * eps)
