"""Plain CPU oracle for the weighted Euler characteristic transform / function.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP path (no
kernels, headers, helpers, tables or constants); the only common module is
the seeded input generator ``synth``, which holds none of the method's
arithmetic.

What it computes, and from which passage of the paper:

* Lower-star filtration (Definition "Lower-Star Filtrations"): a simplex
  enters at the maximum of its vertices' filter values, with the test ``<=``.
* Vertex height function (Definition "Vertex Height Functions and
  Directional Filtrations"): h_s(v) = l(v) . s.  The product is evaluated in
  float32 with round-to-nearest and the fixed order ((x*sx) + (y*sy)) + (z*sz),
  no fused multiply-add: this fixes the filter values bit for bit so that the
  integer results have exactly one correct answer.
* Weighted Euler characteristic (Definition "Weighted Euler
  Characteristic"): chi(K, w) = sum over simplices of (-1)^dim * w.
* WECF / WECT (Definitions "Weighted Euler Characteristic Function" and
  "Weighted Euler Characteristic Transform"): WECT(s, t) = chi(H_s(t), w),
  sampled at every stored threshold t = thr[q].
* The WECT as a special case of the WECF with filter values V * D^T
  (Example "WECT as a special case" in Section "Computation of WECFs").
* Simplex weights taken as the maximum of the vertex weights (caption of
  Figure 1).
* General vertex filters (Section "Computation of WECFs", Algorithm 1 with
  arbitrary filter values per vertex: ``wecf``) and the ECF of an image, whose
  vertex filter is the intensity itself (Remark on the two ECFs of an image:
  ``image_ecf``).
* The sigmoid relaxation of the WECT and its gradients with respect to
  weights, coordinates and directions (the differentiable forms named as
  future work in Section "Discussion"): submodule ``oracle.smooth``.

The forward is the definition evaluated directly: for every direction the
filter values of all cells are sorted (a library sort), the signed weights are
summed in that order (int64 for integer weights, float64 otherwise) and the
sum over {cell : value <= thr[q]} is read off with a binary search on the
sorted values.  No threshold bucketing, histogram or prefix over thresholds
is used, so the oracle does not follow the kernel's route to the answer.
``wect_bruteforce`` is the literal triple loop over (direction, threshold,
cell), for tiny inputs.

The backward is the derivative of that definition: the output is linear in the
cell weights, d out[p][q] / d w(c) = (-1)^dim(c) [f_p^max(c) <= thr[q]], and for
vertex weights the chain rule through the maximum sends each cell's gradient to
the lowest-numbered vertex attaining the maximum weight.  Finite differences in
float64 (``fd_vertex_grad``) check it.

Cubical complexes (the paper states that the method applies to them, Sections
"Introduction" and "Discussion", without fixing a construction) are built
explicitly here: a pixel/voxel is a vertex iff its intensity exceeds the
inclusion level, every axis-aligned edge, square and cube whose corners are
all vertices is a cell of dimension 1, 2, 3, and a cell's weight is the
maximum of its corner intensities (or 1 when unweighted).

Pins (tests marked "not gpu"): hand-computed single triangle / weighted
triangle / unit square / gradient examples (tests/golden), Euler
characteristic closed forms (disk, ball, sphere, torus, solid image, annulus,
hollow shell), the empty filtration below the minimum height, brute force on
random tiny complexes, linearity and permutation invariance, the Galois
property of the threshold rule, the adjoint identity <g, J w> = <J^T g, w>,
and float64 finite differences.
"""
from __future__ import annotations

import itertools
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "heights", "simplicial_cells", "cubical_cells", "cells_of", "wecf_sorted", "wect",
    "wect_bruteforce", "wecf", "wecf_bruteforce", "image_ecf", "image_ecf_cells",
    "owner_vertex", "wect_backward", "wect_backward_bruteforce",
    "loss", "fd_vertex_grad", "euler_characteristic", "total_abs_weight",
]


# ---------------------------------------------------------------------------
# filter values
# ---------------------------------------------------------------------------

def heights(coords: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """h[p, v] = l(v) . s_p in float32, order ((x*sx) + (y*sy)) + (z*sz).

    Definition "Vertex Height Functions and Directional Filtrations"; as a
    matrix V * D^T (Example "WECT as a special case").  numpy evaluates each
    float32 product and sum with one rounding and does not fuse them.
    """
    coords = np.asarray(coords, dtype=np.float32)
    dirs = np.asarray(dirs, dtype=np.float32)
    n = coords.shape[1]
    assert dirs.shape[1] == n
    h = np.multiply.outer(dirs[:, 0], coords[:, 0])  # [d, V] float32
    for k in range(1, n):
        h = h + np.multiply.outer(dirs[:, k], coords[:, k])
    return h.astype(np.float32, copy=False)


# ---------------------------------------------------------------------------
# cells with signed weights
# ---------------------------------------------------------------------------

class Cells:
    """All cells of one complex: per dimension an int array [k, m] of vertex ids
    (m = number of vertices of a cell) and the cell weights omega [k]."""

    def __init__(self, coords, verts: List[np.ndarray], weights: List[np.ndarray], integer: bool,
                 owner_source: Optional[np.ndarray] = None):
        self.coords = coords
        self.verts = verts
        self.weights = weights
        self.integer = integer
        self.owner_source = owner_source  # vertex weights for the max rule, if any

    def signed(self, dim: int) -> np.ndarray:
        w = self.weights[dim]
        return w if dim % 2 == 0 else -w


def simplicial_cells(K, weight_dtype=None) -> Cells:
    """Cells of a weighted simplicial complex (Definition "Weighted Simplicial
    Complexes"; input layout of Section "Computation of WECFs": vertex weights,
    then per dimension i an index tensor [k_i, i+1] and weights [k_i])."""
    V = K.coords.shape[0]
    verts = [np.arange(V, dtype=np.int64).reshape(V, 1)]
    for i in range(1, len(K.simplices)):
        verts.append(np.asarray(K.simplices[i], dtype=np.int64).reshape(-1, i + 1))
    if K.wmode == "ones":
        ws = [np.ones(v.shape[0], dtype=np.int64) for v in verts]
        return Cells(K.coords, verts, ws, True)
    if K.wmode == "explicit":
        integer = np.issubdtype(np.asarray(K.weights[0]).dtype, np.integer)
        dt = np.int64 if integer else np.float64
        if weight_dtype is not None:
            dt = weight_dtype
        ws = [np.asarray(K.weights[i]).astype(dt) for i in range(len(verts))]
        return Cells(K.coords, verts, ws, integer and dt == np.int64)
    if K.wmode == "vertex_max":
        # Figure 1 caption: a simplex's weight is the maximum of its vertices' weights
        w = np.asarray(K.weights[0])
        dt = weight_dtype if weight_dtype is not None else np.float64
        w = w.astype(dt)
        ws = [w[v].max(axis=1) for v in verts]
        return Cells(K.coords, verts, ws, False, owner_source=w)
    raise ValueError(K.wmode)


def cubical_cells(C) -> Cells:
    """Explicit cells of an axis-aligned image/volume.

    Vertex = pixel/voxel with intensity > include_above; an axis-aligned
    edge / square / cube is a cell iff all of its corners are vertices; the
    cell of dimension |S| spanned along the axis set S has sign (-1)^|S| and
    weight max(corner intensities) (or 1 if unweighted).  Vertex (i0,i1,i2)
    sits at (axes[0][i0], axes[1][i1], axes[2][i2]).
    """
    I = np.asarray(C.intensity)
    n = I.ndim
    shp = I.shape[::-1]                      # (n0, n1[, n2]), axis 0 fastest
    Ix = np.transpose(I)                     # index order (i0, i1, i2)
    inc = Ix.astype(np.int64) > int(C.include_above)
    lin = np.arange(I.size, dtype=np.int64).reshape(I.shape).T   # linear id at (i0,i1,i2)
    grids = np.meshgrid(*[np.asarray(a, dtype=np.float32) for a in C.axes], indexing="ij")
    coords = np.stack([g.ravel() for g in grids], axis=1)
    order = np.argsort(lin.ravel())
    coords = coords[order]                   # row = linear vertex id
    verts: List[list] = [[] for _ in range(n + 1)]
    wts: List[list] = [[] for _ in range(n + 1)]
    for r in range(n + 1):
        for S in itertools.combinations(range(n), r):
            corners, cin, cval = [], None, None
            for eps in itertools.product((0, 1), repeat=r):
                off = [0] * n
                for k, e in zip(S, eps):
                    off[k] = e
                sl = tuple(slice(off[k], off[k] + (shp[k] - 1 if k in S else shp[k])) for k in range(n))
                corners.append(lin[sl].ravel())
                ci = inc[sl].ravel()
                cv = Ix[sl].ravel().astype(np.int64)
                cin = ci if cin is None else (cin & ci)
                cval = cv if cval is None else np.maximum(cval, cv)
            cv_ids = np.stack(corners, axis=1)[cin]
            verts[r].append(cv_ids)
            wts[r].append(cval[cin] if C.weighted else np.ones(int(cin.sum()), dtype=np.int64))
    verts_c = [np.concatenate(v) if v else np.zeros((0, 2 ** r), np.int64) for r, v in enumerate(verts)]
    wts_c = [np.concatenate(w) if w else np.zeros(0, np.int64) for w in wts]
    return Cells(coords, verts_c, wts_c, True)


def cells_of(X) -> Cells:
    if isinstance(X, Cells):
        return X
    if hasattr(X, "intensity"):
        return cubical_cells(X)
    return simplicial_cells(X)


# ---------------------------------------------------------------------------
# forward: the definition evaluated with a sort
# ---------------------------------------------------------------------------

def wecf_sorted(fvals: np.ndarray, cells: Cells, thr: np.ndarray):
    """WECF_f(thr[q]) for one vertex filter f (Definition "Weighted Euler
    Characteristic Function", eq. for WECF): the sum of (-1)^dim w(c) over the
    cells c with max_{v in c} f(v) <= thr[q]."""
    vals, sw = [], []
    for dim, v in enumerate(cells.verts):
        if v.shape[0] == 0:
            continue
        vals.append(fvals[v].max(axis=1))
        sw.append(cells.signed(dim))
    acc_dt = np.int64 if cells.integer else np.float64
    T = thr.shape[0]
    if not vals:
        return np.zeros(T, dtype=acc_dt)
    vals = np.concatenate(vals)
    sw = np.concatenate(sw).astype(acc_dt)
    order = np.argsort(vals, kind="stable")
    vs = vals[order]
    csum = np.cumsum(sw[order])
    cnt = np.searchsorted(vs, thr, side="right")   # number of cells with value <= thr[q]
    out = np.zeros(T, dtype=acc_dt)
    m = cnt > 0
    out[m] = csum[cnt[m] - 1]
    return out


def _cubical_values(C, hgrid: np.ndarray):
    """(cell values, signed weights) of every cell of an image/volume for one
    height grid, by shifted views: a cell spanning the axis set S has as value
    the maximum height over its 2^|S| corners, is present iff all corners are
    vertices, and weighs (-1)^|S| * max corner intensity (or (-1)^|S|)."""
    I = np.asarray(C.intensity)
    n = I.ndim
    inc = I.astype(np.int64) > int(C.include_above)
    Iv = I.astype(np.int64)
    vals, sws = [], []
    for r in range(n + 1):
        for S in itertools.combinations(range(n), r):
            mh = mi = ok = None
            for eps in itertools.product((0, 1), repeat=r):
                sl = [slice(None)] * n
                for k, e in zip(S, eps):
                    a = n - 1 - k            # complex axis k is numpy axis n-1-k
                    sl[a] = slice(e, e + I.shape[a] - 1)
                sl = tuple(sl)
                h, iv, ic = hgrid[sl], Iv[sl], inc[sl]
                mh = h if mh is None else np.maximum(mh, h)
                mi = iv if mi is None else np.maximum(mi, iv)
                ok = ic if ok is None else (ok & ic)
            w = mi[ok] if C.weighted else np.ones(int(ok.sum()), dtype=np.int64)
            vals.append(mh[ok])
            sws.append(w if r % 2 == 0 else -w)
    return np.concatenate(vals), np.concatenate(sws)


def _sorted_sums(vals: np.ndarray, sw: np.ndarray, thr: np.ndarray):
    """sum of sw over {value <= thr[q]} for every q, via one sort."""
    T = thr.shape[0]
    if vals.shape[0] == 0:
        return np.zeros(T, dtype=sw.dtype)
    order = np.argsort(vals, kind="stable")
    csum = np.cumsum(sw[order])
    cnt = np.searchsorted(vals[order], thr, side="right")
    out = np.zeros(T, dtype=sw.dtype)
    m = cnt > 0
    out[m] = csum[cnt[m] - 1]
    return out


def wect(X, dirs: np.ndarray, thr: np.ndarray, dir_index: Optional[Sequence[int]] = None):
    """Sampled WECT [d, T] (Definition "Weighted Euler Characteristic
    Transform"): int64 for integer weights, float64 otherwise.  With
    ``dir_index`` only those directions are evaluated (rows in that order)."""
    thr = np.asarray(thr, dtype=np.float32)
    dirs = np.asarray(dirs, dtype=np.float32)
    idx = range(dirs.shape[0]) if dir_index is None else list(dir_index)
    if hasattr(X, "intensity"):
        # heights on the grid: ((x*sx) + (y*sy)) + (z*sz) with x along numpy's last axis
        axes = [np.asarray(a, np.float32) for a in X.axes]
        n = len(axes)
        rows = []
        for p in idx:
            h = None
            for k in range(n):
                shp = [1] * n
                shp[n - 1 - k] = axes[k].shape[0]
                term = (axes[k] * dirs[p, k]).astype(np.float32).reshape(shp)
                h = term if h is None else (h + term).astype(np.float32)
            h = np.broadcast_to(h, np.asarray(X.intensity).shape).astype(np.float32)
            vals, sw = _cubical_values(X, h)
            rows.append(_sorted_sums(vals, sw, thr))
        return np.stack(rows).astype(np.int64) if rows else np.zeros((0, thr.shape[0]), np.int64)
    cells = cells_of(X)
    rows = []
    for p in idx:
        h = heights(cells.coords, dirs[p:p + 1])[0]
        rows.append(wecf_sorted(h, cells, thr))
    dt = np.int64 if cells.integer else np.float64
    return np.stack(rows).astype(dt) if rows else np.zeros((0, thr.shape[0]), dt)


def wect_bruteforce(X, dirs: np.ndarray, thr: np.ndarray):
    """The definition as a literal loop over (direction, threshold, cell).
    Tiny inputs only.  Heights are formed with numpy float32 scalars in the
    same fixed order as ``heights``."""
    cells = cells_of(X)
    coords = np.asarray(cells.coords, dtype=np.float32)
    dirs = np.asarray(dirs, dtype=np.float32)
    thr = np.asarray(thr, dtype=np.float32)
    d, T, n = dirs.shape[0], thr.shape[0], coords.shape[1]
    out = [[0 if cells.integer else 0.0 for _ in range(T)] for _ in range(d)]
    for p in range(d):
        hv = []
        for v in range(coords.shape[0]):
            acc = np.float32(coords[v, 0]) * np.float32(dirs[p, 0])
            for k in range(1, n):
                acc = np.float32(acc + np.float32(coords[v, k]) * np.float32(dirs[p, k]))
            hv.append(np.float32(acc))
        for q in range(T):
            t = thr[q]
            for dim, vv in enumerate(cells.verts):
                for c in range(vv.shape[0]):
                    fmax = max(hv[int(u)] for u in vv[c])
                    if fmax <= t:
                        w = cells.weights[dim][c]
                        w = int(w) if cells.integer else float(w)
                        out[p][q] += w if dim % 2 == 0 else -w
    return np.array(out, dtype=np.int64 if cells.integer else np.float64)


# ---------------------------------------------------------------------------
# general vertex filters and the ECF of an image
# ---------------------------------------------------------------------------

def wecf(X, fvals: np.ndarray, thr: np.ndarray):
    """WECF_{f_p}(thr[q]) [m, T] for m arbitrary vertex filters fvals [V, m] on
    a simplicial complex: Section "Computation of WECFs" takes the filter values
    of every vertex as input (Algorithm 1 returns the (m, T) tensor), and the
    WECT is the case fvals = V D^T.  int64 for integer weights, float64
    otherwise."""
    cells = cells_of(X)
    F = np.asarray(fvals, dtype=np.float32)
    thr = np.asarray(thr, dtype=np.float32)
    rows = [wecf_sorted(F[:, p], cells, thr) for p in range(F.shape[1])]
    dt = np.int64 if cells.integer else np.float64
    return np.stack(rows).astype(dt) if rows else np.zeros((0, thr.shape[0]), dt)


def wecf_bruteforce(X, fvals: np.ndarray, thr: np.ndarray):
    """``wecf`` as a literal loop over (filter, threshold, cell); tiny inputs."""
    cells = cells_of(X)
    F = np.asarray(fvals, dtype=np.float32)
    thr = np.asarray(thr, dtype=np.float32)
    m, T = F.shape[1], thr.shape[0]
    out = [[0 if cells.integer else 0.0 for _ in range(T)] for _ in range(m)]
    for p in range(m):
        for q in range(T):
            for dim, vv in enumerate(cells.verts):
                for c in range(vv.shape[0]):
                    if max(F[int(u), p] for u in vv[c]) <= thr[q]:
                        w = cells.weights[dim][c]
                        w = int(w) if cells.integer else float(w)
                        out[p][q] += w if dim % 2 == 0 else -w
    return np.array(out, dtype=np.int64 if cells.integer else np.float64)


def image_ecf(C, thr: np.ndarray):
    """ECF of an image or volume (Remark on the two ECFs of an image): the
    intensity itself is the vertex filter, a cell enters at the maximum
    intensity of its corners, cells as in ``cubical_cells``; weights 1 (the
    ECF) or, when ``C.weighted``, the maximum corner intensity (a WECF).
    Returns [T] int64: sum of (-1)^dim w(c) over cells with value <= thr[q]."""
    I = np.asarray(C.intensity)
    t = np.asarray(thr, dtype=np.float32).astype(np.float64)
    vals, sw = _cubical_values(C, I.astype(np.float64))   # integer intensities: exact
    out = _sorted_sums(vals, sw.astype(np.int64), t)
    out[np.isnan(t)] = 0   # value <= NaN holds for no cell
    return out


def image_ecf_cells(C, thr: np.ndarray):
    """``image_ecf`` by the other route: the explicit cell list of
    ``cubical_cells`` and ``wecf_sorted`` with the intensity as vertex filter."""
    cells = cubical_cells(C)
    f = np.asarray(C.intensity).ravel().astype(np.float64)   # row = linear vertex id (axis 0 fastest)
    return wecf_sorted(f, cells, np.asarray(thr, dtype=np.float32).astype(np.float64))


def euler_characteristic(X) -> float:
    """chi(K, w) = sum_c (-1)^dim(c) w(c) (Definition "Weighted Euler Characteristic")."""
    cells = cells_of(X)
    tot = 0
    for dim in range(len(cells.verts)):
        s = cells.signed(dim).sum()
        tot += int(s) if cells.integer else float(s)
    return tot


def total_abs_weight(X) -> float:
    cells = cells_of(X)
    return float(sum(np.abs(w.astype(np.float64)).sum() for w in cells.weights))


# ---------------------------------------------------------------------------
# backward
# ---------------------------------------------------------------------------

def owner_vertex(K) -> List[np.ndarray]:
    """For vertex-max weights: the lowest-numbered vertex attaining the maximum
    vertex weight of each simplex, per dimension."""
    w = np.asarray(K.weights[0])
    owners = [np.arange(K.coords.shape[0], dtype=np.int64)]
    for i in range(1, len(K.simplices)):
        s = np.sort(np.asarray(K.simplices[i], dtype=np.int64), axis=1)  # ascending ids
        owners.append(s[np.arange(s.shape[0]), np.argmax(w[s], axis=1)])  # first max = lowest id
    return owners


def _cell_grads(cells: Cells, dirs, thr, grad_out, absolute=False, fvals=None):
    """d L / d w(c) for L = sum_{p,q} g[p][q] out[p][q]:
    (-1)^dim(c) * sum_p sum_{q : f_p^max(c) <= thr[q]} g[p][q]  (float64).
    The vertex filter f_p is the height along dirs[p], or column p of fvals."""
    g = np.asarray(grad_out, dtype=np.float64)
    if absolute:
        g = np.abs(g)
    thr = np.asarray(thr, dtype=np.float32)
    d, T = g.shape
    # sum over the thresholds q >= j; thr is sorted, so {q : thr[q] >= x} = [first q with thr[q] >= x, T)
    tail = np.zeros((d, T + 1), dtype=np.float64)
    tail[:, :T] = np.cumsum(g[:, ::-1], axis=1)[:, ::-1]
    grads = [np.zeros(v.shape[0], dtype=np.float64) for v in cells.verts]
    for p in range(d):
        if fvals is None:
            h = heights(cells.coords, np.asarray(dirs, np.float32)[p:p + 1])[0]
        else:
            h = np.asarray(fvals, np.float32)[:, p]
        for dim, v in enumerate(cells.verts):
            if v.shape[0] == 0:
                continue
            first = np.searchsorted(thr, h[v].max(axis=1), side="left")
            grads[dim] += tail[p, first]
    for dim in range(len(grads)):
        if dim % 2 == 1 and not absolute:
            grads[dim] = -grads[dim]
    return grads


def wect_backward(K, dirs, thr, grad_out, absolute=False, fvals=None):
    """Gradient of L = <grad_out, WECT> with respect to the weights.

    explicit weights -> list per dimension of float64 arrays d L / d w(sigma);
    vertex-max weights -> float64 [V], each simplex's gradient routed to its
    owner vertex (lowest id attaining the max).  ``absolute`` replaces every
    term by its absolute value (used for error bounds).  With ``fvals`` [V, m]
    (dirs unused) it is the gradient of the WECF of those vertex filters
    (Section "Computation of WECFs"), the output being linear in the weights
    for any filter."""
    cells = simplicial_cells(K)
    gc = _cell_grads(cells, dirs, thr, grad_out, absolute, fvals)
    if K.wmode == "vertex_max":
        V = K.coords.shape[0]
        gv = np.zeros(V, dtype=np.float64)
        for dim, own in enumerate(owner_vertex(K)):
            np.add.at(gv, own, np.abs(gc[dim]) if absolute else gc[dim])
        return gv
    return gc


def wect_backward_bruteforce(K, dirs, thr, grad_out):
    """Literal loops: d/dw(sigma) of sum_{p,q} g[p][q] * sum_{c: f_p^max(c) <= thr[q]} (-1)^dim w(c)."""
    cells = simplicial_cells(K)
    coords = np.asarray(cells.coords, np.float32)
    dirs = np.asarray(dirs, np.float32)
    thr = np.asarray(thr, np.float32)
    g = np.asarray(grad_out, np.float64)
    out = [np.zeros(v.shape[0]) for v in cells.verts]
    for p in range(dirs.shape[0]):
        hv = heights(coords, dirs[p:p + 1])[0]
        for dim, vv in enumerate(cells.verts):
            for c in range(vv.shape[0]):
                fmax = max(hv[int(u)] for u in vv[c])
                s = 0.0
                for q in range(thr.shape[0]):
                    if fmax <= thr[q]:
                        s += g[p, q]
                out[dim][c] += s if dim % 2 == 0 else -s
    return out


def loss(out, target) -> float:
    """L = sum (WECT - target)^2."""
    o = np.asarray(out, np.float64)
    t = np.asarray(target, np.float64)
    return float(((o - t) ** 2).sum())


def fd_vertex_grad(K, dirs, thr, target, vertices, eps=1e-3):
    """Central finite differences in float64 of L(w) = sum (WECT(w) - target)^2
    with respect to the listed vertex weights (vertex-max weights)."""
    from copy import deepcopy
    w0 = np.asarray(K.weights[0], dtype=np.float64)
    out = np.zeros(len(vertices))
    for j, v in enumerate(vertices):
        vals = []
        for sgn in (+1.0, -1.0):
            Kp = deepcopy(K)
            w = w0.copy()
            w[v] += sgn * eps
            Kp.weights = [w]
            cells = simplicial_cells(Kp, weight_dtype=np.float64)
            vals.append(loss(wect(cells, dirs, thr), target))
        out[j] = (vals[0] - vals[1]) / (2 * eps)
    return out
