"""Seeded synthetic inputs for the WECT/WECF hot path.

This module only *builds inputs*: vertex coordinates, simplex index lists,
uint8 intensity grids, weights, directions and threshold grids.  It holds
none of the method's arithmetic (no heights, no filtration values, no cell
inclusion or cell weights, no histograms): those live separately in the
oracle and in the HIP kernels, and both read the same arrays produced here.

Workload shapes follow the paper's experiments (Section "Experiments":
images converted to cubical complexes, synthetic 3D volumes, and triangulated
meshes); the datasets themselves are not reproduced, every array here is
random and seeded.

Seeding: ``np.random.SeedSequence(251103909, spawn_key=(cfg, item, stream))``
with streams 0 = jitter, 1 = weights, 2 = random field, 3 = sizes,
4 = target weights.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

ROOT_SEED = 251103909
STREAM_JITTER, STREAM_WEIGHTS, STREAM_FIELD, STREAM_SIZES, STREAM_TARGET = 0, 1, 2, 3, 4


def rng(cfg: int, item: int, stream: int) -> np.random.Generator:
    """Counter-style seeded generator for (config, item, stream)."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(cfg, item, stream))
    return np.random.Generator(np.random.PCG64(ss))


# ---------------------------------------------------------------------------
# containers
# ---------------------------------------------------------------------------

@dataclass
class Simplicial:
    """A geometric simplicial complex with weights (paper: weighted complex
    (K, omega) with a vertex map l: K_0 -> R^n).

    coords     float32 [V, n]
    simplices  list indexed by dimension; [0] is None (vertices are implicit),
               [i] is int32 [k_i, i+1] of vertex ids.
    wmode      'ones' | 'explicit' | 'vertex_max'
    weights    'explicit': list indexed by dimension of arrays [k_i]
               (entry 0 has length V), all int32 or all float32;
               'vertex_max': [w] with w float32 [V]; 'ones': [].
    """
    coords: np.ndarray
    simplices: List[Optional[np.ndarray]]
    wmode: str = "ones"
    weights: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.coords.shape[1])

    @property
    def top_dim(self) -> int:
        return len(self.simplices) - 1

    def counts(self) -> List[int]:
        out = [int(self.coords.shape[0])]
        for i in range(1, len(self.simplices)):
            out.append(int(self.simplices[i].shape[0]))
        return out


@dataclass
class Cubical:
    """An axis-aligned image or volume.

    intensity  uint8 array, numpy shape (n1, n0) or (n2, n1, n0): axis 0 of
               the complex is the *last* numpy axis (fastest in memory).
    axes       list of float32 per-axis coordinates, axes[k] has length n_k.
    include_above  a pixel/voxel is a vertex of the complex iff intensity > it.
    weighted   True: cell weight = max vertex intensity; False: weight 1.
    """
    intensity: np.ndarray
    axes: List[np.ndarray]
    include_above: int = 0
    weighted: bool = True

    @property
    def n(self) -> int:
        return self.intensity.ndim

    @property
    def shape_xyz(self):
        return tuple(int(s) for s in self.intensity.shape[::-1])


# ---------------------------------------------------------------------------
# directions and thresholds
# ---------------------------------------------------------------------------

def s1_directions(d: int) -> np.ndarray:
    """d evenly spaced unit vectors on S^1: theta_p = 2 pi p / d (float64 -> float32)."""
    th = 2.0 * math.pi * np.arange(d, dtype=np.float64) / d
    return np.stack([np.cos(th), np.sin(th)], axis=1).astype(np.float32)


def fibonacci_directions(N: int) -> np.ndarray:
    """N Fibonacci-sphere unit vectors: z_k = 1 - (2k+1)/N, phi_k = k pi (3 - sqrt 5)."""
    k = np.arange(N, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / N
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1).astype(np.float32)


def uniform_thresholds(T: int, R: float) -> np.ndarray:
    """T evenly spaced float32 thresholds over [-R, R] (the paper's beta map,
    Section "Computation of WECFs", evaluated in float64 and stored in float32).
    The end points are forced to -fl32(R) and fl32(R)."""
    if T < 1:
        raise ValueError("T must be >= 1")
    if T == 1:
        return np.array([np.float32(R)], dtype=np.float32)
    q = np.arange(T, dtype=np.float64)
    thr = (-R + q * (2.0 * R) / (T - 1)).astype(np.float32)
    thr[0] = -np.float32(R)
    thr[-1] = np.float32(R)
    if not np.all(np.diff(thr) > 0):
        raise AssertionError("threshold grid is not strictly increasing")
    return thr


def cubical_axis(N: int) -> np.ndarray:
    """Pixel-centre coordinates of one axis mapped onto [-1, 1]: c_i = fl32(-1 + 2 i/(N-1))."""
    if N == 1:
        return np.zeros(1, dtype=np.float32)
    return (-1.0 + 2.0 * np.arange(N, dtype=np.float64) / (N - 1)).astype(np.float32)


# ---------------------------------------------------------------------------
# complexes
# ---------------------------------------------------------------------------

def freudenthal_grid(nx: int, ny: int, jitter: float, g: Optional[np.random.Generator]):
    """Jittered nx*ny grid on [-1,1]^2 with every square split along its main
    diagonal (i,j)-(i+1,j+1). Vertex id = j*nx + i.  Returns (coords, edges, tris)."""
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    X = -1.0 + 2.0 * i / (nx - 1)
    Y = -1.0 + 2.0 * j / (ny - 1)
    XX, YY = np.meshgrid(X, Y)  # shape (ny, nx)
    pts = np.stack([XX.ravel(), YY.ravel()], axis=1)
    if jitter > 0 and g is not None:
        pts = pts + g.uniform(-jitter, jitter, size=pts.shape)
    coords = pts.astype(np.float32)
    vid = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
    a = vid[:-1, :-1].ravel()   # (i, j)
    b = vid[:-1, 1:].ravel()    # (i+1, j)
    c = vid[1:, :-1].ravel()    # (i, j+1)
    dd = vid[1:, 1:].ravel()    # (i+1, j+1)
    horiz = np.stack([vid[:, :-1].ravel(), vid[:, 1:].ravel()], axis=1)
    vert = np.stack([vid[:-1, :].ravel(), vid[1:, :].ravel()], axis=1)
    diag = np.stack([a, dd], axis=1)
    edges = np.concatenate([horiz, vert, diag]).astype(np.int32)
    tris = np.concatenate([np.stack([a, b, dd], axis=1), np.stack([a, c, dd], axis=1)]).astype(np.int32)
    return coords, edges, tris


def kuhn_grid(n: int, jitter: float, g: Optional[np.random.Generator]):
    """Jittered n^3 grid on [-1,1]^3; each cube split into the 6 Kuhn tetrahedra
    sharing its 000-111 diagonal (face diagonals run from the lowest to the
    highest corner).  Vertex id = i + n*j + n*n*k.
    Returns (coords, edges, tris, tets); every face appears exactly once."""
    ax = -1.0 + 2.0 * np.arange(n, dtype=np.float64) / (n - 1)
    K, J, I = np.meshgrid(ax, ax, ax, indexing="ij")
    pts = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    if jitter > 0 and g is not None:
        pts = pts + g.uniform(-jitter, jitter, size=pts.shape)
    coords = pts.astype(np.float32)
    ex, ey, ez = 1, n, n * n
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    vid = (ii + n * jj + n * n * kk).astype(np.int64)

    def sel(mx, my, mz):
        """vertex ids whose (i,j,k) leave room for +mx,+my,+mz steps"""
        m = (ii < n - mx) & (jj < n - my) & (kk < n - mz)
        return vid[m]

    def cat(*arrs):
        return np.concatenate(arrs).astype(np.int32)

    edges = cat(
        np.stack([v := sel(1, 0, 0), v + ex], 1),
        np.stack([v := sel(0, 1, 0), v + ey], 1),
        np.stack([v := sel(0, 0, 1), v + ez], 1),
        np.stack([v := sel(1, 1, 0), v + ex + ey], 1),
        np.stack([v := sel(1, 0, 1), v + ex + ez], 1),
        np.stack([v := sel(0, 1, 1), v + ey + ez], 1),
        np.stack([v := sel(1, 1, 1), v + ex + ey + ez], 1))
    tri_parts = []
    for (ea, eb, ma) in ((ex, ey, (1, 1, 0)), (ex, ez, (1, 0, 1)), (ey, ez, (0, 1, 1))):
        v = sel(*ma)
        tri_parts.append(np.stack([v, v + ea, v + ea + eb], 1))
        tri_parts.append(np.stack([v, v + eb, v + ea + eb], 1))
    c = sel(1, 1, 1)
    diag = ex + ey + ez
    for e in (ex, ey, ez, ex + ey, ex + ez, ey + ez):
        tri_parts.append(np.stack([c, c + e, c + diag], 1))
    tris = cat(*tri_parts)
    import itertools
    tets = []
    for perm in itertools.permutations((ex, ey, ez)):
        v1 = c + perm[0]
        v2 = v1 + perm[1]
        tets.append(np.stack([c, v1, v2, c + diag], 1))
    tets = cat(*tets)
    return coords, edges, tris, tets


def gaussian_random_field(shape, sigma: float, g: np.random.Generator) -> np.ndarray:
    """N(0,1) white noise filtered by a Gaussian of std sigma pixels (periodic,
    via FFT), min-max rescaled to [0,255] and rounded to uint8."""
    noise = g.standard_normal(size=shape)
    F = np.fft.fftn(noise)
    freqs = np.meshgrid(*[np.fft.fftfreq(s) for s in shape], indexing="ij")
    f2 = sum(f * f for f in freqs)
    F *= np.exp(-2.0 * (math.pi ** 2) * (sigma ** 2) * f2)
    field_ = np.real(np.fft.ifftn(F))
    lo, hi = field_.min(), field_.max()
    scaled = (field_ - lo) / (hi - lo) * 255.0 if hi > lo else np.zeros_like(field_)
    return np.rint(scaled).astype(np.uint8)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    complexes: list          # list of Simplicial or Cubical
    dirs: np.ndarray         # [d, n] float32
    thr: np.ndarray          # [T] float32
    out_dtype: str           # 'i32' | 'f32'
    extra: dict = field(default_factory=dict)


def cfg1() -> Workload:
    """2D simplicial, unweighted: 32x32 jittered Freudenthal grid, 32 S^1 directions, T=64."""
    coords, edges, tris = freudenthal_grid(32, 32, 0.01, rng(1, 0, STREAM_JITTER))
    K = Simplicial(coords, [None, edges, tris], "ones", [])
    return Workload("2d_simplicial_32x32_d32_T64", [K], s1_directions(32),
                    uniform_thresholds(64, math.sqrt(2.0)), "i32")


def cfg2(n_images: int = 256, side: int = 128) -> Workload:
    """2D cubical, weighted, batched: 256 uint8 GRF images (sigma 4 px), include > 64,
    cell weight = max vertex intensity, 64 S^1 directions, T=128."""
    ims = []
    ax = cubical_axis(side)
    for b in range(n_images):
        I = gaussian_random_field((side, side), 4.0, rng(2, b, STREAM_FIELD))
        ims.append(Cubical(I, [ax, ax], include_above=64, weighted=True))
    return Workload(f"2d_cubical_{n_images}x{side}x{side}_d64_T128", ims, s1_directions(64),
                    uniform_thresholds(128, math.sqrt(2.0)), "i32")


def cfg3(n: int = 64) -> Workload:
    """3D simplicial, weighted FP32: 64^3 jittered Kuhn grid, lognormal(0,0.5)
    weight per simplex, 256 Fibonacci directions, T=256."""
    coords, edges, tris, tets = kuhn_grid(n, 0.005, rng(3, 0, STREAM_JITTER))
    g = rng(3, 0, STREAM_WEIGHTS)
    w = [g.lognormal(0.0, 0.5, size=c).astype(np.float32)
         for c in (coords.shape[0], edges.shape[0], tris.shape[0], tets.shape[0])]
    K = Simplicial(coords, [None, edges, tris, tets], "explicit", w)
    return Workload(f"3d_simplicial_kuhn{n}_d256_T256", [K], fibonacci_directions(256),
                    uniform_thresholds(256, math.sqrt(3.0)), "f32")


def cfg4(n_volumes: int = 16, lo: int = 64, hi: int = 192) -> Workload:
    """3D cubical, batched uneven sizes: 16 uint8 GRF volumes (sigma 6 voxels)
    with per-axis sides uniform in [lo, hi], include > 100, weight = max vertex
    intensity, 512 Fibonacci directions, T=256."""
    g = rng(4, 0, STREAM_SIZES)
    vols = []
    for b in range(n_volumes):
        sx, sy, sz = (int(v) for v in g.integers(lo, hi + 1, size=3))
        I = gaussian_random_field((sz, sy, sx), 6.0, rng(4, b, STREAM_FIELD))
        vols.append(Cubical(I, [cubical_axis(sx), cubical_axis(sy), cubical_axis(sz)],
                            include_above=100, weighted=True))
    return Workload(f"3d_cubical_{n_volumes}vol_{lo}-{hi}_d512_T256", vols,
                    fibonacci_directions(512), uniform_thresholds(256, math.sqrt(3.0)), "i32")


def cfg5_sizes(n_complexes: int = 64, vmin: int = 10_000, vmax: int = 200_000):
    g = rng(5, 0, STREAM_SIZES)
    out = []
    for _ in range(n_complexes):
        V = int(g.integers(vmin, vmax + 1))
        nx = max(2, int(round(math.sqrt(V))))
        ny = max(2, int(round(V / nx)))
        out.append((nx, ny))
    return out


def cfg5(n_complexes: int = 64, vmin: int = 10_000, vmax: int = 200_000) -> Workload:
    """Differentiation, batched: 64 jittered Freudenthal grids with vertex counts
    uniform in [10k, 200k]; learnable FP32 vertex weights N(1, 0.2); simplex weight
    = max of its vertices' weights; 128 S^1 directions, T=128; the loss target uses
    the same complexes under reseeded weights."""
    comps, targets_w = [], []
    for b, (nx, ny) in enumerate(cfg5_sizes(n_complexes, vmin, vmax)):
        spacing = 2.0 / (nx - 1)
        coords, edges, tris = freudenthal_grid(nx, ny, 0.155 * spacing, rng(5, b, STREAM_JITTER))
        w = rng(5, b, STREAM_WEIGHTS).normal(1.0, 0.2, size=coords.shape[0]).astype(np.float32)
        wt = rng(5, b, STREAM_TARGET).normal(1.0, 0.2, size=coords.shape[0]).astype(np.float32)
        comps.append(Simplicial(coords, [None, edges, tris], "vertex_max", [w]))
        targets_w.append(wt)
    return Workload(f"2d_freudenthal_batch{n_complexes}_{vmin}-{vmax}_d128_T128_vertexmax", comps,
                    s1_directions(128), uniform_thresholds(128, math.sqrt(2.0)), "f32",
                    extra={"target_weights": targets_w})


# ---------------------------------------------------------------------------
# tiny fixtures
# ---------------------------------------------------------------------------

HAND_THRESHOLDS = np.array([-1.0, -0.5, 0.0, 0.5, 1.0, 1.5], dtype=np.float32)


def hand_directions() -> np.ndarray:
    r = np.float32(math.sqrt(0.5))
    return np.array([[1, 0], [0, 1], [-1, 0], [r, r]], dtype=np.float32)


def single_triangle(weighted: bool = False, dtype=np.float32) -> Simplicial:
    coords = np.array([[0, 0], [1, 0], [0, 1]], dtype=np.float32)
    edges = np.array([[0, 1], [0, 2], [1, 2]], dtype=np.int32)
    tris = np.array([[0, 1, 2]], dtype=np.int32)
    if not weighted:
        return Simplicial(coords, [None, edges, tris], "ones", [])
    w = [np.array([1, 2, 3], dtype=dtype), np.array([0.5, 0.25, 4], dtype=dtype),
         np.array([10], dtype=dtype)]
    return Simplicial(coords, [None, edges, tris], "explicit", w)


def single_square(weighted: bool = True) -> Cubical:
    I = np.array([[10, 20], [30, 40]], dtype=np.uint8)
    ax = np.array([0.0, 1.0], dtype=np.float32)
    return Cubical(I, [ax, ax], include_above=0, weighted=weighted)


def octahedron() -> Simplicial:
    """Boundary of the octahedron: 6 vertices, 12 edges, 8 triangles (a 2-sphere)."""
    coords = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                      dtype=np.float32)
    tris = []
    for a in (0, 1):
        for b in (2, 3):
            for c in (4, 5):
                tris.append(sorted((a, b, c)))
    tris = np.array(tris, dtype=np.int32)
    e = np.unique(np.concatenate([tris[:, [0, 1]], tris[:, [0, 2]], tris[:, [1, 2]]]), axis=0)
    return Simplicial(coords, [None, e.astype(np.int32), tris], "ones", [])


def grid_torus(nx: int, ny: int) -> Simplicial:
    """Freudenthal triangulation of the nx*ny periodic grid (nm vertices, 3nm edges,
    2nm triangles), embedded in R^3 as a torus of revolution."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny))
    u = 2 * math.pi * i.ravel() / nx
    v = 2 * math.pi * j.ravel() / ny
    R0, r0 = 1.0, 0.4
    coords = np.stack([(R0 + r0 * np.cos(v)) * np.cos(u), (R0 + r0 * np.cos(v)) * np.sin(u),
                       r0 * np.sin(v)], axis=1).astype(np.float32)

    def vid(a, b):
        return (b % ny) * nx + (a % nx)
    I, J = i.ravel(), j.ravel()
    a, b, c, d_ = vid(I, J), vid(I + 1, J), vid(I, J + 1), vid(I + 1, J + 1)
    edges = np.concatenate([np.stack([a, b], 1), np.stack([a, c], 1), np.stack([a, d_], 1)])
    tris = np.concatenate([np.stack([a, b, d_], 1), np.stack([a, c, d_], 1)])
    return Simplicial(coords, [None, edges.astype(np.int32), tris.astype(np.int32)], "ones", [])


def random_tiny_complex(seed: int, n: int = 2, nv: int = 8, top_dim: int = 2,
                        wmode: str = "explicit", wdtype=np.int32, p_face: float = 0.5) -> Simplicial:
    """A random face-closed simplicial complex on nv <= 12 vertices: random
    top-level simplices, closed under faces. Coordinates and weights are small
    random numbers; integer weights are in [-5, 5]."""
    import itertools
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=(99, seed, 0))))
    coords = g.uniform(-1, 1, size=(nv, n)).astype(np.float32)
    # snap some coordinates to a coarse lattice so that height ties and
    # threshold ties occur
    snap = g.random(size=coords.shape) < 0.3
    coords[snap] = np.round(coords[snap] * 2) / 2
    faces = {d: set() for d in range(1, top_dim + 1)}
    for d in range(top_dim, 0, -1):
        for s in itertools.combinations(range(nv), d + 1):
            if g.random() < p_face * (0.5 ** (d - 1)):
                for dd in range(1, d + 1):
                    for f in itertools.combinations(s, dd + 1):
                        faces[dd].add(f)
    simplices: List[Optional[np.ndarray]] = [None]
    for d in range(1, top_dim + 1):
        arr = np.array(sorted(faces[d]), dtype=np.int32).reshape(-1, d + 1)
        # random row order and within-row order: the method does not depend on them
        arr = arr[g.permutation(arr.shape[0])]
        arr = np.array([g.permutation(r) for r in arr], dtype=np.int32).reshape(-1, d + 1)
        simplices.append(arr)
    counts = [nv] + [s.shape[0] for s in simplices[1:]]
    if wmode == "ones":
        return Simplicial(coords, simplices, "ones", [])
    if wmode == "vertex_max":
        return Simplicial(coords, simplices, "vertex_max",
                          [g.normal(1.0, 0.3, size=nv).astype(np.float32)])
    if np.dtype(wdtype) == np.int32:
        w = [g.integers(-5, 6, size=c).astype(np.int32) for c in counts]
    else:
        w = [g.normal(0.0, 1.0, size=c).astype(np.float32) for c in counts]
    return Simplicial(coords, simplices, "explicit", w)


def solid_image(nx: int, ny: int, value: int = 200) -> Cubical:
    I = np.full((ny, nx), value, dtype=np.uint8)
    return Cubical(I, [cubical_axis(nx), cubical_axis(ny)], include_above=0, weighted=False)


def annulus_image(n: int = 9) -> Cubical:
    I = np.full((n, n), 200, dtype=np.uint8)
    I[n // 2 - 1:n // 2 + 2, n // 2 - 1:n // 2 + 2] = 0
    return Cubical(I, [cubical_axis(n), cubical_axis(n)], include_above=0, weighted=False)


def hollow_shell(n: int = 6) -> Cubical:
    I = np.full((n, n, n), 200, dtype=np.uint8)
    I[2:n - 2, 2:n - 2, 2:n - 2] = 0
    ax = cubical_axis(n)
    return Cubical(I, [ax, ax, ax], include_above=0, weighted=False)


def uniform_image(shape_xyz, seed: int = 0, weighted: bool = False, include_above: int = -1) -> Cubical:
    """Image / volume with intensities drawn uniformly from 0..255 (uint8):
    the input of the paper's ECF-of-an-image throughput measurement (Section
    "Experiments": 2048^2 to 8192^2 images, 128^3 to 512^3 volumes).  Item
    ``seed`` of config 6; every pixel is a vertex unless include_above says
    otherwise."""
    g = rng(6, seed, STREAM_FIELD)
    I = g.integers(0, 256, size=tuple(shape_xyz[::-1]), dtype=np.uint8)
    return Cubical(I, [cubical_axis(s) for s in shape_xyz], include_above=include_above, weighted=weighted)


def ecf_thresholds(T: int) -> np.ndarray:
    """T float32 thresholds evenly over the uint8 intensity range [0, 255]."""
    return np.linspace(0.0, 255.0, T).astype(np.float32)


def random_tiny_cubical(seed: int, shape_xyz=(5, 4), include_above: int = 80,
                        weighted: bool = True) -> Cubical:
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=(98, seed, 0))))
    I = g.integers(0, 256, size=tuple(shape_xyz[::-1])).astype(np.uint8)
    axes = []
    for s in shape_xyz:
        a = np.sort(g.uniform(-1, 1, size=s)).astype(np.float32)
        a = np.unique(a)
        while a.shape[0] < s:  # keep strictly increasing with the right length
            a = np.unique(np.concatenate([a, g.uniform(-1, 1, size=s - a.shape[0]).astype(np.float32)]))
        axes.append(a.astype(np.float32))
    return Cubical(I, axes, include_above=include_above, weighted=weighted)
