"""Parity of the sigmoid relaxation (forward and adjoint) with the float64 oracle.

Forward bound, per output entry of a complex with cells c and weights w:
    16 u sum_c |w(c)| + 2 C M 2^-30     (u = 2^-24, C cells, M = max |w|)
Each term's error is at most about 6 u |w|: the float32 exponent argument
(three roundings, weighted by sig(1 - sig)|x| <= 0.224), exp2 and reciprocal
(one ulp each), 1 + e, the product w sig, and the window cut-off exp(-17) <
0.7 u; every term is rounded to the fixed-point grid 2^-e with 2^-e <= 2M 2^-30
and the terms are summed exactly.

Adjoint bound, per gradient entry: (n + 16) u times the same gradient with every
factor replaced by its absolute value (oracle ``absolute=True``), where n is the
number of float32 additions along the longest chain into that entry (window
terms, lane reduction, atomic adds)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import smooth as osm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
U = 2.0 ** -24


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def W():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_03909_amd import api
    api.set_launch()
    return api


# ---------------------------------------------------------------------------
# inputs
# ---------------------------------------------------------------------------

def _weights(wmode, counts, g):
    if wmode == "ones":
        return []
    if wmode == "vertex_max":
        return [g.normal(1.0, 0.3, size=counts[0]).astype(np.float32)]
    return [g.lognormal(0.0, 0.5, size=k).astype(np.float32) for k in counts]


def tri2d(nx, ny, wmode, seed, n=2):
    g = synth.rng(50, seed, 0)
    coords, edges, tris = synth.freudenthal_grid(nx, ny, 0.3 / nx, g)
    if n == 1:
        coords = np.ascontiguousarray(coords[:, :1])
    counts = [coords.shape[0], edges.shape[0], tris.shape[0]]
    return synth.Simplicial(coords, [None, edges, tris], wmode, _weights(wmode, counts, g))


def tet3d(m, wmode, seed):
    g = synth.rng(51, seed, 0)
    coords, edges, tris, tets = synth.kuhn_grid(m, 0.3 / m, g)
    counts = [coords.shape[0], edges.shape[0], tris.shape[0], tets.shape[0]]
    return synth.Simplicial(coords, [None, edges, tris, tets], wmode, _weights(wmode, counts, g))


def dirs_for(n, d):
    if n == 1:
        return np.array([[1.0], [-1.0], [0.5], [-2.0]][:d], np.float32) if d <= 4 else \
            np.linspace(-2, 2, d).astype(np.float32).reshape(d, 1)
    return synth.s1_directions(d) if n == 2 else synth.fibonacci_directions(d)


def _cells(K):
    return sum(K.counts())


def _maxw(K):
    if K.wmode == "ones":
        return 1.0
    return float(max(np.abs(np.asarray(w, np.float64)).max() for w in K.weights if len(w)))


def _max_degree(K):
    """Largest number of simplices (dimension >= 1) containing one vertex."""
    deg = np.zeros(K.coords.shape[0], np.int64)
    for s in K.simplices[1:]:
        deg += np.bincount(np.asarray(s).ravel(), minlength=K.coords.shape[0])
    return int(deg.max()) if deg.size else 0


def fwd_tol(K):
    """16 u sum|w| plus the fixed-point grid: 2^-e <= 2 M' 2^-30 per term, with
    M' = M for the per-cell kernels (C terms) and M (1 + degree) for the
    vertex-centric ones (V terms per output entry)."""
    grid = max(_cells(K), K.coords.shape[0] * (1 + _max_degree(K)))
    return 16 * U * oracle.total_abs_weight(K) + 2 * grid * _maxw(K) * 2.0 ** -30


def gpu_smooth(W, Ks, dirs, thr, lam, ls=False):
    cx = W.SimplicialBatch.from_host(Ks)
    index = W.lower_star_index(cx) if ls else None
    out = W.smooth_forward(cx, W.Grid(dirs, thr), lam, index=index)
    torch.cuda.synchronize()
    return out.cpu().numpy()


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------

FWD_CASES = [
    # name, complexes, d, T, R, lam
    ("tri2d ones d70 T50 lam4", lambda: [tri2d(40, 30, "ones", 0)], 70, 50, 1.6, 4.0),
    ("tri2d explicit d64 T37 lam40", lambda: [tri2d(13, 11, "explicit", 1)], 64, 37, 1.6, 40.0),
    ("tri2d vmax d5 T64 lam1e4", lambda: [tri2d(12, 12, "vertex_max", 2)], 5, 64, 1.6, 1e4),
    ("tri2d vmax lam0 (whole window)", lambda: [tri2d(9, 8, "vertex_max", 3)], 9, 21, 1.6, 0.0),
    ("tet3d explicit d64 T33 lam6", lambda: [tet3d(8, "explicit", 4)], 64, 33, 2.0, 6.0),
    ("tet3d ones d100 T20 lam2", lambda: [tet3d(4, "ones", 5)], 100, 20, 2.0, 2.0),
    ("line1d explicit d4 T40 lam8", lambda: [tri2d(10, 9, "explicit", 6, n=1)], 4, 40, 2.5, 8.0),
    ("batch vmax ragged d70 T40 lam5", lambda: [tri2d(9, 7, "vertex_max", 7), tri2d(15, 13, "vertex_max", 8),
                                               tri2d(4, 3, "vertex_max", 9)], 70, 40, 1.6, 5.0),
]


@pytest.mark.parametrize("case", FWD_CASES, ids=[c[0] for c in FWD_CASES])
@pytest.mark.parametrize("decomposition", [0, 1, 2])
@pytest.mark.parametrize("ls", [False, True], ids=["cells", "lower_star"])
def test_smooth_forward_parity(W, case, decomposition, ls):
    name, make, d, T, R, lam = case
    _say(f"smooth forward {name} decomposition={decomposition} lower_star={ls}")
    Ks = make()
    n = Ks[0].n
    dirs = dirs_for(n, d)
    thr = synth.uniform_thresholds(T, R)
    W.set_launch(decomposition=decomposition)
    try:
        got = gpu_smooth(W, Ks, dirs, thr, lam, ls)
    finally:
        W.set_launch()
    assert got.shape == (len(Ks), d, T)
    for b, K in enumerate(Ks):
        ref = osm.smooth_wect(K, dirs, thr, lam)
        err = np.abs(got[b].astype(np.float64) - ref).max()
        assert err <= fwd_tol(K), f"{name} complex {b}: error {err} > {fwd_tol(K)}"


@pytest.mark.parametrize("ls", [False, True], ids=["cells", "lower_star"])
def test_smooth_large_lam_tends_to_the_wect(W, ls):
    """At lam = 1e6 with every threshold at least 1e-3 from every height, each
    relaxed term is the step up to exp(-1000): the output equals the WECT."""
    K = tri2d(11, 10, "explicit", 10)
    dirs = synth.s1_directions(6)
    h = oracle.heights(K.coords, dirs).astype(np.float64).ravel()
    thr = np.array([t for t in np.linspace(-1.6, 1.6, 57) if np.min(np.abs(h - t)) >= 1e-3], np.float32)
    got = gpu_smooth(W, [K], dirs, thr, 1e6, ls)[0]
    ref = oracle.wect(K, dirs, thr).astype(np.float64)
    assert np.abs(got - ref).max() <= fwd_tol(K)


@pytest.mark.parametrize("ls", [False, True], ids=["cells", "lower_star"])
def test_smooth_duplicate_thresholds_and_empty_complex(W, ls):
    """Non-decreasing thresholds with repeats (binary-search index), and a
    batch with an empty complex (all-zero rows)."""
    K = tri2d(8, 8, "vertex_max", 11)
    E = synth.Simplicial(np.zeros((0, 2), np.float32), [None, np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32)],
                         "vertex_max", [np.zeros(0, np.float32)])
    dirs = synth.s1_directions(7)
    thr = np.sort(np.concatenate([synth.uniform_thresholds(12, 1.5), synth.uniform_thresholds(6, 1.5)]))
    got = gpu_smooth(W, [K, E], dirs, thr, 3.0, ls)
    ref = osm.smooth_wect(K, dirs, thr, 3.0)
    assert np.abs(got[0] - ref).max() <= fwd_tol(K)
    assert np.all(got[1] == 0.0)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

BWD_CASES = [
    ("tri2d explicit d70 T40 lam5", lambda: [tri2d(12, 10, "explicit", 20)], 70, 40, 1.6, 5.0),
    ("tri2d vmax d64 T64 lam12", lambda: [tri2d(36, 30, "vertex_max", 21)], 64, 64, 1.6, 12.0),
    ("tet3d ones d33 T30 lam4", lambda: [tet3d(4, "ones", 22)], 33, 30, 2.0, 4.0),
    ("tet3d explicit d64 T24 lam0", lambda: [tet3d(3, "explicit", 23)], 64, 24, 2.0, 0.0),
    ("line1d vmax d4 T30 lam3", lambda: [tri2d(9, 9, "vertex_max", 24, n=1)], 4, 30, 2.5, 3.0),
    ("batch explicit ragged d130 T32 lam6", lambda: [tri2d(20, 17, "explicit", 25), tri2d(31, 29, "explicit", 26)],
     130, 32, 1.6, 6.0),
]


@pytest.mark.parametrize("case", BWD_CASES, ids=[c[0] for c in BWD_CASES])
@pytest.mark.parametrize("ls", [False, True], ids=["cells", "lower_star"])
def test_smooth_backward_parity(W, case, ls):
    name, make, d, T, R, lam = case
    _say(f"smooth backward {name} lower_star={ls}")
    Ks = make()
    n = Ks[0].n
    dirs = dirs_for(n, d)
    thr = synth.uniform_thresholds(T, R)
    B = len(Ks)
    g = synth.rng(52, len(name), 0).normal(size=(B, d, T)).astype(np.float32)
    cx = W.SimplicialBatch.from_host(Ks)
    index = W.lower_star_index(cx) if ls else None
    res = W.smooth_backward(cx, W.Grid(dirs, thr), lam, torch.from_numpy(g).cuda(), index=index)
    torch.cuda.synchronize()
    gx = res["coords"].cpu().numpy()
    gd = res["dirs"].cpu().numpy()
    gw = res["weights"]
    ntiles = (d + 63) // 64
    vo = np.concatenate([[0], np.cumsum([K.coords.shape[0] for K in Ks])])
    ref_dirs = np.zeros((d, n))
    abs_dirs = np.zeros((d, n))
    for b, K in enumerate(Ks):
        ref = osm.smooth_wect_vjp(K, dirs, thr, lam, g[b])
        mag = osm.smooth_wect_vjp(K, dirs, thr, lam, g[b], absolute=True)
        ref_dirs += ref["dirs"]
        abs_dirs += mag["dirs"]
        chain = T + 48 + (1 + _max_degree(K)) * ntiles
        e = np.abs(gx[vo[b]:vo[b + 1]] - ref["coords"])
        assert np.all(e <= (chain + 16) * U * mag["coords"] + 1e-30), f"{name} coords, complex {b}: {e.max()}"
        if K.wmode == "vertex_max":
            e = np.abs(gw.cpu().numpy()[vo[b]:vo[b + 1]] - ref["weights"])
            assert np.all(e <= (chain + 16) * U * mag["weights"] + 1e-30), f"{name} vertex weights {b}"
        elif K.wmode == "explicit":
            for dim in range(K.top_dim + 1):
                lo = sum(Kk.counts()[dim] for Kk in Ks[:b])
                got = gw[dim].cpu().numpy()[lo:lo + K.counts()[dim]]
                e = np.abs(got - ref["weights"][dim])
                bound = (T + 48 + 64 * ntiles) * U * mag["weights"][dim] + 1e-30
                assert np.all(e <= bound), f"{name} weights dim {dim}, complex {b}: {e.max()}"
        else:
            assert gw is None
    chain_d = sum(_cells(K) for K in Ks) + T + 1024
    e = np.abs(gd - ref_dirs)
    assert np.all(e <= (chain_d + 16) * U * abs_dirs + 1e-30), f"{name} dirs: {e.max()}"


def test_smooth_backward_optional_outputs(W):
    """Gradients that are not asked for are not written; the others match a full call."""
    K = tri2d(9, 8, "explicit", 30)
    dirs, thr = synth.s1_directions(16), synth.uniform_thresholds(24, 1.6)
    cx = W.SimplicialBatch.from_host([K])
    grid = W.Grid(dirs, thr)
    g = torch.from_numpy(synth.rng(53, 0, 0).normal(size=(1, 16, 24)).astype(np.float32)).cuda()
    full = W.smooth_backward(cx, grid, 7.0, g)
    part = W.smooth_backward(cx, grid, 7.0, g, coords=False, weights=False)
    torch.cuda.synchronize()
    assert part["coords"] is None and part["weights"] is None
    # both calls within the adjoint bound of the oracle (float32 atomics: the
    # two results may differ in the last bits)
    ref = osm.smooth_wect_vjp(K, dirs, thr, 7.0, g.cpu().numpy()[0])
    mag = osm.smooth_wect_vjp(K, dirs, thr, 7.0, g.cpu().numpy()[0], absolute=True)
    bound = (_cells(K) + 24 + 1024 + 16) * U * mag["dirs"] + 1e-30
    for r in (part, full):
        assert np.all(np.abs(r["dirs"].cpu().numpy() - ref["dirs"]) <= bound)


def test_smooth_autograd_layer(W):
    """torch.autograd through SmoothWECT gives the oracle's adjoint for a
    linear loss L = <G, S> (upstream gradient G, a fixed random array)."""
    K = tri2d(10, 9, "vertex_max", 31)
    dirs, thr = synth.s1_directions(12), synth.uniform_thresholds(30, 1.6)
    cx = W.SimplicialBatch.from_host([K])
    layer = W.SmoothWECT(torch.from_numpy(dirs), torch.from_numpy(thr), lam=9.0).cuda()
    coords = cx.coords.clone().requires_grad_(True)
    w = cx.weights[0].clone().requires_grad_(True)
    g = synth.rng(55, 0, 0).normal(size=(12, 30)).astype(np.float32)
    out = layer(cx, coords, w)
    loss = (out * torch.from_numpy(g).cuda()[None]).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref = osm.smooth_wect_vjp(K, dirs, thr, 9.0, g)
    mag = osm.smooth_wect_vjp(K, dirs, thr, 9.0, g, absolute=True)
    chain = 30 + 48 + 1 + _max_degree(K)
    for got, key, n in ((coords.grad, "coords", chain), (w.grad, "weights", chain),
                        (layer.dirs.grad, "dirs", _cells(K) + 30 + 1024)):
        e = np.abs(got.cpu().numpy() - ref[key])
        assert np.all(e <= (n + 16) * U * mag[key] + 1e-30), f"{key}: {e.max()}"


def smooth_lam(thr):
    """Sharpness of the benchmark: the sigmoid rises over about two threshold
    spacings (lam x spacing = 2), so each cell's window spans about 17 thresholds."""
    thr = np.asarray(thr, np.float64)
    return float(np.float32(2.0 * (thr.size - 1) / (thr[-1] - thr[0])))


@pytest.mark.parametrize("ls", [False, True], ids=["cells", "lower_star"])
def test_smooth_differentiation_batch_sampled(W, ls):
    """Full size, in the launch configuration the benchmark times (defaults):
    the differentiation batch (64 jittered Freudenthal grids of 10k-200k
    vertices, vertex-max weights, 128 directions, 128 thresholds).  Sampled
    (complex, direction) rows of the forward against the oracle; the adjoint
    with grad_out non-zero on the sampled rows only, against the oracle
    restricted to those directions (the other rows contribute exact zeros)."""
    _say(f"smooth differentiation batch, full size, lower_star={ls}")
    w = synth.cfg5()
    lam = smooth_lam(w.thr)
    cx = W.SimplicialBatch.from_host(w.complexes)
    grid = W.Grid(w.dirs, w.thr)
    index = W.lower_star_index(cx) if ls else None
    out = W.smooth_forward(cx, grid, lam, index=index).cpu().numpy()
    Vs = [K.coords.shape[0] for K in w.complexes]
    small, mid = int(np.argmin(Vs)), int(np.argsort(Vs)[len(Vs) // 2])
    samples = [(small, 5), (small, 77), (mid, 40)]
    for b, p in samples:
        K = w.complexes[b]
        ref = osm.smooth_wect(K, w.dirs[p:p + 1], w.thr, lam)[0]
        err = np.abs(out[b, p].astype(np.float64) - ref).max()
        assert err <= fwd_tol(K), f"complex {b} direction {p}: {err}"
    B, d, T = out.shape
    g = np.zeros((B, d, T), np.float32)
    rg = synth.rng(54, 0, 0)
    for b, p in samples:
        g[b, p] = rg.normal(size=T)
    res = W.smooth_backward(cx, grid, lam, torch.from_numpy(g).cuda(), index=index)
    torch.cuda.synchronize()
    gx, gd, gv = res["coords"].cpu().numpy(), res["dirs"].cpu().numpy(), res["weights"].cpu().numpy()
    vo = np.concatenate([[0], np.cumsum(Vs)])
    ref_d = np.zeros((d, 2))
    mag_d = np.zeros((d, 2))
    for b in sorted({b for b, _ in samples}):
        K = w.complexes[b]
        ps = [p for bb, p in samples if bb == b]
        ref = osm.smooth_wect_vjp(K, w.dirs[ps], w.thr, lam, g[b, ps])
        mag = osm.smooth_wect_vjp(K, w.dirs[ps], w.thr, lam, g[b, ps], absolute=True)
        chain = T + 48 + (1 + _max_degree(K)) * 2
        e = np.abs(gx[vo[b]:vo[b + 1]] - ref["coords"])
        assert np.all(e <= (chain + 16) * U * mag["coords"] + 1e-30), f"coords of complex {b}: {e.max()}"
        e = np.abs(gv[vo[b]:vo[b + 1]] - ref["weights"])
        assert np.all(e <= (chain + 16) * U * mag["weights"] + 1e-30), f"vertex weights of complex {b}: {e.max()}"
        for i, p in enumerate(ps):
            ref_d[p] += ref["dirs"][i]
            mag_d[p] += mag["dirs"][i]
    e = np.abs(gd - ref_d)
    chain_d = sum(_cells(K) for K in w.complexes) + T + 1024
    assert np.all(e <= (chain_d + 16) * U * mag_d + 1e-30), f"directions: {e.max()}"
    others = np.ones(len(Vs), bool)
    others[[b for b, _ in samples]] = False
    for b in np.nonzero(others)[0][:8]:
        assert np.all(gx[vo[b]:vo[b + 1]] == 0.0)


def _fan(spokes, seed):
    """A disc fanned around one centre vertex with `spokes` > 32 edges (the
    centre cannot use neighbour bits)."""
    g = np.random.default_rng(seed)
    ang = np.sort(g.uniform(0, 2 * np.pi, size=spokes))
    ring = np.stack([np.cos(ang), np.sin(ang)], axis=1) * g.uniform(0.8, 1.2, size=(spokes, 1))
    coords = np.concatenate([g.normal(0, 0.05, size=(1, 2)), ring]).astype(np.float32)
    k = np.arange(1, spokes + 1)
    nxt = np.where(k == spokes, 1, k + 1)
    edges = np.concatenate([np.stack([np.zeros_like(k), k], 1), np.stack([k, nxt], 1)]).astype(np.int32)
    tris = np.stack([np.zeros_like(k), k, nxt], 1).astype(np.int32)
    counts = [coords.shape[0], edges.shape[0], tris.shape[0]]
    return synth.Simplicial(coords, [None, edges, tris], "explicit",
                            [g.lognormal(0, 0.5, size=c).astype(np.float32) for c in counts])


def _not_face_closed(seed):
    """A triangulated grid with a third of its edges removed: triangles whose
    vertex pairs have no edge (those vertices cannot use neighbour bits)."""
    K = tri2d(12, 10, "vertex_max", seed)
    g = np.random.default_rng(seed)
    keep = g.random(K.simplices[1].shape[0]) > 0.33
    return synth.Simplicial(K.coords, [None, K.simplices[1][keep], K.simplices[2]], K.wmode, K.weights)


@pytest.mark.parametrize("make", [lambda: _fan(40, 1), lambda: _not_face_closed(2)], ids=["fan40", "not_closed"])
@pytest.mark.parametrize("ls", [False, True], ids=["cells", "lower_star"])
def test_smooth_general_complexes(W, make, ls):
    """The per-row height test of the vertex-centric kernels (vertices with more
    than 32 edges, cofaces without edges), forward and adjoint."""
    K = make()
    _say(f"smooth general complex lower_star={ls}")
    dirs, thr, lam = synth.s1_directions(70), synth.uniform_thresholds(40, 1.6), 6.0
    got = gpu_smooth(W, [K], dirs, thr, lam, ls)[0]
    ref = osm.smooth_wect(K, dirs, thr, lam)
    assert np.abs(got - ref).max() <= fwd_tol(K)
    g = synth.rng(56, 0, 0).normal(size=(1, 70, 40)).astype(np.float32)
    cx = W.SimplicialBatch.from_host([K])
    index = W.lower_star_index(cx) if ls else None
    res = W.smooth_backward(cx, W.Grid(dirs, thr), lam, torch.from_numpy(g).cuda(), index=index)
    torch.cuda.synchronize()
    r = osm.smooth_wect_vjp(K, dirs, thr, lam, g[0])
    mag = osm.smooth_wect_vjp(K, dirs, thr, lam, g[0], absolute=True)
    chain = 40 + 48 + (1 + _max_degree(K)) * 2
    e = np.abs(res["coords"].cpu().numpy() - r["coords"])
    assert np.all(e <= (chain + 16) * U * mag["coords"] + 1e-30), e.max()
    if K.wmode == "vertex_max":
        e = np.abs(res["weights"].cpu().numpy() - r["weights"])
        assert np.all(e <= (chain + 16) * U * mag["weights"] + 1e-30), e.max()
    else:
        for dim in range(3):
            e = np.abs(res["weights"][dim].cpu().numpy() - r["weights"][dim])
            assert np.all(e <= (40 + 48 + 64 * 2 + 16) * U * mag["weights"][dim] + 1e-30), (dim, e.max())


@pytest.mark.parametrize("ls", [False, True], ids=["cells", "lower_star"])
@pytest.mark.parametrize("T", [256, 600])
def test_smooth_many_thresholds(W, ls, T):
    """T = 256: the 64-bit histogram leaves less LDS for staging (smaller
    blocks and 32 staged coface rows per wavefront for the vertex-centric
    kernels); T = 600 runs in threshold tiles (each output column depends on
    its own threshold, and each tile's windows are cut at its ends).  Forward
    and adjoint, on a 2D mesh and a 3D Kuhn mesh whose inner vertices have
    more than 32 cofaces (staged in chunks)."""
    for K, dirs in ((tri2d(16, 14, "explicit", 40), synth.s1_directions(20)),
                    (tet3d(5, "explicit", 42), synth.fibonacci_directions(20))):
        lam = 40.0
        thr = synth.uniform_thresholds(T, 1.6 if K.n == 2 else 2.0)
        _say(f"smooth T={T} n={K.n} lower_star={ls}: forward")
        got = gpu_smooth(W, [K], dirs, thr, lam, ls)[0]
        ref = osm.smooth_wect(K, dirs, thr, lam)
        assert np.abs(got - ref).max() <= fwd_tol(K)
        _say(f"smooth T={T} n={K.n} lower_star={ls}: adjoint")
        d = dirs.shape[0]
        g = synth.rng(54, T, K.n).normal(size=(1, d, T)).astype(np.float32)
        cx = W.SimplicialBatch.from_host([K])
        index = W.lower_star_index(cx) if ls else None
        res = W.smooth_backward(cx, W.Grid(dirs, thr), lam, torch.from_numpy(g).cuda(), index=index)
        torch.cuda.synchronize()
        r = osm.smooth_wect_vjp(K, dirs, thr, lam, g[0])
        mag = osm.smooth_wect_vjp(K, dirs, thr, lam, g[0], absolute=True)
        chain = T + 48 + (1 + _max_degree(K)) * 4
        e = np.abs(res["coords"].cpu().numpy() - r["coords"])
        assert np.all(e <= (chain + 16) * U * mag["coords"] + 1e-30), e.max()
        for dim in range(K.top_dim + 1):
            e = np.abs(res["weights"][dim].cpu().numpy() - r["weights"][dim])
            assert np.all(e <= (T + 48 + 64 * 4 + 16) * U * mag["weights"][dim] + 1e-30), (dim, e.max())
        e = np.abs(res["dirs"].cpu().numpy() - r["dirs"])
        assert np.all(e <= (_cells(K) + T + 1024 + 16) * U * mag["dirs"] + 1e-30), e.max()


@pytest.mark.parametrize("ls", [False, True], ids=["cells", "lower_star"])
@pytest.mark.parametrize("wmode", ["explicit", "vertex_max"])
def test_smooth_forward_invariant_to_simplex_order(W, ls, wmode):
    """Permuting the simplex rows of each dimension, and the vertices within
    each row, reorders the stream and the lower-star index's entries, but no
    cell's term and no vertex's set of cofaces changes: with exact integer
    histogram sums (and exact float64 sums of these weights per vertex) the
    forward is bit-identical."""
    K = tri2d(30, 24, wmode, 41)
    g = np.random.default_rng(41)
    simp, ws = [None], [K.weights[0]] if K.weights else []
    for dim in (1, 2):
        perm = g.permutation(K.simplices[dim].shape[0])
        rows = np.array([g.permutation(r) for r in K.simplices[dim][perm]], np.int32)
        simp.append(np.ascontiguousarray(rows))
        if wmode == "explicit":
            ws.append(K.weights[dim][perm])
    K2 = synth.Simplicial(K.coords, simp, wmode, ws)
    dirs, thr, lam = synth.s1_directions(64), synth.uniform_thresholds(48, 1.6), 30.0
    _say(f"simplex order wmode={wmode} ls={ls}")
    a = gpu_smooth(W, [K], dirs, thr, lam, ls)[0]
    b = gpu_smooth(W, [K2], dirs, thr, lam, ls)[0]
    assert np.array_equal(a, b)
    assert np.abs(a - osm.smooth_wect(K, dirs, thr, lam)).max() <= fwd_tol(K)


def test_smooth_lower_star_large_block_request(W):
    """A 1024-thread block with one block per group (what the automatic
    choice takes for many large groups) does not fit the vertex-centric
    kernels' coface rows at T = 256: the plan lowers the block to one that
    fits instead of refusing, for the forward and the adjoint."""
    Ks = [tri2d(12, 10, "vertex_max", 60), tri2d(9, 13, "vertex_max", 61)]
    dirs, thr, lam = synth.s1_directions(70), synth.uniform_thresholds(256, 1.6), 30.0
    cx = W.SimplicialBatch.from_host(Ks)
    index = W.lower_star_index(cx)
    g = synth.rng(55, 0, 0).normal(size=(2, 70, 256)).astype(np.float32)
    try:
        W.set_launch(1024, 0, 0, 2)
        _say("lower-star relaxation, requested block 1024, group decomposition, T=256")
        out = W.smooth_forward(cx, W.Grid(dirs, thr), lam, index=index)
        res = W.smooth_backward(cx, W.Grid(dirs, thr), lam, torch.from_numpy(g).cuda(), index=index)
        torch.cuda.synchronize()
    finally:
        W.set_launch()
    out = out.cpu().numpy()
    vo = np.concatenate([[0], np.cumsum([K.coords.shape[0] for K in Ks])])
    for b, K in enumerate(Ks):
        assert np.abs(out[b] - osm.smooth_wect(K, dirs, thr, lam)).max() <= fwd_tol(K)
        r = osm.smooth_wect_vjp(K, dirs, thr, lam, g[b])
        mag = osm.smooth_wect_vjp(K, dirs, thr, lam, g[b], absolute=True)
        chain = 256 + 48 + (1 + _max_degree(K)) * 2
        e = np.abs(res["weights"].cpu().numpy()[vo[b]:vo[b + 1]] - r["weights"])
        assert np.all(e <= (chain + 16) * U * mag["weights"] + 1e-30), e.max()
        e = np.abs(res["coords"].cpu().numpy()[vo[b]:vo[b + 1]] - r["coords"])
        assert np.all(e <= (chain + 16) * U * mag["coords"] + 1e-30), e.max()
