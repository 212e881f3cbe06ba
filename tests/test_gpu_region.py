"""The simplicial forward through the region index (wect_region_build, then
the forward with wect_complex.cell_index set), through the C ABI.

The index changes where a vertex's threshold index is computed (once per region
and direction tile, into an LDS table) but not what is summed: integer and
64-bit fixed-point histogram sums are exact, so the output must have the same
bits as the per-cell forward's, and match the CPU oracle (bit-exact for
integer weights, within 1e-5 * sum|w| for float32 weights).  The index itself
is downloaded and checked against its documented layout: every cell exactly
once, in the region of its lowest vertex, halos sorted and complete, local ids
that decode to the cell's vertices."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F32_RTOL = 1e-5


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


def _pair(W, complexes, dirs, thr):
    """Forward without and with the region index on the same batch."""
    cx = W.SimplicialBatch.from_host(list(complexes))
    g = W.Grid(dirs, thr)
    plain = W.wect_forward(cx, g).cpu().numpy()
    W.region_index(cx)
    reg = W.wect_forward(cx, g).cpu().numpy()
    torch.cuda.synchronize()
    return plain, reg


def _check(W, complexes, dirs, thr, what, oracle_check=True):
    _say(what)
    plain, reg = _pair(W, complexes, dirs, thr)
    assert plain.dtype == reg.dtype
    bad = np.argwhere(plain.view(np.int32) != reg.view(np.int32))
    assert bad.size == 0, f"{what}: {len(bad)} entries differ from the per-cell forward, first {bad[:5].tolist()}"
    if oracle_check:
        for b, K in enumerate(complexes):
            ref = oracle.wect(K, dirs, thr)
            if np.issubdtype(ref.dtype, np.integer):
                assert np.array_equal(reg[b].astype(np.int64), ref), f"{what}: complex {b}"
            else:
                tol = F32_RTOL * max(oracle.total_abs_weight(K), 1e-30)
                err = np.abs(reg[b].astype(np.float64) - ref).max() if ref.size else 0.0
                assert err <= tol, f"{what}: complex {b}: {err} > {tol}"


def _reweight(K, mode, seed):
    g = np.random.default_rng(seed)
    counts = K.counts()
    if mode == "ones":
        return synth.Simplicial(K.coords, K.simplices, "ones", [])
    if mode == "int":
        return synth.Simplicial(K.coords, K.simplices, "explicit",
                                [g.integers(-50, 51, size=c).astype(np.int32) for c in counts])
    if mode == "f32":
        return synth.Simplicial(K.coords, K.simplices, "explicit",
                                [g.lognormal(0.0, 0.5, size=c).astype(np.float32) for c in counts])
    return synth.Simplicial(K.coords, K.simplices, "vertex_max",
                            [g.normal(1.0, 0.2, size=counts[0]).astype(np.float32)])


def _freud(nx, ny, seed, jitter=0.01):
    coords, edges, tris = synth.freudenthal_grid(nx, ny, jitter, synth.rng(77, seed, 0))
    return synth.Simplicial(coords, [None, edges, tris], "ones", [])


def _kuhn(n, seed, jitter=0.005):
    coords, edges, tris, tets = synth.kuhn_grid(n, jitter, synth.rng(78, seed, 0))
    return synth.Simplicial(coords, [None, edges, tris, tets], "ones", [])


def _shuffled(K, seed):
    """Same complex with its vertex ids permuted at random (no locality)."""
    g = np.random.default_rng(seed)
    V = K.coords.shape[0]
    perm = g.permutation(V)          # new id of old vertex v
    inv = np.argsort(perm)
    coords = K.coords[inv]
    simp = [None] + [perm[s].astype(np.int32) for s in K.simplices[1:]]
    w = list(K.weights)
    if K.wmode == "vertex_max" or (K.wmode == "explicit" and w):
        w[0] = w[0][inv]
    return synth.Simplicial(coords, simp, K.wmode, w)


# ---------------------------------------------------------------------------
# forward parity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["ones", "int", "f32", "vmax"])
def test_region_2d_weight_modes(W, mode):
    Ks = [_reweight(_freud(30, 17, 0), mode, 1), _reweight(_freud(12, 41, 1), mode, 2),
          _reweight(_freud(47, 9, 2), mode, 3)]
    _check(W, Ks, synth.s1_directions(64), synth.uniform_thresholds(64, 1.45), f"2d batch {mode} d64 T64")


@pytest.mark.parametrize("T", [1, 2, 129, 255, 256, 300, 1000])
def test_region_3d_thresholds(W, T):
    """T = 256 takes the table's overflow bits (thresholds below the largest
    heights, so some vertices are above every threshold); 300 and 1000 run as
    threshold tiles of at most 256."""
    Ks = [_reweight(_kuhn(7, 0), "f32", 5), _reweight(_kuhn(5, 1), "f32", 6)]
    thr = synth.uniform_thresholds(T, 1.2) if T > 1 else np.array([0.1], np.float32)
    _check(W, Ks, synth.fibonacci_directions(70), thr, f"3d kuhn f32 d70 T{T}")
    Ki = [_reweight(K, "int", 7) for K in Ks]
    _check(W, Ki, synth.fibonacci_directions(70), thr, f"3d kuhn int d70 T{T}", oracle_check=(T <= 300))


def test_region_tiny_random_complexes(W):
    """Random face-closed complexes of dimensions 1..3 in R^1..R^3 (height and
    threshold ties from lattice-snapped coordinates), in one batch per mode."""
    for n, top in ((1, 1), (2, 2), (3, 3), (3, 2), (2, 1)):
        for mode, wd in (("explicit", np.int32), ("explicit", np.float32), ("vertex_max", np.float32),
                         ("ones", np.int32)):
            Ks = [synth.random_tiny_complex(100 * n + 10 * top + s, n=n, nv=10, top_dim=top, wmode=mode,
                                            wdtype=wd) for s in range(5)]
            thr = synth.uniform_thresholds(9, 1.5)
            _check(W, Ks, synth.s1_directions(5) if n == 2 else
                   (synth.fibonacci_directions(5) if n == 3 else np.array([[1.0], [-1.0]], np.float32)),
                   thr, f"tiny random n{n} top{top} {mode} {np.dtype(wd).name}")


def test_region_uneven_batch_with_vertex_only_complex(W):
    """A batch mixing sizes (several regions, one region, a complex of one
    triangle, a complex whose vertices have no cofaces in range of the others)."""
    tri = synth.single_triangle(True)
    Ks = [_reweight(_freud(40, 33, 3), "vmax", 8), _reweight(_freud(3, 3, 4), "vmax", 9),
          synth.Simplicial(tri.coords, tri.simplices, "vertex_max", [np.array([0.5, 2.0, 1.0], np.float32)]),
          _reweight(_freud(25, 2, 5), "vmax", 10)]
    _check(W, Ks, synth.s1_directions(130), synth.uniform_thresholds(128, 1.42), "uneven 2d batch vmax d130 T128")


def test_region_shuffled_vertex_ids_take_the_slow_path(W):
    """Vertex ids without locality: a region's halo exceeds the LDS table, so
    those vertices' indices come from global memory; same bits as without."""
    Ks = [_shuffled(_reweight(_freud(70, 70, 6), "f32", 11), 12)]
    _check(W, Ks, synth.s1_directions(64), synth.uniform_thresholds(128, 1.42), "shuffled 70x70 f32")
    Ks = [_shuffled(_reweight(_kuhn(9, 2), "f32", 13), 14)]
    _check(W, Ks, synth.fibonacci_directions(64), synth.uniform_thresholds(256, 1.2), "shuffled kuhn9 f32 T256")


def test_region_full_size_workloads_same_bits(W):
    """The 3D Kuhn mesh 64^3 (float32 weights, d = 256, T = 256) and the
    differentiation batch (64 complexes of 10^4..2*10^5 vertices, vertex-max
    weights, d = 128, T = 128): same bits as the per-cell forward, which the
    other parity tests compare with the oracle at these sizes."""
    w3 = synth.cfg3()
    _check(W, w3.complexes, w3.dirs, w3.thr, "kuhn64 full", oracle_check=False)
    w5 = synth.cfg5()
    _check(W, w5.complexes, w5.dirs, w5.thr, "differentiation batch full", oracle_check=False)


def test_region_batched_forward_and_backward(W):
    """wect_batched with the index: the forward reads the index, the adjoint
    streams cells as before (same gradients as without the index)."""
    w = synth.cfg5(n_complexes=5, vmin=500, vmax=4000)
    cx = W.SimplicialBatch.from_host(w.complexes)
    g = W.Grid(w.dirs, w.thr)
    gout = torch.randn(cx.B, g.d, g.T, device="cuda")
    o0, g0 = W.wect_batched(cx, g, gout)
    o0, g0 = o0.clone(), g0.clone()
    W.region_index(cx)
    o1, g1 = W.wect_batched(cx, g, gout)
    torch.cuda.synchronize()
    assert torch.equal(o0.view(torch.int32), o1.view(torch.int32))
    scale = float(g0.abs().max())
    assert torch.allclose(g0, g1, rtol=1e-5, atol=1e-5 * scale)


def test_region_graph_capture(W):
    w = synth.cfg5(n_complexes=6, vmin=500, vmax=3000)
    cx = W.SimplicialBatch.from_host(w.complexes)
    g = W.Grid(w.dirs, w.thr)
    W.region_index(cx)
    ref = W.wect_forward(cx, g).clone()
    ws = torch.empty(max(1, W.wect_workspace_bytes(cx, g, False)), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        W.wect_forward(cx, g, out=out, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    _say("region forward graph capture")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        W.wect_forward(cx, g, out=out, ws=ws)
    for rep in range(3):
        out.fill_(-7.0)
        _ = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), rep


def test_region_noalloc(W):
    from paper_2511_03909_amd import _lib as L
    w = synth.cfg3(n=12)
    cx = W.SimplicialBatch.from_host(w.complexes)
    g = W.Grid(w.dirs, w.thr)
    W.region_index(cx)
    ref = W.wect_forward(cx, g).clone()
    out = torch.full_like(ref, -7)
    c, gg = cx.struct(), g.struct()
    st = L.lib().wect_forward_noalloc(ctypes.byref(c), ctypes.byref(gg), out.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == 0
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))


def test_region_refuses_a_hub_and_a_short_buffer(W):
    """A vertex of degree 20000 whose region references more vertices above it
    than the build sorts: WECT_ERR_UNSUPPORTED, and the forward without the
    index still works.  An index buffer below wect_region_bytes is refused."""
    from paper_2511_03909_amd import _lib as L
    V = 20001
    g = np.random.default_rng(0)
    coords = g.uniform(-1, 1, size=(V, 2)).astype(np.float32)
    edges = np.stack([np.zeros(V - 1, np.int32), np.arange(1, V, dtype=np.int32)], 1)
    K = synth.Simplicial(coords, [None, edges], "ones", [])
    cx = W.SimplicialBatch.from_host([K])
    with pytest.raises(L.WectError) as ei:
        W.region_index(cx)
    assert ei.value.status == L.WECT_ERR_UNSUPPORTED
    assert cx.cell_index is None
    out = W.wect_forward(cx, W.Grid(synth.s1_directions(8), synth.uniform_thresholds(16, 1.5))).cpu().numpy()
    assert np.array_equal(out[0].astype(np.int64), oracle.wect(K, synth.s1_directions(8),
                                                               synth.uniform_thresholds(16, 1.5)))
    K2 = _freud(10, 10, 0)
    cx2 = W.SimplicialBatch.from_host([K2])
    idx = W.region_index(cx2)
    cx2.cell_index = idx[: idx.numel() - 256]
    with pytest.raises(L.WectError) as ei:
        W.wect_forward(cx2, W.Grid(synth.s1_directions(8), synth.uniform_thresholds(16, 1.5)))
    assert ei.value.status == L.WECT_ERR_ARG


# ---------------------------------------------------------------------------
# the index against its documented layout
# ---------------------------------------------------------------------------

def _a256(x):
    return (x + 255) // 256 * 256


def _decode(idx, B, counts, top_dim):
    """Split the downloaded index into its sections (layout of include/wect.h)."""
    R = 64 if top_dim >= 3 else 384
    V = counts[0]
    nrmax = (V + R - 1) // R + B
    raw = idx.cpu().numpy()
    o = 0
    sec = {}

    def take(name, nbytes, dt):
        nonlocal o
        sec[name] = raw[o:o + nbytes].view(dt) if nbytes else np.zeros(0, dt)
        o += _a256(nbytes)

    take("hdr", 64, np.int64)
    take("reg", (B + 1) * 8, np.int64)
    take("cnt", 4 * (nrmax + 1) * 8, np.int64)
    for i in range(1, top_dim + 1):
        take(f"coff{i}", (nrmax + 1) * 8, np.int64)
        take(f"perm{i}", counts[i] * 4, np.int32)
        take(f"rec{i}", counts[i] * (4 if i == 1 else 8), np.uint16)
    take("hoff", (nrmax + 1) * 8, np.int64)
    take("hcnt", nrmax * 4, np.int32)
    nhalo = sum(i * counts[i] for i in range(1, top_dim + 1))
    take("halo", max(nhalo, 1) * 4, np.int32)
    return R, sec


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_region_index_layout(W, which):
    if which == "2d":
        Ks = [_freud(30, 17, 0), _freud(5, 4, 1), _freud(41, 20, 2)]
    else:
        Ks = [_kuhn(6, 0), _kuhn(3, 1), _kuhn(5, 2)]
    _say(f"region index layout {which}")
    cx = W.SimplicialBatch.from_host(Ks)
    idx = W.region_index(cx, attach=False)
    torch.cuda.synchronize()
    top = cx.top_dim
    counts = cx.counts + [0] * (4 - len(cx.counts))
    R, sec = _decode(idx, cx.B, counts, top)
    vcount = [K.coords.shape[0] for K in Ks]
    voffs = np.concatenate([[0], np.cumsum(vcount)])
    nreg = [(v + R - 1) // R for v in vcount]
    assert sec["hdr"][0] == R and sec["hdr"][1] == sum(nreg) and sec["hdr"][2] == 0
    assert np.array_equal(sec["reg"], np.concatenate([[0], np.cumsum(nreg)]))
    NR = sum(nreg)
    # per dimension: global rows of every complex's cells, and their complex
    for i in range(1, top + 1):
        rows_of = []
        for b, K in enumerate(Ks):
            rows_of.append(np.asarray(K.simplices[i], np.int64))
        simp = np.concatenate(rows_of)
        comp = np.concatenate([np.full(len(r), b) for b, r in enumerate(rows_of)])
        coff, perm = sec[f"coff{i}"], sec[f"perm{i}"]
        assert coff[0] == 0 and coff[NR] == counts[i]
        assert np.array_equal(np.sort(perm), np.arange(counts[i])), f"dim {i}: not a permutation"
        rec = sec[f"rec{i}"].reshape(counts[i], 2 if i == 1 else 4)
        for r in range(NR):
            b = int(np.searchsorted(sec["reg"][1:], r, side="right"))
            k = r - sec["reg"][b]
            vlo, vhi = k * R, min(k * R + R, vcount[b])
            nown = vhi - vlo
            cells = perm[coff[r]:coff[r + 1]]
            assert np.all(comp[cells] == b)
            verts = simp[cells]
            assert np.all((verts.min(1) >= vlo) & (verts.min(1) < vhi)), f"dim {i} region {r}: wrong region"
            H = sec["hcnt"][r]
            halo = sec["halo"][sec["hoff"][r]:sec["hoff"][r] + H] - voffs[b]
            assert np.all(np.diff(halo) > 0), "halo not sorted / not unique"
            # decode local ids
            ids = rec[coff[r]:coff[r + 1], :i + 1].astype(np.int64)
            dec = np.where(ids < nown, ids + vlo, halo[np.clip(ids - nown, 0, H - 1)] if H else ids + vlo)
            assert np.array_equal(dec, verts), f"dim {i} region {r}: local ids do not decode"
            if i == 2:
                assert np.array_equal(rec[coff[r]:coff[r + 1], 3], rec[coff[r]:coff[r + 1], 2])
    # halos are exactly the vertices above the region that its cells use
    for r in range(NR):
        b = int(np.searchsorted(sec["reg"][1:], r, side="right"))
        k = r - sec["reg"][b]
        vhi = min(k * R + R, vcount[b])
        want = set()
        for i in range(1, top + 1):
            simp = np.concatenate([np.asarray(K.simplices[i], np.int64) for K in Ks])
            cells = sec[f"perm{i}"][sec[f"coff{i}"][r]:sec[f"coff{i}"][r + 1]]
            v = simp[cells].ravel()
            want.update(int(x) for x in v[v >= vhi])
        H = sec["hcnt"][r]
        got = set(int(x) for x in sec["halo"][sec["hoff"][r]:sec["hoff"][r] + H] - voffs[b])
        assert got == want, f"region {r}: halo {sorted(got)[:5]} != {sorted(want)[:5]}"
