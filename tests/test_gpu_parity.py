"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer outputs must be bit-exact.  Float32 outputs must be within
1e-5 * sum|w| of the oracle's float64 value for every complex; every float32
case is also re-run with unit and with integer weights, bit-exact, so that the
tolerance cannot hide a dropped or duplicated cell."""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")
F32_RTOL = 1e-5


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def W():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_03909_amd import api
    api.set_launch()  # defaults
    return api


def gpu_wect(W, complexes, dirs, thr):
    complexes = list(complexes)
    if hasattr(complexes[0], "intensity"):
        cx = W.CubicalBatch.from_host(complexes)
    else:
        cx = W.SimplicialBatch.from_host(complexes)
    g = W.Grid(dirs, thr)
    out = W.wect_forward(cx, g)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_match(got, ref, X, what):
    if np.issubdtype(ref.dtype, np.integer):
        assert got.dtype == np.int32
        assert np.all(np.abs(ref) < 2 ** 31), "oracle value outside int32"
        bad = np.argwhere(got.astype(np.int64) != ref)
        assert bad.size == 0, f"{what}: {len(bad)} mismatches, first {bad[:5].tolist()}"
    else:
        tol = F32_RTOL * max(oracle.total_abs_weight(X), 1e-30)
        err = np.abs(got.astype(np.float64) - ref).max() if ref.size else 0.0
        assert err <= tol, f"{what}: max error {err} > {tol}"


def with_weights(K, mode, seed=0):
    """Same complex, weights replaced: 'ones' or random 'int'."""
    if mode == "ones":
        return synth.Simplicial(K.coords, K.simplices, "ones", [])
    g = np.random.default_rng(seed)
    counts = K.counts()
    return synth.Simplicial(K.coords, K.simplices, "explicit",
                            [g.integers(-50, 51, size=c).astype(np.int32) for c in counts])


# ---------------------------------------------------------------------------
# hand examples
# ---------------------------------------------------------------------------

def test_hand_examples(W):
    with open(os.path.join(GOLD, "hand_examples.json")) as f:
        hand = json.load(f)
    dirs = synth.hand_directions()
    thr = np.array(hand["thresholds"], np.float32)
    _say("hand triangle unweighted")
    got = gpu_wect(W, [synth.single_triangle(False)], dirs, thr)[0]
    assert np.array_equal(got, hand["triangle"]["unweighted"])
    _say("hand triangle weighted")
    got = gpu_wect(W, [synth.single_triangle(True)], dirs, thr)[0]
    assert np.allclose(got, hand["triangle"]["weighted"], rtol=0, atol=1e-6)
    for weighted, key in ((True, "weighted"), (False, "unweighted")):
        _say(f"hand square {key}")
        got = gpu_wect(W, [synth.single_square(weighted)], dirs, thr)[0]
        assert np.array_equal(got, hand["square"][key]), key


def test_rounding_order(W):
    with open(os.path.join(GOLD, "rounding_order.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        _say(f"rounding {case['name']}")
        K = synth.Simplicial(np.array([case["coord"]], np.float32), [None], "ones", [])
        got = gpu_wect(W, [K], np.array([case["dir"]], np.float32), np.array([case["threshold"]], np.float32))
        assert got[0, 0, 0] == case["expected_count"]


# ---------------------------------------------------------------------------
# random tiny complexes
# ---------------------------------------------------------------------------

TINY = [(seed, n, top, wm, wdt) for seed in range(3) for n, top in ((1, 1), (2, 2), (3, 3))
        for wm, wdt in (("ones", np.int32), ("explicit", np.int32), ("explicit", np.float32),
                        ("vertex_max", np.float32))]


@pytest.mark.parametrize("seed,n,top,wm,wdt", TINY)
def test_tiny_simplicial(W, seed, n, top, wm, wdt):
    _say(f"tiny simplicial seed={seed} n={n} top={top} {wm} {np.dtype(wdt).name}")
    K = synth.random_tiny_complex(seed, n=n, nv=10, top_dim=top, wmode=wm, wdtype=wdt)
    dirs = (synth.fibonacci_directions(70) if n == 3 else synth.s1_directions(70) if n == 2
            else np.array([[1.0], [-1.0], [0.5], [0.0]], np.float32))
    thr = synth.uniform_thresholds(37, 1.6)
    got = gpu_wect(W, [K], dirs, thr)[0]
    assert_match(got, oracle.wect(K, dirs, thr), K, "tiny")


@pytest.mark.parametrize("seed", range(3))
def test_tiny_cubical(W, seed):
    for shape in ((7, 5), (1, 6), (5, 4, 3), (3, 1, 4)):
        for weighted in (True, False):
            _say(f"tiny cubical seed={seed} shape={shape} weighted={weighted}")
            C = synth.random_tiny_cubical(seed, shape, include_above=60, weighted=weighted)
            dirs = synth.s1_directions(66) if len(shape) == 2 else synth.fibonacci_directions(66)
            # directions along the axes (zero components) exercise the ties of the top-corner rule
            extra = np.eye(len(shape), dtype=np.float32)
            dirs = np.concatenate([dirs, extra, -extra])
            thr = synth.uniform_thresholds(19, 1.8)
            got = gpu_wect(W, [C], dirs, thr)[0]
            assert_match(got, oracle.wect(C, dirs, thr), C, f"cubical {shape}")


# ---------------------------------------------------------------------------
# threshold arrays: fallback search, duplicates, T = 1, ties
# ---------------------------------------------------------------------------

def test_threshold_variants(W):
    K = synth.random_tiny_complex(7, n=2, nv=12, top_dim=2, wmode="explicit", wdtype=np.int32)
    dirs = synth.s1_directions(40)
    H = oracle.heights(K.coords, dirs)
    g = np.random.default_rng(3)
    variants = {
        "uniform": synth.uniform_thresholds(50, 1.5),
        "random_sorted": np.sort(g.uniform(-1.5, 1.5, size=45)).astype(np.float32),
        "duplicates": np.sort(np.concatenate([synth.uniform_thresholds(20, 1.2)] * 2)).astype(np.float32),
        "T1": np.array([0.25], np.float32),
        "T2": np.array([-0.3, 0.4], np.float32),
        "on_heights": np.unique(np.sort(H.ravel()))[::7].astype(np.float32),
        "perturbed": synth.uniform_thresholds(64, 1.5),
    }
    variants["perturbed"][10] = np.nextafter(variants["perturbed"][10], np.float32(2))
    for name, thr in variants.items():
        _say(f"thresholds {name} T={thr.shape[0]}")
        got = gpu_wect(W, [K], dirs, thr)[0]
        assert_match(got, oracle.wect(K, dirs, thr), K, name)


def test_direction_counts(W):
    K = synth.random_tiny_complex(2, n=3, nv=11, top_dim=3, wmode="explicit", wdtype=np.int32)
    thr = synth.uniform_thresholds(33, 1.8)
    for d in (1, 63, 64, 65, 130):
        _say(f"directions d={d}")
        dirs = synth.fibonacci_directions(d)
        got = gpu_wect(W, [K], dirs, thr)[0]
        assert_match(got, oracle.wect(K, dirs, thr), K, f"d={d}")


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def test_cfg1_full(W):
    _say("cfg1 full")
    w = synth.cfg1()
    got = gpu_wect(W, w.complexes, w.dirs, w.thr)[0]
    assert_match(got, oracle.wect(w.complexes[0], w.dirs, w.thr), w.complexes[0], "cfg1")


def test_cfg2_full_batch_sampled(W):
    _say("cfg2 full batch")
    w = synth.cfg2()
    got = gpu_wect(W, w.complexes, w.dirs, w.thr)
    assert got.shape == (256, 64, 128)
    for b in (0, 1, 77, 255):
        _say(f"cfg2 image {b} all directions")
        assert_match(got[b], oracle.wect(w.complexes[b], w.dirs, w.thr), w.complexes[b], f"cfg2[{b}]")
    for b in range(0, 256, 9):
        assert_match(got[b, [5, 40]], oracle.wect(w.complexes[b], w.dirs, w.thr, dir_index=[5, 40]),
                     w.complexes[b], f"cfg2[{b}] sampled")


def test_cfg3_full_sampled_directions(W):
    _say("cfg3 full")
    w = synth.cfg3()
    K = w.complexes[0]
    got = gpu_wect(W, [K], w.dirs, w.thr)[0]
    sample = [0, 97, 200, 255]
    assert_match(got[sample], oracle.wect(K, w.dirs, w.thr, dir_index=sample), K, "cfg3 f32")
    for mode in ("ones", "int"):
        _say(f"cfg3 rerun with {mode} weights")
        K2 = with_weights(K, mode)
        got2 = gpu_wect(W, [K2], w.dirs, w.thr)[0]
        assert_match(got2[sample], oracle.wect(K2, w.dirs, w.thr, dir_index=sample), K2, f"cfg3 {mode}")
        # full-size property: at the last threshold every cell below it is counted
        chi = oracle.euler_characteristic(K2)
        if mode == "ones":
            H = oracle.heights(K.coords, w.dirs)
            ok_dirs = np.where(H.max(axis=1) <= w.thr[-1])[0]
            assert np.all(got2[ok_dirs, -1] == chi)


def test_cfg4_full_batch_sampled(W):
    _say("cfg4 full batch")
    w = synth.cfg4()
    got = gpu_wect(W, w.complexes, w.dirs, w.thr)
    sizes = [C.intensity.size for C in w.complexes]
    order = np.argsort(sizes)
    for b in (int(order[0]), int(order[-1])):
        _say(f"cfg4 volume {b} size {w.complexes[b].intensity.shape}")
        sample = [3, 300]
        assert_match(got[b, sample], oracle.wect(w.complexes[b], w.dirs, w.thr, dir_index=sample),
                     w.complexes[b], f"cfg4[{b}]")


def test_cfg5_forward_backward(W):
    _say("cfg5 build")
    w = synth.cfg5()
    Ks = w.complexes
    cx = W.SimplicialBatch.from_host(Ks)
    g = W.Grid(w.dirs, w.thr)
    out = W.wect_forward(cx, g)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    sizes = [K.coords.shape[0] for K in Ks]
    pick = [int(np.argmin(sizes)), 17]
    targets = {}
    for b in pick:
        _say(f"cfg5 forward complex {b} V={sizes[b]}")
        sample = [0, 31, 64, 127]
        assert_match(out[b, sample], oracle.wect(Ks[b], w.dirs, w.thr, dir_index=sample), Ks[b], f"cfg5[{b}]")
    # backward: loss = sum (out - target)^2 with target from reseeded weights
    _say("cfg5 backward")
    Kt = [synth.Simplicial(K.coords, K.simplices, "vertex_max", [wt]) for K, wt in
          zip(Ks, w.extra["target_weights"])]
    tgt = W.wect_forward(W.SimplicialBatch.from_host(Kt), g)
    gout = 2.0 * (torch.from_numpy(out).cuda() - tgt)
    gv = W.wect_backward(cx, g, gout)
    torch.cuda.synchronize()
    gv = gv.cpu().numpy()
    voff = np.concatenate([[0], np.cumsum(sizes)])
    b = pick[0]
    _say(f"cfg5 oracle gradient complex {b}")
    gb = gout[b].cpu().numpy().astype(np.float64)
    ref = oracle.wect_backward(Ks[b], w.dirs, w.thr, gb)
    bound = oracle.wect_backward(Ks[b], w.dirs, w.thr, gb, absolute=True)
    mine = gv[voff[b]:voff[b + 1]]
    assert np.all(np.abs(mine - ref) <= 1e-5 * bound + 1e-6), np.abs(mine - ref).max()
    # float64 central differences on a few vertices away from weight ties
    _say("cfg5 finite differences")
    tgt_b = oracle.wect(Kt[b], w.dirs, w.thr)
    wv = Ks[b].weights[0].astype(np.float64)
    e = Ks[b].simplices[1]
    gap = np.full(sizes[b], np.inf)
    diff = np.abs(wv[e[:, 0]] - wv[e[:, 1]])
    np.minimum.at(gap, e[:, 0], diff)
    np.minimum.at(gap, e[:, 1], diff)
    cand = [v for v in range(0, sizes[b], max(1, sizes[b] // 60)) if gap[v] > 2e-3][:6]
    assert len(cand) >= 4
    fd = oracle.fd_vertex_grad(Ks[b], w.dirs, w.thr, tgt_b, cand, eps=1e-3)
    # the oracle's own loss gradient (float64 output) must match the differences
    out_b = oracle.wect(Ks[b], w.dirs, w.thr)
    g64 = 2.0 * (out_b - tgt_b)
    ref64 = oracle.wect_backward(Ks[b], w.dirs, w.thr, g64)
    assert np.allclose(fd, ref64[cand], rtol=1e-8, atol=1e-6)
    # the GPU adjoint seeded with the same loss gradient matches the differences
    cb = W.SimplicialBatch.from_host([Ks[b]])
    gv64 = W.wect_backward(cb, g, torch.from_numpy(g64[None].astype(np.float32)).cuda()).cpu().numpy()
    bound64 = oracle.wect_backward(Ks[b], w.dirs, w.thr, g64, absolute=True)
    assert np.all(np.abs(gv64[cand] - fd) <= 1e-5 * bound64[cand] + 1e-6), (gv64[cand], fd)


# ---------------------------------------------------------------------------
# batching, launch shapes, graphs
# ---------------------------------------------------------------------------

def test_batched_equals_singles(W):
    w = synth.cfg2(n_images=12, side=40)
    _say("cubical batch vs singles")
    both = gpu_wect(W, w.complexes, w.dirs, w.thr)
    for b, C in enumerate(w.complexes):
        assert np.array_equal(both[b], gpu_wect(W, [C], w.dirs, w.thr)[0])
    _say("simplicial uneven batch with an empty member")
    Ks = [synth.random_tiny_complex(s, n=2, nv=6 + 2 * s, top_dim=2, wmode="explicit", wdtype=np.int32)
          for s in range(5)]
    empty = synth.Simplicial(np.zeros((0, 2), np.float32), [None, np.zeros((0, 2), np.int32),
                                                            np.zeros((0, 3), np.int32)],
                             "explicit", [np.zeros(0, np.int32)] * 3)
    Ks.insert(2, empty)
    dirs, thr = synth.s1_directions(70), synth.uniform_thresholds(29, 1.5)
    both = gpu_wect(W, Ks, dirs, thr)
    assert np.all(both[2] == 0)
    for b, K in enumerate(Ks):
        if b == 2:
            continue
        assert_match(both[b], oracle.wect(K, dirs, thr), K, f"batch member {b}")


def test_launch_shapes_give_identical_integers(W):
    K = with_weights(synth.cfg3(n=12).complexes[0], "int")
    dirs, thr = synth.fibonacci_directions(100), synth.uniform_thresholds(77, 1.8)
    ref = None
    try:
        for block in (256, 512, 1024):
            for bpc in (1, 2):
                for mi in (64, 4096):
                    for dec in (W.DECOMP_STREAM, W.DECOMP_GROUP):
                        _say(f"launch block={block} bpc={bpc} min_items={mi} decomposition={dec}")
                        W.set_launch(block, bpc, mi, dec)
                        got = gpu_wect(W, [K], dirs, thr)
                        if ref is None:
                            ref = got
                            assert_match(got[0], oracle.wect(K, dirs, thr), K, "launch ref")
                        assert np.array_equal(got, ref)
    finally:
        W.set_launch()


def test_random_launch_knobs_give_identical_bits(W):
    """Forty random combinations of every launch knob (block, blocks per
    CU, minimum items, decomposition, threshold tile, directions per lane,
    voxel records, cell packing, staging tile) on a 3D volume batch, a 2D
    image batch and simplicial batches with integer and float32 weights: the
    same bits as the automatic plan (integer and 64-bit fixed-point sums are
    exact), which matches the oracle."""
    g = np.random.default_rng(2024)
    vols = [synth.random_tiny_cubical(s, shp, include_above=70) for s, shp in
            enumerate(((9, 7, 5), (4, 11, 3), (6, 6, 6)))]
    ims, Ks = _uneven_batches()
    Kf = [synth.random_tiny_complex(40 + s, n=3, nv=10, top_dim=3, wdtype=np.float32) for s in range(4)]
    cases = [(vols, synth.fibonacci_directions(150), synth.uniform_thresholds(100, 2.0)),
             (ims, synth.s1_directions(20), synth.uniform_thresholds(61, 1.7)),
             (Ks, synth.s1_directions(90), synth.uniform_thresholds(100, 1.8)),
             (Kf, synth.fibonacci_directions(30), synth.uniform_thresholds(300, 2.2))]
    try:
        for ci, (Cs, dirs, thr) in enumerate(cases):
            W.set_launch()
            ref = gpu_wect(W, Cs, dirs, thr)
            for b, C in enumerate(Cs):
                assert_match(ref[b], oracle.wect(C, dirs, thr), C, f"case {ci} complex {b}")
            for trial in range(10):
                knobs = dict(block=int(g.choice([0, 256, 512, 1024])), blocks_per_cu=int(g.choice([0, 1, 2])),
                             min_items_per_block=int(g.choice([0, 64, 5000])), decomposition=int(g.choice([0, 1, 2])),
                             threshold_tile=int(g.choice([0, 7, 33, 64])),
                             directions_per_lane=int(g.choice([0, 1, 2])), cubical_records=int(g.choice([0, 1, 2, 3])),
                             cell_packing=int(g.choice([0, 1])), stage_entries=int(g.choice([0, 64, 192, 448, 1024])))
                _say(f"case {ci} trial {trial}: {knobs}")
                W.set_launch(**knobs)
                got = gpu_wect(W, Cs, dirs, thr)
                assert np.array_equal(got.view(np.int32), ref.view(np.int32)), f"case {ci}: {knobs}"
    finally:
        W.set_launch()


def test_cubical_sparse_volumes_empty_staging_tiles(W):
    """Volumes whose included voxels sit in three small blobs, so that most
    staging tiles stage nothing: the alternating compaction counters and the
    tile barriers meet empty tiles, in stream mode with several blocks per
    group, with and without voxel records and with small staging and
    threshold tiles; against the oracle."""
    g = np.random.default_rng(77)
    vols = []
    for n2, n1, n0 in ((30, 24, 40), (12, 50, 33)):
        a = np.zeros((n2, n1, n0), np.uint8)
        for _ in range(3):
            c = [int(g.integers(0, n)) for n in (n2, n1, n0)]
            sl = tuple(slice(max(0, ci - 2), ci + 3) for ci in c)
            a[sl] = g.integers(1, 256, size=a[sl].shape)
        vols.append(synth.Cubical(a, [synth.cubical_axis(n0), synth.cubical_axis(n1), synth.cubical_axis(n2)], 0, True))
    dirs, thr = synth.fibonacci_directions(200), synth.uniform_thresholds(50, 2.0)
    refs = [oracle.wect(C, dirs, thr) for C in vols]
    try:
        for knobs in (dict(), dict(decomposition=W.DECOMP_STREAM, min_items_per_block=64),
                      dict(decomposition=W.DECOMP_STREAM, min_items_per_block=64, cubical_records=1),
                      dict(cubical_records=2, stage_entries=64, threshold_tile=17),
                      dict(cubical_records=3, decomposition=W.DECOMP_STREAM, min_items_per_block=64)):
            _say(f"sparse volumes {knobs}")
            W.set_launch(**knobs)
            got = gpu_wect(W, vols, dirs, thr)
            for b, C in enumerate(vols):
                assert_match(got[b], refs[b], C, f"{knobs} volume {b}")
    finally:
        W.set_launch()


def test_cubical_two_voxels_per_thread_overflow(W):
    """Records with two voxels per thread (cubical_records = 3) on dense
    volumes and images, where nearly every voxel contributes, so that the
    stage overflows in every tile and the second round carries the rest: the
    oracle's values, at the automatic stage and at a small one, in group and
    stream mode."""
    vols = [synth.random_tiny_cubical(40 + s, shp, include_above=-1) for s, shp in
            enumerate(((20, 18, 23), (31, 7, 12), (9, 40, 10)))]
    ims = [synth.random_tiny_cubical(50 + s, shp, include_above=-1) for s, shp in enumerate(((45, 38), (60, 29)))]
    cases = ((vols, synth.fibonacci_directions(200), synth.uniform_thresholds(60, 2.0)),
             (ims, synth.s1_directions(150), synth.uniform_thresholds(40, 1.7)))
    try:
        for ci, (Cs, dirs, thr) in enumerate(cases):
            refs = [oracle.wect(C, dirs, thr) for C in Cs]
            for knobs in (dict(cubical_records=3), dict(cubical_records=3, stage_entries=128),
                          dict(cubical_records=3, decomposition=W.DECOMP_STREAM, min_items_per_block=64)):
                _say(f"two voxels per thread, case {ci}: {knobs}")
                W.set_launch(**knobs)
                got = gpu_wect(W, Cs, dirs, thr)
                for b, C in enumerate(Cs):
                    assert_match(got[b], refs[b], C, f"case {ci} {knobs} complex {b}")
    finally:
        W.set_launch()


def _uneven_batches():
    ims = [synth.random_tiny_cubical(s, shp, include_above=80) for s, shp in
           enumerate(((12, 9), (3, 17), (20, 1), (7, 7), (16, 11), (9, 30), (2, 2), (25, 13)))]
    ims.insert(3, synth.Cubical(np.zeros((5, 6), np.uint8), [synth.cubical_axis(6), synth.cubical_axis(5)], 80, True))
    Ks = [synth.random_tiny_complex(s, n=2, nv=6 + 3 * s, top_dim=2, wmode="explicit", wdtype=np.int32)
          for s in range(9)]
    Ks.insert(4, synth.Simplicial(np.zeros((0, 2), np.float32), [None, np.zeros((0, 2), np.int32),
                                                                 np.zeros((0, 3), np.int32)],
                                  "explicit", [np.zeros(0, np.int32)] * 3))
    return ims, Ks


@pytest.mark.parametrize("block,mi,dec", [(256, 64, 1), (256, 100000, 1), (1024, 100000, 1), (512, 0, 2),
                                          (1024, 0, 2), (256, 0, 2)])
def test_stream_and_group_decompositions(W, block, mi, dec):
    """Stream ranges that cover several whole groups (written by the block
    itself) next to groups split over blocks (partial histograms + reduction),
    and one block per group; batches with an empty member, ragged tiles."""
    ims, Ks = _uneven_batches()
    dirs, thr = synth.s1_directions(70), synth.uniform_thresholds(37, 1.7)
    try:
        W.set_launch(block, 0, mi, dec)
        _say(f"decomposition={dec} block={block} min_items={mi}: cubical")
        got = gpu_wect(W, ims, dirs, thr)
        for b, C in enumerate(ims):
            assert_match(got[b], oracle.wect(C, dirs, thr), C, f"image {b}")
        _say(f"decomposition={dec} block={block} min_items={mi}: simplicial")
        got = gpu_wect(W, Ks, dirs, thr)
        for b, K in enumerate(Ks):
            assert_match(got[b], oracle.wect(K, dirs, thr), K, f"complex {b}")
        _say(f"decomposition={dec} block={block} min_items={mi}: float weights")
        w = synth.cfg5(n_complexes=5, vmin=300, vmax=2000)
        Kf = w.complexes
        got = gpu_wect(W, Kf, w.dirs, w.thr)
        W.set_launch()
        ref = gpu_wect(W, Kf, w.dirs, w.thr)
        assert np.array_equal(got, ref)  # fixed point: the decomposition does not change the bits
        for b, K in enumerate(Kf[:2]):
            assert_match(got[b], oracle.wect(K, w.dirs, w.thr), K, f"float complex {b}")
        # T a multiple of 4 (vector stores of the directly written groups), into
        # an aligned buffer and into one offset by one element
        W.set_launch(block, 0, mi, dec)
        thr36 = synth.uniform_thresholds(36, 1.7)
        cx = W.CubicalBatch.from_host(ims)
        g = W.Grid(dirs, thr36)
        n = cx.B * g.d * g.T
        flat = torch.full((n + 1,), -7, dtype=torch.int32, device="cuda")
        for off in (0, 1):
            _say(f"decomposition={dec} block={block} min_items={mi}: T=36, out offset {off}")
            view = flat[off:off + n].view(cx.B, g.d, g.T)
            W.wect_forward(cx, g, out=view)
            got = view.cpu().numpy()
            for b, C in enumerate(ims):
                assert_match(got[b], oracle.wect(C, dirs, thr36), C, f"T=36 image {b}")
    finally:
        W.set_launch()


@pytest.mark.parametrize("dec", [1, 2])
def test_cubical_threshold_ranges(W, dec):
    """The cubical forward drops the clamp of its threshold index when every
    height of a complex provably maps inside the threshold range, and keeps a
    per-lane copy of the thresholds when LDS allows: threshold arrays that
    cover every height, that cut heights off at either end, that lie on the
    lattice heights of the diagonal directions, and that are too long for the
    copy, on pixel-lattice and random axes."""
    # 40 x 40 pixel lattice on [-1, 1]^2 with 40 thresholds on [-sqrt2, sqrt2]: along the diagonals
    # every other pixel height is a threshold up to rounding
    ims = [synth.Cubical(synth.random_tiny_cubical(11, (40, 40), include_above=60).intensity,
                         [synth.cubical_axis(40), synth.cubical_axis(40)], 60, True),
           synth.random_tiny_cubical(12, (37, 29), include_above=60),
           synth.Cubical(np.full((6, 9), 200, np.uint8), [synth.cubical_axis(9), synth.cubical_axis(6)], 60, True)]
    vols = [synth.Cubical(synth.random_tiny_cubical(13, (9, 8, 7), include_above=50).intensity,
                          [synth.cubical_axis(9), synth.cubical_axis(8), synth.cubical_axis(7)], 50, True),
            synth.random_tiny_cubical(14, (6, 10, 5), include_above=50)]
    thresholds = {
        "covering": synth.uniform_thresholds(128, 3.0),
        "lattice": synth.uniform_thresholds(40, math.sqrt(2)),
        "narrow": synth.uniform_thresholds(128, 0.4),
        "above": np.linspace(0.3, 1.2, 100).astype(np.float32),
        "below": np.linspace(-1.6, -0.9, 77).astype(np.float32),
        "long": synth.uniform_thresholds(300, 1.5),
        "T2": np.array([-0.2, 0.3], np.float32),
    }
    d2 = np.concatenate([synth.s1_directions(64), np.eye(2, dtype=np.float32)])
    d3 = np.concatenate([synth.fibonacci_directions(60), np.eye(3, dtype=np.float32)])
    try:
        W.set_launch(1024, 0, 0, dec)
        for name, thr in thresholds.items():
            for batch, dirs in ((ims, d2), (vols, d3)):
                _say(f"cubical thresholds {name} T={thr.shape[0]} n={len(batch[0].axes)} decomposition={dec}")
                got = gpu_wect(W, batch, dirs, thr)
                for b, C in enumerate(batch):
                    assert_match(got[b], oracle.wect(C, dirs, thr), C, f"{name} complex {b}")
    finally:
        W.set_launch()


def test_float_results_independent_of_launch_shape(W):
    """Float32 weights accumulate as 64-bit fixed point, so the result does not
    depend on the order of the additions: every launch shape gives the same bits."""
    K = synth.cfg3(n=14).complexes[0]
    dirs, thr = synth.fibonacci_directions(100), synth.uniform_thresholds(77, 1.8)
    ref = None
    try:
        for block, bpc, mi in ((1024, 1, 0), (512, 2, 64), (256, 4, 300), (1024, 1, 100000)):
            _say(f"float launch block={block} bpc={bpc} min_items={mi}")
            W.set_launch(block, bpc, mi)
            got = gpu_wect(W, [K], dirs, thr)
            if ref is None:
                ref = got
                assert_match(got[0], oracle.wect(K, dirs, thr), K, "float launch ref")
            assert np.array_equal(got, ref)
    finally:
        W.set_launch()


def test_graph_capture_forward_backward(W):
    w = synth.cfg5(n_complexes=6, vmin=500, vmax=3000)
    cx = W.SimplicialBatch.from_host(w.complexes)
    g = W.Grid(w.dirs, w.thr)
    B, d, T = cx.B, g.d, g.T
    gout = torch.randn(B, d, T, device="cuda")
    out_e, gv_e = W.wect_batched(cx, g, gout)
    torch.cuda.synchronize()
    out_e, gv_e = out_e.clone(), gv_e.clone()
    ws = torch.empty(W.wect_workspace_bytes(cx, g, True), dtype=torch.uint8, device="cuda")
    out = torch.empty(B, d, T, device="cuda")
    gv = torch.empty(cx.counts[0], device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        W.wect_batched(cx, g, gout, out=out, grads=gv, ws=ws)  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    _say("graph capture")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        W.wect_batched(cx, g, gout, out=out, grads=gv, ws=ws)
    for rep in range(3):
        out.fill_(-7.0)
        gv.fill_(123.0)
        _ = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.allclose(out, out_e, rtol=0, atol=1e-4 * float(out_e.abs().max()) + 1e-6), rep
        assert torch.allclose(gv, gv_e, rtol=1e-5, atol=1e-4 * float(gv_e.abs().max()) + 1e-6), rep


def test_autograd_function(W):
    w = synth.cfg5(n_complexes=3, vmin=300, vmax=900)
    cx = W.SimplicialBatch.from_host(w.complexes)
    g = W.Grid(w.dirs, w.thr)
    wv = cx.weights[0].clone().requires_grad_(True)
    out = W.wect(cx, g, wv)
    loss = (out ** 2).sum()
    loss.backward()
    ref = W.wect_backward(cx.with_weights([wv.detach()]), g, 2 * out.detach())
    torch.cuda.synchronize()
    # float atomics accumulate the per-vertex sums in no fixed order
    scale = float(ref.abs().max())
    assert torch.allclose(wv.grad, ref, rtol=1e-5, atol=1e-5 * scale)


def test_validate_detects_bad_data(W):
    from paper_2511_03909_amd import _lib as L
    K = synth.random_tiny_complex(1, n=2, nv=8, top_dim=2, wmode="explicit", wdtype=np.float32)
    dirs, thr = synth.s1_directions(8), synth.uniform_thresholds(9, 1.5)
    cx = W.SimplicialBatch.from_host([K])
    W.wect_validate(cx, W.Grid(dirs, thr))
    bad = cx.simplices[1].clone()
    bad[0, 0] = 99
    cxb = W.SimplicialBatch(cx.coords, [None, bad, cx.simplices[2]], cx.wmode, cx.weights)
    with pytest.raises(L.WectError) as e:
        W.wect_validate(cxb, W.Grid(dirs, thr))
    assert e.value.status == L.WECT_ERR_INDEX
    with pytest.raises(L.WectError) as e:
        W.wect_validate(cx, W.Grid(dirs, thr[::-1].copy()))
    assert e.value.status == L.WECT_ERR_THRESHOLDS
    nanc = cx.coords.clone()
    nanc[1, 0] = float("nan")
    with pytest.raises(L.WectError) as e:
        W.wect_validate(W.SimplicialBatch(nanc, cx.simplices, cx.wmode, cx.weights), W.Grid(dirs, thr))
    assert e.value.status == L.WECT_ERR_NONFINITE
    C = synth.random_tiny_cubical(0, (5, 4))
    cc = W.CubicalBatch.from_host([C])
    W.wect_validate(cc, W.Grid(dirs, thr))
    cc.axis[1] = cc.axis[0]
    with pytest.raises(L.WectError) as e:
        W.wect_validate(cc, W.Grid(dirs, thr))
    assert e.value.status == L.WECT_ERR_THRESHOLDS


def test_autotuner_caches_and_keeps_results(W, tmp_path):
    from paper_2511_03909_amd import tune
    w = synth.cfg2(n_images=6, side=48)
    cx = W.CubicalBatch.from_host(w.complexes)
    g = W.Grid(w.dirs, w.thr)
    ref = W.wect_forward(cx, g).cpu().numpy()
    cache = str(tmp_path / "tune.json")
    try:
        best = tune.tune(cx, g, candidates=((512, 0, 0, 1), (1024, 1, 0, 1), (256, 4, 64, 1), (512, 0, 0, 2)),
                         reps=3, cache=cache)
        assert tune.lookup(cx, g, cache) is not None
        # four shapes, then the threshold tiles with the fastest of them
        assert best["block"] in (256, 512, 1024)
        assert len(best["tried"]) == 4 + len(tune.tile_candidates(g.T)) - 1 + len(tune.lane_candidates(cx, g))
        assert best["threshold_tile"] in tune.tile_candidates(g.T)
        assert np.array_equal(W.wect_forward(cx, g).cpu().numpy(), ref)
    finally:
        W.set_launch()


def test_autotuner_simplicial_staging_tiles(W, tmp_path):
    """Simplicial requests also time staging tiles of a half and three
    quarters of the block; the chosen shape gives the same bits (64-bit fixed
    point)."""
    from paper_2511_03909_amd import tune
    w = synth.cfg5(n_complexes=5, vmin=3000, vmax=9000)
    cx = W.SimplicialBatch.from_host(w.complexes)
    g = W.Grid(w.dirs, w.thr)
    ref = W.wect_forward(cx, g).cpu().numpy()
    try:
        best = tune.tune(cx, g, candidates=((1024, 0, 0, 1), (512, 0, 0, 1)), reps=3, cache=str(tmp_path / "t.json"))
        tried = best["tried"]
        assert len(tried) == 2 + len(tune.tile_candidates(g.T)) - 1 + len(tune.stage_candidates(cx, best["block"]))
        assert {t["stage_entries"] for t in tried} >= set(tune.stage_candidates(cx, best["block"]))
        assert best["stage_entries"] in (0, *tune.stage_candidates(cx, best["block"]))
        assert W.get_launch()["stage_entries"] == best["stage_entries"]
        assert np.array_equal(W.wect_forward(cx, g).cpu().numpy().view(np.int32), ref.view(np.int32))
        for st in (64, 192, 640):
            W.set_launch(stage_entries=st)
            assert np.array_equal(W.wect_forward(cx, g).cpu().numpy().view(np.int32), ref.view(np.int32)), st
    finally:
        W.set_launch()


def test_cubical_staging_tiles_give_identical_integers(W):
    """wect_launch.stage_entries on the cubical forward: every staging tile (one
    and two directions per lane, with and without per-voxel records) gives the
    oracle's integers."""
    ims = [synth.random_tiny_cubical(s, shp, include_above=60) for s, shp in
           enumerate(((33, 29), (17, 40), (5, 3), (50, 21)))]
    vols = [synth.random_tiny_cubical(s, shp, include_above=80) for s, shp in
            enumerate(((13, 11, 9), (7, 20, 6), (4, 4, 4)))]
    cases = ((ims, synth.s1_directions(150), synth.uniform_thresholds(67, 1.7)),
             (vols, synth.fibonacci_directions(140), synth.uniform_thresholds(256, 2.0)))
    try:
        for Cs, dirs, thr in cases:
            refs = [oracle.wect(C, dirs, thr) for C in Cs]
            for st in (64, 192, 320, 1024):
                for dpl in (1, 2):
                    for rec in (1, 2):
                        _say(f"cubical staging tile {st}, dpl={dpl}, records={rec}, n={Cs[0].n}")
                        W.set_launch(stage_entries=st, directions_per_lane=dpl, cubical_records=rec)
                        got = gpu_wect(W, Cs, dirs, thr)
                        for b, C in enumerate(Cs):
                            assert_match(got[b], refs[b], C, f"stage={st} dpl={dpl} rec={rec} complex {b}")
    finally:
        W.set_launch()


def test_many_small_complexes_one_block_per_group(W):
    """Batches with more groups than compute units run one block per group
    (512-thread blocks for small groups): hundreds of tiny images of uneven
    shapes, some without any vertex, and hundreds of tiny simplicial complexes
    with two direction tiles, each against the oracle."""
    g = np.random.default_rng(91)
    ims = []
    for i in range(600):
        nx, ny = (int(v) for v in g.integers(1, 7, size=2))
        if i % 97 == 0:
            ims.append(synth.Cubical(np.zeros((ny, nx), np.uint8), [synth.cubical_axis(nx), synth.cubical_axis(ny)],
                                     50, True))
        else:
            ims.append(synth.random_tiny_cubical(1000 + i, (nx, ny), include_above=50))
    dirs, thr = synth.s1_directions(64), synth.uniform_thresholds(40, 1.6)
    _say("600 tiny images, one block per group")
    got = gpu_wect(W, ims, dirs, thr)
    for b, C in enumerate(ims):
        assert_match(got[b], oracle.wect(C, dirs, thr), C, f"image {b}")
    Ks = [synth.random_tiny_complex(2000 + i, n=2, nv=7, top_dim=2, wmode="explicit", wdtype=np.int32)
          for i in range(300)]
    dirs2, thr2 = synth.s1_directions(70), synth.uniform_thresholds(33, 1.8)
    _say("300 tiny complexes, d = 70, one block per group")
    got = gpu_wect(W, Ks, dirs2, thr2)
    for b, K in enumerate(Ks):
        assert_match(got[b], oracle.wect(K, dirs2, thr2), K, f"complex {b}")


@pytest.mark.parametrize("T", [255, 256, 257, 300, 500])
def test_many_thresholds(W, T):
    """T above 256 takes the two-pass scan (row-group totals, then the scan) and smaller staging tiles."""
    _say(f"many thresholds T={T}")
    Ki = synth.random_tiny_complex(11, n=3, nv=12, top_dim=3, wmode="explicit", wdtype=np.int32)
    Kf = synth.random_tiny_complex(11, n=3, nv=12, top_dim=3, wmode="explicit", wdtype=np.float32)
    dirs, thr = synth.fibonacci_directions(70), synth.uniform_thresholds(T, 2.0)
    for K in (Ki, Kf):
        # float weights above about 290 thresholds (64-bit histogram) run in threshold tiles
        assert_match(gpu_wect(W, [K], dirs, thr)[0], oracle.wect(K, dirs, thr), K, f"T={T}")
    C = synth.random_tiny_cubical(3, (9, 7, 5), include_above=40)
    assert_match(gpu_wect(W, [C], dirs, thr)[0], oracle.wect(C, dirs, thr), C, f"cubical T={T}")


def test_many_directions_and_uneven_cubical_batch(W):
    """d = 300 (five tiles, ragged last one) on a batch of images of different
    shapes, one of them with no vertex at all."""
    ims = [synth.random_tiny_cubical(s, shp, include_above=90) for s, shp in
           enumerate(((12, 9), (3, 17), (20, 1), (7, 7), (16, 11)))]
    ims.append(synth.Cubical(np.zeros((5, 6), np.uint8), [synth.cubical_axis(6), synth.cubical_axis(5)], 90, True))
    dirs, thr = synth.s1_directions(300), synth.uniform_thresholds(41, 1.8)
    _say("uneven cubical batch, d=300")
    got = gpu_wect(W, ims, dirs, thr)
    assert np.all(got[-1] == 0)
    for b, C in enumerate(ims[:-1]):
        assert_match(got[b], oracle.wect(C, dirs, thr), C, f"image {b}")
    vols = [synth.random_tiny_cubical(s, shp, include_above=70) for s, shp in
            enumerate(((6, 5, 4), (3, 8, 2), (1, 1, 9), (5, 5, 5)))]
    dirs3 = synth.fibonacci_directions(130)
    _say("uneven cubical volume batch, d=130")
    got = gpu_wect(W, vols, dirs3, thr)
    for b, C in enumerate(vols):
        assert_match(got[b], oracle.wect(C, dirs3, thr), C, f"volume {b}")


def test_include_all_and_unweighted_volume(W):
    C = synth.random_tiny_cubical(5, (6, 7, 5), include_above=-1, weighted=False)
    dirs, thr = synth.fibonacci_directions(64), synth.uniform_thresholds(33, 1.8)
    got = gpu_wect(W, [C], dirs, thr)[0]
    ref = oracle.wect(C, dirs, thr)
    assert_match(got, ref, C, "all included")
    assert np.all(ref[:, -1] == 1)  # a solid box is contractible


def test_graph_replay_cubical_forward(W):
    w = synth.cfg2(n_images=9, side=33)
    cx = W.CubicalBatch.from_host(w.complexes)
    g = W.Grid(w.dirs, w.thr)
    ref = W.wect_forward(cx, g).clone()
    out = torch.empty_like(ref)
    ws = torch.empty(max(1, W.wect_workspace_bytes(cx, g)), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        W.wect_forward(cx, g, out=out, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        W.wect_forward(cx, g, out=out, ws=ws)
    for _ in range(3):
        out.fill_(-1)
        _ = torch.randn(500, device="cuda").sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


@pytest.mark.parametrize("T", [300, 301])
def test_group_decomposition_many_thresholds(W, T):
    """One block per group with long rows: the in-place chunked scan of the
    directly written groups (vector stores when T is a multiple of 4)."""
    ims = [synth.random_tiny_cubical(s, shp, include_above=60) for s, shp in
           enumerate(((40, 33), (7, 51), (64, 9)))]
    dirs, thr = synth.s1_directions(70), synth.uniform_thresholds(T, 1.8)
    try:
        W.set_launch(1024, 0, 0, W.DECOMP_GROUP)
        _say(f"group decomposition, T={T}")
        got = gpu_wect(W, ims, dirs, thr)
    finally:
        W.set_launch()
    for b, C in enumerate(ims):
        assert_match(got[b], oracle.wect(C, dirs, thr), C, f"image {b}")


@pytest.mark.parametrize("wdt", [np.int32, np.float32])
def test_simplex_order_gives_identical_bits(W, wdt):
    """Permuting the simplex rows of each dimension and the vertices within each
    row changes the stream order but no cell's index or weight: the forward
    (integer sums, or 64-bit fixed point for float weights) is bit-identical,
    and so is the explicit-weight adjoint once its rows are put back (one
    direction tile: each simplex's gradient is one lane sum, no atomics)."""
    K = synth.cfg3(n=8).complexes[0]  # 3D Kuhn grid, 9,843 simplices, float32 weights
    g = np.random.default_rng(21)
    if wdt == np.int32:
        K = synth.Simplicial(K.coords, K.simplices, "explicit",
                             [g.integers(-50, 51, size=c).astype(np.int32) for c in K.counts()])
    simp, ws, perms = [None], [K.weights[0]], [None]
    for dim in range(1, 4):
        perm = g.permutation(K.simplices[dim].shape[0])
        rows = np.array([g.permutation(r) for r in K.simplices[dim][perm]], np.int32).reshape(-1, dim + 1)
        simp.append(np.ascontiguousarray(rows))
        ws.append(K.weights[dim][perm])
        perms.append(perm)
    K2 = synth.Simplicial(K.coords, simp, "explicit", ws)
    dirs, thr = synth.fibonacci_directions(64), synth.uniform_thresholds(40, 1.8)
    _say(f"simplex order forward wdt={np.dtype(wdt).name}")
    a = gpu_wect(W, [K], dirs, thr)
    b = gpu_wect(W, [K2], dirs, thr)
    assert np.array_equal(a, b)
    assert_match(a[0], oracle.wect(K, dirs, thr), K, "simplex order")
    if wdt == np.float32:
        _say("simplex order adjoint")
        G = torch.from_numpy(np.random.default_rng(5).normal(size=(1, 64, 40)).astype(np.float32)).cuda()
        ga = W.wect_backward(W.SimplicialBatch.from_host([K]), W.Grid(dirs, thr), G)
        gb = W.wect_backward(W.SimplicialBatch.from_host([K2]), W.Grid(dirs, thr), G)
        torch.cuda.synchronize()
        assert np.array_equal(ga[0].cpu().numpy(), gb[0].cpu().numpy())
        for dim in range(1, 4):
            x, y = ga[dim].cpu().numpy(), gb[dim].cpu().numpy()
            assert np.array_equal(x[perms[dim]], y), dim
