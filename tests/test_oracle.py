"""Pins for the CPU oracle (no GPU): every check here compares the oracle with
something other than itself -- hand-derived values, closed forms, invariants,
brute force, finite differences -- so that a dropped term, a wrong sign, a
wrong comparison or a transposed operand fails at least one of them."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# primitive semantics (Appendix "Examples of Tensor Operations")
# ---------------------------------------------------------------------------

def test_appendix_tensor_primitives():
    """The library primitives the oracle is built from (cumulative sum, max
    over an axis, gather, scatter-add) against the appendix's worked values:
    a check of the building blocks' semantics, not of the oracle itself."""
    g = _gold("appendix_tensor_ops.json")
    T = np.array(g["T"])
    U = np.array(g["U"])
    V = np.array(g["V"])
    assert np.array_equal(np.cumsum(T, axis=1), g["cumsum_T"])
    assert np.array_equal(T.max(axis=1), g["rmax_T_axis1"])
    assert np.array_equal(T[U], g["T_index_U"])
    S = T.T.copy()
    assert np.array_equal(S, g["S_equals_T_transpose"])
    # scatter-add: D[i, j] = sum_k [U[i,k] == j] V[k]
    for i in range(U.shape[0]):
        for k in range(U.shape[1]):
            np.add.at(S[i], U[i, k], V[k])
    assert np.array_equal(S, g["scatter_add_U_V_into_S"])


# ---------------------------------------------------------------------------
# height arithmetic
# ---------------------------------------------------------------------------

def test_rounding_order_pins():
    for case in _gold("rounding_order.json")["cases"]:
        coords = np.array([case["coord"]], dtype=np.float32)
        K = synth.Simplicial(coords, [None], "ones", [])
        dirs = np.array([case["dir"]], dtype=np.float32)
        thr = np.array([case["threshold"]], dtype=np.float32)
        out = oracle.wect(K, dirs, thr)
        assert out[0, 0] == case["expected_count"], case["name"]
        assert oracle.wect_bruteforce(K, dirs, thr)[0, 0] == case["expected_count"]
        # the case is sensitive: exact (double) evaluation lands above the threshold
        exact = float(np.dot(coords[0].astype(np.float64), dirs[0].astype(np.float64)))
        assert exact > case["threshold"]


# ---------------------------------------------------------------------------
# hand examples
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def hand():
    return _gold("hand_examples.json")


def _hand_grid(hand):
    return synth.hand_directions(), np.array(hand["thresholds"], dtype=np.float32)


def test_hand_triangle_unweighted(hand):
    dirs, thr = _hand_grid(hand)
    K = synth.single_triangle(weighted=False)
    exp = np.array(hand["triangle"]["unweighted"])
    assert np.array_equal(oracle.wect(K, dirs, thr), exp)
    assert np.array_equal(oracle.wect_bruteforce(K, dirs, thr), exp)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_hand_triangle_weighted(hand, dtype):
    dirs, thr = _hand_grid(hand)
    K = synth.single_triangle(weighted=True, dtype=np.float32)
    exp = np.array(hand["triangle"]["weighted"])
    assert np.allclose(oracle.wect(K, dirs, thr), exp, rtol=0, atol=1e-12)
    assert np.allclose(oracle.wect_bruteforce(K, dirs, thr), exp, rtol=0, atol=1e-12)


def test_hand_square(hand):
    dirs, thr = _hand_grid(hand)
    for weighted, key in ((True, "weighted"), (False, "unweighted")):
        C = synth.single_square(weighted=weighted)
        exp = np.array(hand["square"][key])
        assert np.array_equal(oracle.wect(C, dirs, thr), exp), key
        assert np.array_equal(oracle.wect_bruteforce(C, dirs, thr), exp), key
    assert oracle.euler_characteristic(synth.single_square(True)) == 10


def test_total_abs_weight_hand_values():
    """sum over all cells of |w(c)|, which sets every float32 tolerance, by hand:
    the weighted triangle 1+2+3 + 0.5+0.25+4 + 10; the unweighted one 3+3+1;
    signs do not count; vertex-max weights (1,2,3) give vertices 6, edges
    max(1,2)+max(1,3)+max(2,3) = 8, triangle 3; the square with intensities
    10,20,30,40 gives vertices 100, edges 20+40+30+40, square 40; with the
    pixel of intensity 10 excluded only the 3 vertices, the top and right
    edges (40 each) remain."""
    assert oracle.total_abs_weight(synth.single_triangle(True)) == 20.75
    assert oracle.total_abs_weight(synth.single_triangle(False)) == 7
    K = synth.single_triangle(True)
    neg = synth.Simplicial(K.coords, K.simplices, "explicit",
                           [np.array([-1, 2, -3], np.float32), np.array([0.5, -0.25, 4], np.float32),
                            np.array([-10], np.float32)])
    assert oracle.total_abs_weight(neg) == 20.75
    vm = synth.Simplicial(K.coords, K.simplices, "vertex_max", [np.array([1, 2, 3], np.float32)])
    assert oracle.total_abs_weight(vm) == 17
    assert oracle.total_abs_weight(synth.single_square(True)) == 270
    assert oracle.total_abs_weight(synth.single_square(False)) == 9
    cut = synth.single_square(True)
    cut = synth.Cubical(cut.intensity, cut.axes, include_above=15, weighted=True)
    assert oracle.total_abs_weight(cut) == 20 + 30 + 40 + 40 + 40


def test_hand_gradient(hand):
    dirs, thr = _hand_grid(hand)
    K = synth.single_triangle(weighted=True)
    gh = hand["triangle"]["gradient"]
    g = np.zeros((4, 6))
    for p, q, v in gh["grad_out_nonzero"]:
        g[p, q] = v
    got = oracle.wect_backward(K, dirs, thr, g)
    exp = gh["d_weights"]
    for dim, key in enumerate(("vertices", "edges", "triangles")):
        assert np.array_equal(got[dim], exp[key]), key
    bf = oracle.wect_backward_bruteforce(K, dirs, thr, g)
    for dim in range(3):
        assert np.array_equal(bf[dim], got[dim])
    out = oracle.wect(K, dirs, thr)
    assert float((g * out).sum()) == gh["inner_product"]
    wsum = sum(float((got[d] * K.weights[d].astype(np.float64)).sum()) for d in range(3))
    assert wsum == gh["inner_product"]
    for case in gh["vertex_max"]:
        Kv = synth.Simplicial(K.coords, K.simplices, "vertex_max", [np.array(case["w"], np.float32)])
        # the owner rule only redistributes the per-simplex gradients above
        assert np.array_equal(oracle.wect_backward(Kv, dirs, thr, g), case["d_w"]), case["note"]


# ---------------------------------------------------------------------------
# closed forms: Euler characteristic at the top threshold, 0 below the bottom
# ---------------------------------------------------------------------------

def _data_dependent_thresholds(X, dirs, T):
    """The paper's grid: M = max |f| over all directions and vertices, T evenly
    spaced values over [-M, M] (Section "Computation of WECFs"), with thr[T-1] = M
    stored exactly so that every cell is present at the last threshold."""
    cells = oracle.cells_of(X)
    M = np.float32(np.abs(oracle.heights(cells.coords, dirs)).max())
    thr = synth.uniform_thresholds(T, float(M))
    thr[-1] = M
    thr[0] = -M
    return thr


CLOSED_FORMS = [
    ("disk_freudenthal", lambda: synth.cfg1().complexes[0], 1, 2),
    ("ball_kuhn", lambda: synth.Simplicial(*(lambda c: (c[0], [None, c[1], c[2], c[3]]))(
        synth.kuhn_grid(5, 0.01, synth.rng(0, 0, 0))), "ones", []), 1, 3),
    ("octahedron_sphere", synth.octahedron, 2, 3),
    ("grid_torus", lambda: synth.grid_torus(7, 5), 0, 3),
    ("solid_image", lambda: synth.solid_image(7, 5), 1, 2),
    ("annulus_image", lambda: synth.annulus_image(9), 0, 2),
    ("hollow_shell", lambda: synth.hollow_shell(6), 2, 3),
]


@pytest.mark.parametrize("name,make,chi,n", CLOSED_FORMS, ids=[c[0] for c in CLOSED_FORMS])
def test_euler_characteristic_closed_forms(name, make, chi, n):
    X = make()
    assert oracle.euler_characteristic(X) == chi
    dirs = synth.s1_directions(12) if n == 2 else synth.fibonacci_directions(12)
    thr = _data_dependent_thresholds(X, dirs, 17)
    out = oracle.wect(X, dirs, thr)
    assert np.all(out[:, -1] == chi), name
    # below the smallest height the filtration is empty
    cells = oracle.cells_of(X)
    hmin = oracle.heights(cells.coords, dirs)
    if hasattr(X, "intensity"):
        inc = (np.asarray(X.intensity).T.ravel(order="F") > X.include_above)
        hmin = hmin[:, inc]
    hmin = hmin.min(axis=1)
    for p in range(dirs.shape[0]):
        below = thr < hmin[p]
        assert np.all(out[p, below] == 0)
    # and at least one threshold is below it in every direction for these grids
    assert np.all(thr[0] <= hmin)


def test_cfg1_overflow_rule():
    """With the fixed [-sqrt2, sqrt2] grid some jittered vertices lie above the
    last threshold: they are in no column, so out[p][T-1] + (signed weight of
    the cells above thr[T-1]) equals chi in every direction."""
    w = synth.cfg1()
    K = w.complexes[0]
    out = oracle.wect(K, w.dirs, w.thr)
    cells = oracle.cells_of(K)
    H = oracle.heights(cells.coords, w.dirs)
    over = np.zeros(w.dirs.shape[0], dtype=np.int64)
    n_above = 0
    for dim, v in enumerate(cells.verts):
        above = H[:, v].max(axis=2) > w.thr[-1]
        over += (above * cells.signed(dim)[None, :]).sum(axis=1)
        n_above += int(above.sum())
    assert np.all(out[:, -1] + over == 1)
    # some cells do lie above the last threshold on this workload (a corner's
    # upper star, whose signed mass happens to be 0)
    assert n_above > 0


# ---------------------------------------------------------------------------
# brute force on random tiny complexes
# ---------------------------------------------------------------------------

TINY = []
for seed in range(6):
    for n, top in ((1, 1), (2, 2), (3, 3)):
        for wmode, wdt in (("ones", np.int32), ("explicit", np.int32), ("explicit", np.float32),
                           ("vertex_max", np.float32)):
            TINY.append((seed, n, top, wmode, wdt))


@pytest.mark.parametrize("seed,n,top,wmode,wdt", TINY)
def test_bruteforce_tiny(seed, n, top, wmode, wdt):
    K = synth.random_tiny_complex(seed, n=n, nv=7 if top == 3 else 8, top_dim=top, wmode=wmode, wdtype=wdt)
    dirs = (synth.fibonacci_directions(5) if n == 3 else synth.s1_directions(5) if n == 2
            else np.array([[1.0], [-1.0], [0.5]], np.float32))
    thr = np.concatenate([synth.uniform_thresholds(9, 1.5), np.array([0.5], np.float32)])
    thr = np.sort(thr)
    a = oracle.wect(K, dirs, thr)
    b = oracle.wect_bruteforce(K, dirs, thr)
    if np.issubdtype(a.dtype, np.integer):
        assert np.array_equal(a, b)
    else:
        assert np.allclose(a, b, rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_bruteforce_tiny_cubical(seed):
    for shape in ((5, 4), (4, 3, 3)):
        for weighted in (True, False):
            C = synth.random_tiny_cubical(seed, shape, include_above=60, weighted=weighted)
            dirs = synth.s1_directions(6) if len(shape) == 2 else synth.fibonacci_directions(6)
            thr = synth.uniform_thresholds(7, 1.8)
            assert np.array_equal(oracle.wect(C, dirs, thr), oracle.wect_bruteforce(C, dirs, thr))


def test_backward_bruteforce_tiny():
    for seed in range(5):
        for n, top in ((2, 2), (3, 3)):
            K = synth.random_tiny_complex(seed, n=n, nv=7, top_dim=top, wmode="explicit", wdtype=np.float32)
            dirs = synth.fibonacci_directions(4) if n == 3 else synth.s1_directions(4)
            thr = synth.uniform_thresholds(6, 1.6)
            g = np.random.default_rng(seed).normal(size=(4, 6))
            a = oracle.wect_backward(K, dirs, thr, g)
            b = oracle.wect_backward_bruteforce(K, dirs, thr, g)
            for x, y in zip(a, b):
                assert np.allclose(x, y, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_linearity_in_weights():
    K1 = synth.random_tiny_complex(3, n=3, nv=9, top_dim=3, wmode="explicit", wdtype=np.int32)
    K2 = synth.random_tiny_complex(4, n=3, nv=9, top_dim=3, wmode="explicit", wdtype=np.int32)
    K2 = synth.Simplicial(K1.coords, K1.simplices, "explicit",
                          [np.resize(w, K1.weights[i].shape).astype(np.int32) for i, w in enumerate(K2.weights)])
    K12 = synth.Simplicial(K1.coords, K1.simplices, "explicit",
                           [(a * 3 - 2 * b).astype(np.int32) for a, b in zip(K1.weights, K2.weights)])
    dirs, thr = synth.fibonacci_directions(9), synth.uniform_thresholds(11, 2.0)
    assert np.array_equal(oracle.wect(K12, dirs, thr),
                          3 * oracle.wect(K1, dirs, thr) - 2 * oracle.wect(K2, dirs, thr))


def test_permutation_invariance():
    K = synth.random_tiny_complex(5, n=3, nv=10, top_dim=3, wmode="explicit", wdtype=np.int32)
    dirs, thr = synth.fibonacci_directions(8), synth.uniform_thresholds(13, 2.0)
    ref = oracle.wect(K, dirs, thr)
    g = np.random.default_rng(0)
    V = K.coords.shape[0]
    perm = g.permutation(V)           # new id of old vertex v is perm[v]
    inv = np.argsort(perm)
    coords = K.coords[inv]
    simp = [None]
    w = [K.weights[0][inv]]
    for i in range(1, len(K.simplices)):
        rows = g.permutation(K.simplices[i].shape[0])
        s = perm[K.simplices[i][rows]]
        s = np.array([g.permutation(r) for r in s], dtype=np.int32)
        simp.append(s)
        w.append(K.weights[i][rows])
    K2 = synth.Simplicial(coords, simp, "explicit", w)
    assert np.array_equal(oracle.wect(K2, dirs, thr), ref)


def test_adjoint_identity_exact():
    """<g, J w> = <J^T g, w>: the forward is linear in the weights and the
    backward is its transpose; exact with small integers."""
    for seed in range(4):
        K = synth.random_tiny_complex(seed, n=2, nv=9, top_dim=2, wmode="explicit", wdtype=np.int32)
        dirs, thr = synth.s1_directions(7), synth.uniform_thresholds(10, 1.6)
        g = np.random.default_rng(seed).integers(-4, 5, size=(7, 10)).astype(np.float64)
        out = oracle.wect(K, dirs, thr)
        gw = oracle.wect_backward(K, dirs, thr, g)
        lhs = float((g * out).sum())
        rhs = sum(float((gw[d] * K.weights[d]).sum()) for d in range(len(gw)))
        assert lhs == rhs


def test_duplicates_count_twice():
    K = synth.single_triangle(weighted=False)
    dirs, thr = synth.hand_directions(), synth.HAND_THRESHOLDS
    K2 = synth.Simplicial(K.coords, [None, np.concatenate([K.simplices[1], K.simplices[1][:1]]),
                                     K.simplices[2]], "ones", [])
    a = oracle.wect(K, dirs, thr)
    b = oracle.wect(K2, dirs, thr)
    # the duplicated edge (0,1) enters at max(h0, h1) and subtracts once more
    H = oracle.heights(K.coords, dirs)
    e = np.maximum(H[:, 0], H[:, 1])
    assert np.array_equal(a - b, (e[:, None] <= thr[None, :]).astype(np.int64))


# ---------------------------------------------------------------------------
# finite differences (float64) for vertex-max weights
# ---------------------------------------------------------------------------

def test_finite_differences_vertex_max():
    eps = 1e-3
    coords, edges, tris = synth.freudenthal_grid(9, 8, 0.155 * 2 / 8, synth.rng(5, 999, 0))
    w = synth.rng(5, 999, 1).normal(1.0, 0.2, size=coords.shape[0]).astype(np.float32)
    wt = synth.rng(5, 999, 4).normal(1.0, 0.2, size=coords.shape[0]).astype(np.float32)
    K = synth.Simplicial(coords, [None, edges, tris], "vertex_max", [w])
    Kt = synth.Simplicial(coords, [None, edges, tris], "vertex_max", [wt])
    dirs, thr = synth.s1_directions(16), synth.uniform_thresholds(16, math.sqrt(2))
    target = oracle.wect(Kt, dirs, thr)
    out = oracle.wect(K, dirs, thr)
    g = 2.0 * (out - target)
    gv = oracle.wect_backward(K, dirs, thr, g)
    # only vertices whose star has no other weight within 2 eps (no argmax switch inside +-eps)
    nbr = {v: set() for v in range(coords.shape[0])}
    for s in np.concatenate([edges, tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [0, 2]]]):
        nbr[int(s[0])].add(int(s[1]))
        nbr[int(s[1])].add(int(s[0]))
    ok = [v for v in range(coords.shape[0]) if all(abs(float(w[v]) - float(w[u])) > 2 * eps for u in nbr[v])]
    assert len(ok) > 0.9 * coords.shape[0]
    sample = ok[::5]
    fd = oracle.fd_vertex_grad(K, dirs, thr, target, sample, eps=eps)
    assert np.allclose(fd, gv[sample], rtol=1e-9, atol=1e-7)
    assert np.abs(gv[sample]).max() > 0


# ---------------------------------------------------------------------------
# generator sizes
# ---------------------------------------------------------------------------

def test_generator_counts():
    K = synth.cfg1().complexes[0]
    assert K.counts() == [1024, 2945, 1922]
    assert oracle.euler_characteristic(K) == 1
    c = synth.cfg3().complexes[0].counts()
    assert c == [262144, 1786239, 3024378, 1500282]
    assert c[0] - c[1] + c[2] - c[3] == 1
    T = synth.grid_torus(6, 5)
    assert T.counts() == [30, 90, 60]
    assert synth.octahedron().counts() == [6, 12, 8]


def test_cubical_views_match_explicit_cells():
    """The shifted-view evaluation of image/volume cells equals the explicit
    cell enumeration (which the brute force and the closed forms pin)."""
    for seed in range(4):
        for shape in ((6, 5), (5, 4, 3)):
            for weighted in (True, False):
                C = synth.random_tiny_cubical(seed, shape, include_above=70, weighted=weighted)
                dirs = synth.s1_directions(9) if len(shape) == 2 else synth.fibonacci_directions(9)
                thr = synth.uniform_thresholds(11, 1.8)
                a = oracle.wect(C, dirs, thr)
                b = oracle.wect(oracle.cubical_cells(C), dirs, thr)
                assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# general vertex filters and the ECF of an image
# ---------------------------------------------------------------------------

def _image(case):
    I = np.asarray(case["intensity"], dtype=np.uint8)
    axes = [synth.cubical_axis(s) for s in I.shape[::-1]]
    return synth.Cubical(I, axes, include_above=-1, weighted=case["weighted"])


def test_image_ecf_hand_examples():
    with open(os.path.join(GOLD, "image_ecf_examples.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        C = _image(case)
        thr = np.asarray(case["thr"], dtype=np.float32)
        assert oracle.image_ecf(C, thr).tolist() == case["ecf"], case["name"]
        assert oracle.image_ecf_cells(C, thr).tolist() == case["ecf"], case["name"]


@pytest.mark.parametrize("seed", range(8))
def test_image_ecf_views_equal_explicit_cells(seed):
    """Tie-heavy tiny images and volumes (intensities in 0..3), with and without
    an inclusion level and weights: the shifted-view route equals the explicit
    cell list."""
    g = np.random.default_rng(seed)
    shape = [(5, 4), (1, 7), (6, 6), (3, 4, 2), (2, 2, 5)][seed % 5]
    I = g.integers(0, 4, size=shape[::-1]).astype(np.uint8)
    C = synth.Cubical(I, [synth.cubical_axis(s) for s in shape], include_above=int(seed % 3) - 1,
                      weighted=bool(seed & 1))
    thr = np.array([-1, 0, 0.5, 1, 2, 2.5, 3, 4], dtype=np.float32)
    assert np.array_equal(oracle.image_ecf(C, thr), oracle.image_ecf_cells(C, thr))


def test_image_ecf_nan_threshold_admits_no_cell():
    C = synth.uniform_image((6, 5), 2)
    out = oracle.image_ecf(C, np.array([np.nan, 255.0], dtype=np.float32))
    assert out.tolist() == [0, 1]


def test_image_ecf_closed_forms():
    """Above the largest intensity the ECF is chi of the whole image (a solid
    rectangle or box: 1); below the smallest it is 0."""
    g = np.random.default_rng(5)
    for shape in ((7, 5), (4, 3, 6)):
        I = g.integers(0, 256, size=shape[::-1]).astype(np.uint8)
        C = synth.Cubical(I, [synth.cubical_axis(s) for s in shape], include_above=-1, weighted=False)
        out = oracle.image_ecf(C, np.array([-0.5, float(I.min()) - 0.5, 255.0], dtype=np.float32))
        assert out.tolist() == [0, 0, 1]


def test_wecf_of_heights_is_the_wect():
    """The WECT is the WECF with filter values V D^T."""
    K = synth.random_tiny_complex(4, n=3, nv=9, top_dim=3, wmode="explicit", wdtype=np.int32)
    dirs, thr = synth.fibonacci_directions(7), synth.uniform_thresholds(11, 1.8)
    F = oracle.heights(K.coords, dirs).T
    assert np.array_equal(oracle.wecf(K, F, thr), oracle.wect(K, dirs, thr))


@pytest.mark.parametrize("seed", range(6))
def test_wecf_matches_bruteforce(seed):
    """Arbitrary filters with many ties (values from a small set) and thresholds
    on filter values."""
    g = np.random.default_rng(100 + seed)
    wm = ["ones", "explicit", "vertex_max"][seed % 3]
    wdt = np.float32 if wm == "vertex_max" or seed % 2 else np.int32
    K = synth.random_tiny_complex(seed, n=2, nv=8, top_dim=2, wmode=wm, wdtype=wdt)
    F = g.choice(np.array([-1.0, -0.25, 0.0, 0.5, 0.75], np.float32), size=(8, 5))
    thr = np.array([-1.0, -0.5, 0.0, 0.5, 1.0], dtype=np.float32)
    got, ref = oracle.wecf(K, F, thr), oracle.wecf_bruteforce(K, F, thr)
    if np.issubdtype(ref.dtype, np.integer):
        assert np.array_equal(got, ref)
    else:
        assert np.allclose(got, ref, rtol=0, atol=1e-9)


def test_wecf_closed_forms():
    """chi at a threshold above every filter value (octahedron boundary: 2;
    Freudenthal torus: 0) and 0 below every filter value."""
    g = np.random.default_rng(7)
    for K, chi in ((synth.octahedron(), 2), (synth.grid_torus(5, 4), 0)):
        F = g.uniform(-1, 1, size=(K.coords.shape[0], 6)).astype(np.float32)
        out = oracle.wecf(K, F, np.array([-1.5, 1.5], dtype=np.float32))
        assert np.all(out[:, 0] == 0) and np.all(out[:, 1] == chi)


def test_wecf_backward_of_heights_is_the_wect_backward():
    """With the heights as filter values the WECF adjoint is the WECT adjoint
    (pinned by the hand examples and brute force above)."""
    for wmode in ("explicit", "vertex_max"):
        K = synth.random_tiny_complex(31, n=2, nv=10, top_dim=2, wmode=wmode, wdtype=np.float32)
        dirs = synth.s1_directions(5)
        thr = np.linspace(-1.5, 1.5, 13).astype(np.float32)
        g = np.random.default_rng(3).normal(size=(5, 13))
        F = oracle.heights(K.coords, dirs).T.copy()
        a = oracle.wect_backward(K, None, thr, g, fvals=F)
        b = oracle.wect_backward(K, dirs, thr, g)
        if wmode == "vertex_max":
            np.testing.assert_array_equal(a, b)
        else:
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)


def test_wecf_backward_adjoint_identity():
    """<g, J w> = <J^T g, w> for a general filter: the WECF is linear in the
    weights, so the forward of the oracle and its adjoint must agree."""
    K = synth.random_tiny_complex(32, n=2, nv=11, top_dim=2, wmode="explicit", wdtype=np.float32)
    g0 = np.random.default_rng(5)
    F = g0.normal(size=(11, 7)).astype(np.float32)
    thr = np.linspace(-2, 2, 9).astype(np.float32)
    g = g0.normal(size=(7, 9))
    out = oracle.wecf(K, F, thr)
    grads = oracle.wect_backward(K, None, thr, g, fvals=F)
    lhs = float((g * out).sum())
    rhs = sum(float(np.dot(gr, np.asarray(w, np.float64))) for gr, w in zip(grads, K.weights))
    assert abs(lhs - rhs) <= 1e-9 * (1 + abs(lhs))
