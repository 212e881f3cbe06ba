"""Pins of the float64 oracle of the sigmoid relaxation (CPU only)."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import smooth as osm

HERE = os.path.dirname(__file__)


@pytest.fixture(scope="module")
def gold():
    with open(os.path.join(HERE, "golden", "smooth_examples.json")) as f:
        return json.load(f)


def _triangle(gold, weights=None):
    t = gold["triangle_unweighted"]
    coords = np.array(t["coords"], np.float32)
    simp = [None, np.array(t["edges"], np.int32), np.array(t["triangles"], np.int32)]
    if weights is None:
        return synth.Simplicial(coords, simp, "ones", [])
    w = [np.array(weights[k], np.float32) for k in ("vertices", "edges", "triangles")]
    return synth.Simplicial(coords, simp, "explicit", w)


def test_hand_triangle_values(gold):
    K = _triangle(gold)
    S = osm.smooth_wect(K, np.array(gold["directions"], np.float32), np.array(gold["thresholds"], np.float32),
                        gold["lam"])
    np.testing.assert_allclose(S, np.array(gold["triangle_unweighted"]["S"]), rtol=0, atol=1e-15)
    Kw = _triangle(gold, gold["triangle_weighted"]["weights"])
    Sw = osm.smooth_wect(Kw, np.array([[1, 0]], np.float32), np.array([0.0], np.float32), gold["lam"])
    assert abs(Sw[0, 0] - gold["triangle_weighted"]["S_dir0_t0"]) < 1e-14


def test_hand_triangle_gradients(gold):
    gr = gold["gradient"]
    K = _triangle(gold, {"vertices": [1, 1, 1], "edges": [1, 1, 1], "triangles": [1]})
    dirs = np.array([gr["direction"]], np.float32)
    res = osm.smooth_wect_vjp(K, dirs, np.array([0.0], np.float32), gold["lam"], np.array([[gr["g_at_t0"]]]))
    for dim, key in enumerate(("vertices", "edges", "triangles")):
        np.testing.assert_allclose(res["weights"][dim], gr["d_weights"][key], rtol=0, atol=1e-15)
    np.testing.assert_allclose(res["coords"], np.array(gr["d_coords"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(res["dirs"][0], np.array(gr["d_direction"]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed,wmode", [(0, "ones"), (1, "explicit"), (2, "vertex_max"), (3, "explicit")])
def test_lambda_zero_is_half_the_euler_characteristic(seed, wmode):
    K = synth.random_tiny_complex(seed, n=3, nv=9, top_dim=3, wmode=wmode, wdtype=np.float32)
    dirs = synth.fibonacci_directions(5)
    thr = np.linspace(-2, 2, 7).astype(np.float32)
    S = osm.smooth_wect(K, dirs, thr, 0.0)
    chi = float(oracle.euler_characteristic(K))
    np.testing.assert_allclose(S, np.full_like(S, 0.5 * chi), rtol=0, atol=1e-12 * (1 + oracle.total_abs_weight(K)))


@pytest.mark.parametrize("seed,wmode", [(4, "ones"), (5, "explicit"), (6, "vertex_max")])
def test_large_lambda_is_the_step_wect(seed, wmode):
    """Away from the cell values the sigmoid tends to the step: with every
    threshold at least 1e-3 from every height and lam = 1e5, each term differs
    from the step by less than exp(-100)."""
    K = synth.random_tiny_complex(seed, n=2, nv=10, top_dim=2, wmode=wmode, wdtype=np.float32)
    dirs = synth.s1_directions(6)
    h = oracle.heights(K.coords, dirs).astype(np.float64).ravel()
    cand = np.linspace(-1.6, 1.6, 41)
    thr = np.array([t for t in cand if np.min(np.abs(h - t)) >= 1e-3], np.float32)
    assert thr.size >= 10
    S = osm.smooth_wect(K, dirs, thr, 1e5)
    ref = oracle.wect(K, dirs, thr).astype(np.float64)
    np.testing.assert_allclose(S, ref, rtol=0, atol=1e-12 * (1 + oracle.total_abs_weight(K)))


def _generic(seed, wmode, n=2, top=2):
    """A random tiny complex with fresh uniform coordinates (no equal heights)."""
    K = synth.random_tiny_complex(seed, n=n, nv=9, top_dim=top, wmode=wmode, wdtype=np.float32)
    g = np.random.default_rng(1000 + seed)
    K.coords = g.uniform(-1, 1, size=K.coords.shape).astype(np.float32)
    return K


@pytest.mark.parametrize("seed,wmode,n,top", [(10, "explicit", 2, 2), (11, "vertex_max", 3, 3), (12, "ones", 3, 2)])
def test_gradients_match_finite_differences(seed, wmode, n, top):
    K = _generic(seed, wmode, n, top)
    dirs = synth.fibonacci_directions(4) if n == 3 else synth.s1_directions(4)
    thr = np.linspace(-1.5, 1.5, 9).astype(np.float32)
    lam = 3.0
    g = np.random.default_rng(seed).normal(size=(dirs.shape[0], thr.size))
    res = osm.smooth_wect_vjp(K, dirs, thr, lam, g)
    V = K.coords.shape[0]
    for v in range(V):
        for k in range(n):
            fd = osm.fd_smooth(K, dirs, thr, lam, g, "coords", (v, k))
            assert abs(fd - res["coords"][v, k]) <= 1e-5 * (1 + abs(fd)), (v, k, fd, res["coords"][v, k])
    for p in range(dirs.shape[0]):
        for k in range(n):
            fd = osm.fd_smooth(K, dirs, thr, lam, g, "dirs", (p, k))
            assert abs(fd - res["dirs"][p, k]) <= 1e-5 * (1 + abs(fd)), (p, k, fd, res["dirs"][p, k])
    if wmode == "vertex_max":
        for v in range(V):
            fd = osm.fd_smooth(K, dirs, thr, lam, g, "vweight", v)
            assert abs(fd - res["weights"][v]) <= 1e-6 * (1 + abs(fd))
    elif wmode == "explicit":
        for dim in range(top + 1):
            for r in range(min(4, K.counts()[dim])):
                fd = osm.fd_smooth(K, dirs, thr, lam, g, ("weight", dim), r)
                assert abs(fd - res["weights"][dim][r]) <= 1e-6 * (1 + abs(fd))
    else:
        assert res["weights"] is None


def test_translation_shifts_the_thresholds():
    """Moving every vertex by u moves every height along s by <u, s>: with
    dyadic coordinates, directions and shifts all float32 sums are exact."""
    K = synth.random_tiny_complex(7, n=2, nv=8, top_dim=2, wmode="explicit", wdtype=np.float32)
    g = np.random.default_rng(7)
    K.coords = (g.integers(-16, 17, size=K.coords.shape) / 16).astype(np.float32)
    dirs = np.array([[1, 0], [0, 1], [0.5, -0.75]], np.float32)
    u = np.array([0.25, -0.5], np.float32)
    thr = (np.arange(-20, 21) / 8).astype(np.float32)
    K2 = synth.Simplicial(K.coords + u, K.simplices, K.wmode, K.weights)
    for p in range(3):
        shift = float(dirs[p] @ u)
        a = osm.smooth_wect(K2, dirs[p:p + 1], thr, 2.5)
        b = osm.smooth_wect(K, dirs[p:p + 1], (thr - shift).astype(np.float32), 2.5)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)
