"""Parity of the adjoint (gradient with respect to the weights) with the CPU oracle.

The forward is linear in the cell weights, so the gradient of
L = sum grad_out * out with respect to w(c) is (-1)^dim(c) times the reverse
cumulative sum of grad_out along the thresholds, read at c's threshold index
and summed over the directions (the transpose of Algorithm 1's map; the paper
names differentiable transforms as future work in Section "Discussion").

Bound per entry: 1e-5 * (the same gradient with |grad_out|) + 1e-6, with the
oracle in float64.  Cases cover the explicit-weight gradient (one write per
simplex when all direction tiles fit in one pass, atomic accumulation over
direction groups otherwise), and the vertex-max gradient on the largest
complex of the differentiation batch."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _check(got, ref, bound, what):
    err = np.abs(np.asarray(got, np.float64) - ref)
    lim = 1e-5 * bound + 1e-6
    bad = np.argwhere(err > lim)
    assert bad.size == 0, f"{what}: {len(bad)} entries over the bound, worst {float((err - lim).max())}"


def _sub_complex(K, rows):
    """The same vertices with only the given simplex rows of each dimension
    (the gradient of a simplex depends on its own vertices only)."""
    simp = [None] + [K.simplices[d][rows[d]] for d in range(1, K.top_dim + 1)]
    ws = [K.weights[0]] + [K.weights[d][rows[d]] for d in range(1, K.top_dim + 1)]
    return synth.Simplicial(K.coords, simp, "explicit", ws)


def test_explicit_adjoint_3d_kuhn_full_size(W):
    """The 3D Kuhn mesh at full size (64^3 vertices, 6.6M simplices), 256
    directions, T = 256, float32 weights: four direction tiles that do not fit
    the adjoint's LDS together, so the gradient accumulates over direction
    groups with atomics.  Every vertex and 20,000 sampled rows of each other
    dimension are compared with the oracle."""
    w = synth.cfg3()
    K = w.complexes[0]
    g = synth.rng(60, 0, 0).normal(size=(1, w.dirs.shape[0], w.thr.shape[0])).astype(np.float32)
    _say("adjoint 3d kuhn64 explicit d=256 T=256")
    cx = W.SimplicialBatch.from_host([K])
    gw = W.wect_backward(cx, W.Grid(w.dirs, w.thr), torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    gw = [t.cpu().numpy() for t in gw]
    pick = synth.rng(60, 0, 1)
    rows = [None] + [np.sort(pick.choice(K.simplices[d].shape[0], 20000, replace=False))
                     for d in range(1, 4)]
    Ks = _sub_complex(K, rows)
    _say("adjoint 3d kuhn64: oracle on the sampled rows")
    ref = oracle.wect_backward(Ks, w.dirs, w.thr, g[0])
    bound = oracle.wect_backward(Ks, w.dirs, w.thr, g[0], absolute=True)
    _check(gw[0], ref[0], bound[0], "vertices")
    for d in range(1, 4):
        _check(gw[d][rows[d]], ref[d], bound[d], f"dimension {d}")


@pytest.mark.parametrize("d,T", [(300, 37), (64, 29), (130, 300)])
def test_explicit_adjoint_tiny_all_rows(W, d, T):
    """Tiny random complexes of dimension 1-3, every row compared: d = 300
    (five direction tiles, two direction groups, atomic accumulation), d = 64
    (one tile, one write per simplex), d = 130 at T = 300."""
    for seed, n, top in ((0, 1, 1), (1, 2, 2), (2, 3, 3)):
        K = synth.random_tiny_complex(seed, n=n, nv=12, top_dim=top, wmode="explicit", wdtype=np.float32)
        dirs = (synth.fibonacci_directions(d) if n == 3 else synth.s1_directions(d) if n == 2
                else np.linspace(-2, 2, d).astype(np.float32).reshape(d, 1))
        thr = synth.uniform_thresholds(T, 1.8)
        g = synth.rng(61, seed, d).normal(size=(1, d, T)).astype(np.float32)
        _say(f"adjoint tiny explicit seed={seed} n={n} d={d} T={T}")
        gw = W.wect_backward(W.SimplicialBatch.from_host([K]), W.Grid(dirs, thr), torch.from_numpy(g).cuda())
        torch.cuda.synchronize()
        ref = oracle.wect_backward(K, dirs, thr, g[0])
        bound = oracle.wect_backward(K, dirs, thr, g[0], absolute=True)
        for dim in range(top + 1):
            _check(gw[dim].cpu().numpy(), ref[dim], bound[dim], f"seed {seed} dimension {dim}")


def test_explicit_adjoint_finite_differences(W):
    """The loss <g, WECT(w)> is linear in the explicit weights, so float64
    central differences of the oracle's forward equal the gradient up to
    rounding; the GPU adjoint (two direction groups) matches them."""
    K = synth.random_tiny_complex(4, n=2, nv=12, top_dim=2, wmode="explicit", wdtype=np.float32)
    d, T = 260, 41
    dirs, thr = synth.s1_directions(d), synth.uniform_thresholds(T, 1.7)
    g = synth.rng(62, 0, 0).normal(size=(d, T))
    gw = W.wect_backward(W.SimplicialBatch.from_host([K]), W.Grid(dirs, thr),
                         torch.from_numpy(g[None].astype(np.float32)).cuda())
    torch.cuda.synchronize()
    g32 = g.astype(np.float32).astype(np.float64)
    bound = oracle.wect_backward(K, dirs, thr, g32, absolute=True)
    eps = 1e-3
    w64 = [np.asarray(x, np.float64) for x in K.weights]
    for dim in range(3):
        for r in range(0, K.counts()[dim], max(1, K.counts()[dim] // 4)):
            lv = []
            for s in (1.0, -1.0):
                ws = [x.copy() for x in w64]
                ws[dim][r] += s * eps
                Kp = synth.Simplicial(K.coords, K.simplices, "explicit", ws)
                lv.append(float((g32 * oracle.wect(Kp, dirs, thr)).sum()))
            fd = (lv[0] - lv[1]) / (2 * eps)
            got = float(gw[dim].cpu().numpy()[r])
            assert abs(got - fd) <= 1e-5 * bound[dim][r] + 1e-6, (dim, r, got, fd)


def test_vertex_max_adjoint_largest_complex(W):
    """The differentiation batch (64 complexes, 10k-200k vertices, d = 128,
    T = 128): the vertex-weight gradient of its largest complex, from one
    batched adjoint call, against the oracle."""
    w = synth.cfg5()
    Ks = w.complexes
    sizes = [K.coords.shape[0] for K in Ks]
    b = int(np.argmax(sizes))
    cx = W.SimplicialBatch.from_host(Ks)
    g = synth.rng(63, 0, 0).normal(size=(len(Ks), w.dirs.shape[0], w.thr.shape[0])).astype(np.float32)
    _say(f"adjoint differentiation batch, complex {b} with V={sizes[b]}")
    gv = W.wect_backward(cx, W.Grid(w.dirs, w.thr), torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    voff = np.concatenate([[0], np.cumsum(sizes)])
    mine = gv.cpu().numpy()[voff[b]:voff[b + 1]]
    ref = oracle.wect_backward(Ks[b], w.dirs, w.thr, g[b])
    bound = oracle.wect_backward(Ks[b], w.dirs, w.thr, g[b], absolute=True)
    _check(mine, ref, bound, f"complex {b}")
