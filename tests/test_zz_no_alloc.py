"""wect_forward_noalloc (workspace in a static device array) against
wect_forward with a caller's workspace, through the C ABI: the same plan and
kernels, so integer and 64-bit fixed-point results must be identical.  Two
calls in a row on the same array, the second with a smaller input; a request
whose workspace exceeds the array is refused before anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest

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


def _noalloc(W, cx, grid, out):
    from paper_2511_03909_amd import _lib as L
    c, g = cx.struct(), grid.struct()
    return L.lib().wect_forward_noalloc(ctypes.byref(c), ctypes.byref(g), out.data_ptr(),
                                        torch.cuda.current_stream().cuda_stream)


def _both(W, cx, grid):
    ref = W.wect_forward(cx, grid).clone()
    out = torch.full_like(ref, -7)
    st = _noalloc(W, cx, grid, out)
    torch.cuda.synchronize()
    assert st == 0, st
    return out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("decomposition", [0, 1])
def test_noalloc_matches_forward_two_calls(W, decomposition):
    """Float32 weights (partial histograms, their sums and the max-|w| area in
    the scratch array) and integer cubical images, each twice: a larger input,
    then a smaller one that reuses the array."""
    try:
        W.set_launch(decomposition=decomposition)
        for n, side in ((10, 8), (6, 5)):
            _say(f"noalloc float simplicial kuhn{n} decomposition={decomposition}")
            K = synth.cfg3(n=n).complexes[0]
            cx = W.SimplicialBatch.from_host([K])
            grid = W.Grid(synth.fibonacci_directions(130), synth.uniform_thresholds(77, 1.8))
            got, ref = _both(W, cx, grid)
            assert np.array_equal(got, ref)
        for nim, side in ((12, 40), (3, 17)):
            _say(f"noalloc cubical {nim}x{side}^2 decomposition={decomposition}")
            w = synth.cfg2(n_images=nim, side=side)
            cx = W.CubicalBatch.from_host(w.complexes)
            got, ref = _both(W, cx, W.Grid(w.dirs, w.thr))
            assert np.array_equal(got, ref)
    finally:
        W.set_launch()


def test_noalloc_refuses_a_workspace_above_the_array(W):
    """1024 blocks of partial 64-bit histograms at 256 thresholds need about
    135 MB: refused with WECT_ERR_WORKSPACE, the output untouched; the same
    request then runs with a caller's workspace."""
    from paper_2511_03909_amd import _lib as L
    K = synth.cfg3(n=12).complexes[0]
    cx = W.SimplicialBatch.from_host([K])
    grid = W.Grid(synth.fibonacci_directions(64), synth.uniform_thresholds(256, 1.8))
    try:
        W.set_launch(256, 4, 1, 1)
        assert W.wect_workspace_bytes(cx, grid) > 64 << 20
        out = torch.full((1, 64, 256), -3.0, device="cuda")
        st = _noalloc(W, cx, grid, out)
        torch.cuda.synchronize()
        assert st == L.WECT_ERR_WORKSPACE
        assert "static scratch" in L.lib().wect_last_error().decode()
        assert bool((out == -3.0).all())
    finally:
        W.set_launch()
