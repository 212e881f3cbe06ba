"""The device builder of weighted Freudenthal complexes from images: its arrays
equal the seeded generator's layout, and the WECT of the built batch matches the
oracle on the same complexes."""
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


SHAPES = ((9, 7), (1, 5), (6, 1), (1, 1), (33, 20), (2, 2))


def _images():
    return [synth.random_tiny_cubical(s, shp, include_above=-1, weighted=True) for s, shp in enumerate(SHAPES)]


def _host_complex(C):
    """The same weighted Freudenthal complex built on the host from the seeded generator."""
    n0, n1 = C.intensity.shape[1], C.intensity.shape[0]
    with np.errstate(divide="ignore", invalid="ignore"):  # its own coordinates divide by n - 1; not used
        _, edges, tris = synth.freudenthal_grid(n0, n1, 0.0, None)
    ax0, ax1 = (np.asarray(a, np.float32) for a in C.axes)
    coords = np.stack(np.meshgrid(ax0, ax1), axis=-1).reshape(-1, 2).astype(np.float32)
    w = np.asarray(C.intensity, np.float32).ravel()
    return synth.Simplicial(coords, [None, edges, tris], "vertex_max", [w])


def test_arrays_match_the_generator_layout(W):
    ims = _images()
    _say("Freudenthal builder, 6 images")
    sb = W.freudenthal_from_images(W.CubicalBatch.from_host(ims))
    torch.cuda.synchronize()
    vo, eo, to = (t.cpu().numpy() for t in (sb.vert_off, sb.simp_off[1], sb.simp_off[2]))
    coords, vw = sb.coords.cpu().numpy(), sb.weights[0].cpu().numpy()
    edges, tris = sb.simplices[1].cpu().numpy(), sb.simplices[2].cpu().numpy()
    for b, C in enumerate(ims):
        K = _host_complex(C)
        assert np.array_equal(coords[vo[b]:vo[b + 1]], K.coords)
        assert np.array_equal(vw[vo[b]:vo[b + 1]], K.weights[0])
        assert np.array_equal(edges[eo[b]:eo[b + 1]], K.simplices[1]), b
        assert np.array_equal(tris[to[b]:to[b + 1]], K.simplices[2]), b


def test_wect_of_built_complexes(W):
    ims = _images()
    dirs, thr = synth.s1_directions(40), synth.uniform_thresholds(23, 1.5)
    _say("WECT of built Freudenthal complexes")
    sb = W.freudenthal_from_images(W.CubicalBatch.from_host(ims))
    out = W.wect_forward(sb, W.Grid(dirs, thr)).cpu().numpy()
    ones = W.wect_forward(W.SimplicialBatch(sb.coords, sb.simplices, "ones", [], sb.vert_off, sb.simp_off, sb.B),
                          W.Grid(dirs, thr)).cpu().numpy()
    for b, C in enumerate(ims):
        K = _host_complex(C)
        ref = oracle.wect(K, dirs, thr)
        tol = 1e-5 * oracle.total_abs_weight(K)
        assert np.abs(out[b] - ref).max() <= tol, b
        # unweighted: a triangulated rectangle is contractible
        assert np.all(ones[b][:, -1] == 1), b
