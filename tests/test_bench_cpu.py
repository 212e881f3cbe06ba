"""Bench bookkeeping that needs no GPU: the count of staged vertices behind
the cubical roofline's frac_staged, against a brute-force count."""
import itertools

import numpy as np

import bench
import synth


def _brute_staged(C):
    """Included vertices with a nonzero combined weight in some orthant: for
    each sign pattern, the signed weights of the cells whose top corner is the
    vertex (cells extend towards +k where the pattern's bit k is set)."""
    I = C.intensity.astype(np.int64)
    P = I > C.include_above
    n = I.ndim
    count = 0
    for idx in zip(*np.nonzero(P)):
        nonzero = False
        for o in range(1 << n):
            dirs = [1 if (o >> k) & 1 else -1 for k in range(n)]
            acc = 0
            for S in itertools.product((0, 1), repeat=n):
                ok, mx = True, 0
                for c in itertools.product(*[(0, 1) if S[k] else (0,) for k in range(n)]):
                    pos = list(idx)
                    for k in range(n):
                        pos[n - 1 - k] += c[k] * dirs[k]  # axis k is numpy axis n - 1 - k
                    if any(q < 0 or q >= I.shape[a] for a, q in enumerate(pos)) or not P[tuple(pos)]:
                        ok = False
                        break
                    mx = max(mx, int(I[tuple(pos)]))
                if ok:
                    acc += (mx if C.weighted else 1) * (-1) ** sum(S)
            nonzero |= acc != 0
        count += nonzero
    return count


def test_staged_vertices_brute_force():
    for seed in range(4):
        for shape in ((7, 5), (6, 4, 5)):
            C = synth.random_tiny_cubical(seed, shape, include_above=60 + 10 * seed)
            for weighted in (True, False):
                Cw = synth.Cubical(C.intensity, C.axes, C.include_above, weighted)
                assert bench.staged_vertices(Cw, "cpu") == _brute_staged(Cw), (seed, shape, weighted)


def test_staged_vertices_special_cases():
    # a solid unweighted image: only the corners of the square have a nonzero
    # combined weight (interior and edge vertices cancel in every orthant)
    solid = synth.solid_image(6, 5, value=200)
    solid = synth.Cubical(solid.intensity, solid.axes, solid.include_above, False)
    assert bench.staged_vertices(solid, "cpu") == _brute_staged(solid) == 4
    # no vertex at all
    empty = synth.Cubical(np.zeros((4, 3), np.uint8), [synth.cubical_axis(3), synth.cubical_axis(4)], 10, True)
    assert bench.staged_vertices(empty, "cpu") == 0
