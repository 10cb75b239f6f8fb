"""The library's host list builder (row runs, one-step intervalization) on
large polygons like the skewed workload's (20k-100k vertices), whose cell
windows are too large for the oracle to classify whole.  Cells are sampled
and each is classified by the oracle's brute-force rule over all edges:
uniform cells of the polygon's window, and the cells around random points on
its edges, where a boundary mistake would show.  A cell must be in the
library's A-list iff the oracle calls it Partial or Full, and in its F-list
iff Full.  The per-cell oracle is first checked against the oracle's
whole-window classification on small polygons.
"""

import numpy as np

import oracle
import synth
from paper_2307_01716_amd import april
from synth.grid import Grid, grid_covering
from synth.polygons import LATTICE

EMPTY, PARTIAL, FULL = 0, 1, 2


def test_classify_cells_equals_window_classification():
    R, _, g = synth.configs.tiny()
    for k in range(0, len(R), 25):
        whole = oracle.classify(g, R.polygon(k))
        got = oracle.classify_cells(g, R.polygon(k), whole[:, :2])
        assert np.array_equal(got, whole[:, 2].astype(np.uint8)), k
    # a rectangle on grid lines: the ring of cells that only touch it is
    # Partial (closed cells), the cells inside are Full
    w = 1 << 20
    g6 = Grid(0.0, 0.0, float(w * 64) * LATTICE, 6)
    i0, j0, i1, j1 = 3, 5, 10, 9
    xy = np.array([[x * w * LATTICE, y * w * LATTICE] for x, y in ((i0, j0), (i1, j0), (i1, j1), (i0, j1))])
    whole = oracle.classify(g6, xy)
    got = oracle.classify_cells(g6, xy, whole[:, :2])
    assert np.array_equal(got, whole[:, 2].astype(np.uint8))
    assert (got == FULL).sum() == (i1 - i0) * (j1 - j0)
    assert (got != EMPTY).sum() == (i1 - i0 + 2) * (j1 - j0 + 2)


def _member(d, s, e):
    """Is each id in d inside one of the sorted, disjoint intervals [s, e)?"""
    t = np.searchsorted(s, d, side="right").astype(np.int64) - 1
    return (t >= 0) & (d < e[np.maximum(t, 0)])


def test_builder_on_sampled_cells_of_large_polygons():
    rng = np.random.default_rng(3003)
    L = synth.configs.large_collection(rng, 2, 3)
    g = grid_covering([L], 16)
    offA, sA, eA, offF, sF, eF = april.april_build_lists(g, L.xy, L.voff, april.STRICT).export()
    w = g.side / (1 << g.order)
    seen = set()
    for k in range(len(L)):
        xy = L.polygon(k)
        assert len(xy) >= 20_000
        lo = np.floor((xy.min(axis=0) - (g.x0, g.y0)) / w).astype(np.int64) - 1
        hi = np.floor((xy.max(axis=0) - (g.x0, g.y0)) / w).astype(np.int64) + 1
        uni = np.stack([rng.integers(lo[0], hi[0] + 1, 4000), rng.integers(lo[1], hi[1] + 1, 4000)], 1)
        # cells at and around random points on random edges
        e = rng.integers(0, len(xy), 2000)
        f = rng.random(2000)[:, None]
        pts = xy[e] * (1 - f) + xy[(e + 1) % len(xy)] * f
        c = np.floor((pts - (g.x0, g.y0)) / w).astype(np.int64)
        near = np.concatenate([c + (di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)])
        ij = np.concatenate([uni, near])
        cls = oracle.classify_cells(g, xy, ij)
        d = oracle.hilbert(g.order, ij[:, 0], ij[:, 1]).astype(np.uint64)
        a0, a1, f0, f1 = int(offA[k]), int(offA[k + 1]), int(offF[k]), int(offF[k + 1])
        in_a = _member(d, sA[a0:a1].astype(np.uint64), eA[a0:a1].astype(np.uint64))
        in_f = _member(d, sF[f0:f1].astype(np.uint64), eF[f0:f1].astype(np.uint64))
        assert np.array_equal(in_a, cls != EMPTY), k
        assert np.array_equal(in_f, cls == FULL), k
        seen |= set(np.unique(cls).tolist())
    assert seen == {EMPTY, PARTIAL, FULL}
