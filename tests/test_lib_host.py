"""Host-side checks of the HIP library (no GPU needed).

* libapril.so loads and exports every function include/april.h declares;
* the library's own list builder (one-step intervalization, Sec. 6.2) gives
  lists identical to the oracle's brute-force classification (Sec. 4.1), on
  the tiny workload, on grid-aligned shapes full of exact contacts, and on a
  sample of the at-scale workload;
* the library's MBR join gives the oracle's candidate pairs;
* argument and geometry errors come back as the documented codes.
"""

import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2307_01716_amd import april
from synth.grid import Grid
from synth.polygons import LATTICE, PolygonSet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "april.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(april_\w+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert "april_filter_pairs" in names and "april_build_lists" in names
    L = april.lib()
    for n in names:
        assert hasattr(L, n), n


def _same(L, O):
    got = L.export()
    exp = (O.offA, O.sA, O.eA, O.offF, O.sF, O.eF)
    return all(np.array_equal(a, b) for a, b in zip(got, exp))


def test_builder_matches_oracle_tiny():
    R, S, g = synth.configs.tiny()
    for P in (R, S):
        assert _same(april.april_build_lists(g, P.xy, P.voff, april.STRICT), oracle.build_lists(g, P))


@pytest.mark.parametrize("aligned", [False, True])
def test_builder_matches_oracle_edge_cases(aligned):
    from test_oracle_classify import G6, small_star_polys
    ps = small_star_polys(21 + aligned, 300, lattice_to_grid_points=aligned)
    assert _same(april.april_build_lists(G6, ps.xy, ps.voff, april.STRICT), oracle.build_lists(G6, ps))


def test_builder_matches_oracle_closed_forms():
    from test_oracle_classify import G6, world
    shapes = [world([(3, 5), (10, 5), (10, 9), (3, 9)]),
              world([(3.5, 5.5), (10.5, 5.5), (10.5, 9.5), (3.5, 9.5)]),
              world([(10, 10), (17, 10), (10, 17)]),
              world([(20.25, 20.25), (20.75, 20.25), (20.5, 20.75)])]
    voff = np.cumsum([0] + [len(s) for s in shapes]).astype(np.int64)
    ps = PolygonSet(np.concatenate(shapes), voff)
    assert _same(april.april_build_lists(G6, ps.xy, ps.voff, april.STRICT), oracle.build_lists(G6, ps))


def test_builder_matches_oracle_scale_sample():
    R, S, g = synth.configs.scale()
    sub = R.subset(np.arange(0, len(R), 97))
    assert _same(april.april_build_lists(g, sub.xy, sub.voff, april.STRICT), oracle.build_lists(g, sub))


def _by_rs(r, s):
    k = np.lexsort((s, r))
    return r[k], s[k]


def _check_grouping(r, s):
    # every r forms one contiguous run; s ascends within it
    starts = np.flatnonzero(np.diff(r.astype(np.int64)) != 0) + 1
    assert len(np.unique(r)) == len(starts) + 1
    same = r[1:] == r[:-1]
    assert np.all(s[1:][same] > s[:-1][same])


def test_mbr_join_matches_oracle():
    R, S, g = synth.configs.tiny()
    r, s = april.april_mbr_join(R.mbrs(), S.mbrs())
    ro, so = oracle.mbr_join(R, S)
    _check_grouping(r, s)
    r, s = _by_rs(r, s)
    assert np.array_equal(r, ro) and np.array_equal(s, so)


def test_mbr_join_matches_oracle_scale():
    R, S, g = synth.configs.scale()
    r, s = april.april_mbr_join(R.mbrs(), S.mbrs())
    ro, so = oracle.mbr_join(R, S)
    assert len(r) > 4_000_000
    _check_grouping(r, s)
    r, s = _by_rs(r, s)
    assert np.array_equal(r, ro) and np.array_equal(s, so)


def test_mbr_join_touching_boxes():
    a = np.array([[0.0, 0.0, 1.0, 1.0]])
    b = np.array([[1.0, 1.0, 2.0, 2.0], [1.0 + 2 ** -30, 0.0, 2.0, 1.0], [0.5, 1.0, 0.6, 3.0]])
    r, s = april.april_mbr_join(a, b)
    assert list(zip(r.tolist(), s.tolist())) == [(0, 0), (0, 2)]
    r, s = april.april_mbr_join(a, np.zeros((0, 4)))
    assert len(r) == 0


# ------------------------------------------------------------------ errors

G6 = Grid(0.0, 0.0, float((1 << 20) * 64) * LATTICE, 6)
U = (1 << 20) * LATTICE


def _poly(pts):
    xy = np.array(pts, dtype=np.float64) * U
    return xy, np.array([0, len(xy)], dtype=np.uint64)


def test_error_guard_ring():
    xy, vo = _poly([(0.5, 10), (5, 10), (5, 15)])
    with pytest.raises(april.AprilError) as e:
        april.april_build_lists(G6, xy, vo)
    assert e.value.code == april.E_GRID


def test_error_too_few_vertices():
    xy, vo = _poly([(5, 10), (6, 10)])
    with pytest.raises(april.AprilError) as e:
        april.april_build_lists(G6, xy, vo)
    assert e.value.code == april.E_INVALID


def test_error_non_lattice_strict():
    xy, vo = _poly([(5, 10), (9, 10), (9, 15)])
    xy[0, 0] += LATTICE / 3
    with pytest.raises(april.AprilError) as e:
        april.april_build_lists(G6, xy, vo, april.STRICT)
    assert e.value.code == april.E_INVALID
    # without STRICT the coordinate is rounded to the lattice
    L = april.april_build_lists(G6, xy, vo)
    assert L.info().n_a > 0


def test_error_inexact_grid():
    bad = Grid(0.0, 0.0, 1.0 + LATTICE, 6)
    xy, vo = _poly([(5, 10), (9, 10), (9, 15)])
    with pytest.raises(april.AprilError) as e:
        april.april_build_lists(bad, xy, vo)
    assert e.value.code == april.E_GRID


def test_error_corrupt_lists():
    off = np.array([0, 2], np.uint64)
    with pytest.raises(april.AprilError) as e:
        april.april_lists_from_arrays(G6, off, [5, 3], [6, 4], off, [5, 3], [6, 4])
    assert e.value.code == april.E_CORRUPT
    L = april.april_lists_from_arrays(G6, off, [3, 5], [4, 6], np.array([0, 0], np.uint64), [], [])
    assert L.info().n_a == 2 and L.info().n_f == 0
    # an F interval that leaves its A interval: not an APRIL approximation
    with pytest.raises(april.AprilError) as e:
        april.april_lists_from_arrays(G6, off, [3, 10], [6, 20], np.array([0, 1], np.uint64), [5], [7])
    assert e.value.code == april.E_CORRUPT
    L = april.april_lists_from_arrays(G6, off, [3, 10], [6, 20], np.array([0, 2], np.uint64), [3, 12],
                                      [5, 20])
    assert L.info().n_f == 2


def test_filter_rejects_host_lists():
    off = np.array([0, 1], np.uint64)
    L = april.april_lists_from_arrays(G6, off, [3], [4], off, [3], [4])
    with pytest.raises(april.AprilError) as e:
        april.april_filter_pairs(L, L, 0, 0, 0, None, stream=0)
    assert e.value.code == april.E_INVALID


def test_partitioned_build_and_pairs_match_oracle():
    from paper_2307_01716_amd import partitioned
    R, S, g = synth.configs.tiny(n=400)
    lay = synth.partitions.layout(R, S, 4, 10)
    hR = partitioned.build_instances(lay, R, "r")
    hS = partitioned.build_instances(lay, S, "s")
    # every instance's lists equal the oracle's on its partition's grid
    offA, sA, eA, offF, sF, eF = hR.export()
    part = lay.r_part()
    for p in range(16):
        a, b = int(lay.r_off[p]), int(lay.r_off[p + 1])
        if a == b:
            continue
        O = oracle.build_lists(lay.grids[p], R.subset(lay.r_obj[a:b]))
        assert np.array_equal(offA[a:b + 1] - offA[a], O.offA)
        assert np.array_equal(sA[offA[a]:offA[b]], O.sA)
        assert np.array_equal(eF[offF[a]:offF[b]], O.eF)
    assert np.all(part[:-1] <= part[1:])
    r, s = partitioned.pairs(lay, R, S)
    rg, sg = lay.r_obj[r], lay.s_obj[s]
    k = np.lexsort((sg, rg))
    ro, so = oracle.mbr_join(R, S)
    assert np.array_equal(rg[k], ro) and np.array_equal(sg[k], so)
    assert hR.info().n_objects == len(lay.r_obj)


def _one(P, k):
    a, b = int(P.voff[k]), int(P.voff[k + 1])
    return PolygonSet(np.ascontiguousarray(P.xy[a:b]), np.array([0, b - a], np.int64))


def test_parallel_builder_matches_oracle(monkeypatch):
    """A polygon built alone takes the multi-threaded path (forced here for
    every size); its lists equal the oracle's brute-force ones."""
    monkeypatch.setenv("APRIL_PAR_BUILD_CELLS", "1")
    R, _, g = synth.configs.tiny()
    from test_oracle_classify import G6, small_star_polys
    cases = [(g, R, k) for k in range(0, len(R), 37)]
    ps = small_star_polys(23, 40, lattice_to_grid_points=True)
    cases += [(G6, ps, k) for k in range(len(ps))]
    for grid, P, k in cases:
        one = _one(P, k)
        assert _same(april.april_build_lists(grid, one.xy, one.voff, april.STRICT), oracle.build_lists(grid, one)), k


def test_parallel_builder_large_polygon_equals_sequential():
    """A large jagged query polygon: built alone (split over threads) and
    inside a collection (one thread per polygon) the lists are identical."""
    S, Q, g = synth.configs.serving(n_s=1000, n_queries=400)
    mb = Q.mbrs()
    k = int(np.argmax((mb[:, 2] - mb[:, 0]) * np.diff(Q.voff)))
    alone = april.april_build_lists(g, _one(Q, k).xy, _one(Q, k).voff, 0)
    assert alone.info().n_a > 10_000
    many = Q.subset(np.r_[k, np.arange(64)])     # more polygons than threads
    both = april.april_build_lists(g, many.xy, many.voff, 0).export()
    got = alone.export()
    na, nf = int(both[0][1]), int(both[3][1])
    assert np.array_equal(got[1], both[1][:na]) and np.array_equal(got[2], both[2][:na])
    assert np.array_equal(got[4], both[4][:nf]) and np.array_equal(got[5], both[5][:nf])


def test_cells_builder_matches_oracle():
    """Linestring cell lists (Sec. 4.3.3): the library's host builder (exact
    edge traversal) equals the oracle's brute force, and rejects the same
    inputs."""
    from synth.polygons import LATTICE, PolygonSet
    P, L, g = synth.configs.linestring_scale(n_poly=300, n_lines=800)
    C = april.april_build_cells(g, L.xy, L.voff, april.STRICT)
    off, ids = C.export()
    O = oracle.build_cells(g, L)
    assert np.array_equal(off, O.off) and np.array_equal(ids, O.ids)
    assert C.info() == (len(L), len(O.ids))
    # a vertex in the outer ring; a single-vertex linestring
    bad = PolygonSet(np.array([[g.x0 + LATTICE, g.y0 + LATTICE], [g.x0 + 0.5, g.y0 + 0.5]]), np.array([0, 2]))
    with pytest.raises(april.AprilError) as e:
        april.april_build_cells(g, bad.xy, bad.voff, april.STRICT)
    assert e.value.code == april.E_GRID
    one = PolygonSet(L.xy[:1].copy(), np.array([0, 1]))
    with pytest.raises(april.AprilError) as e:
        april.april_build_cells(g, one.xy, one.voff, april.STRICT)
    assert e.value.code == april.E_INVALID
