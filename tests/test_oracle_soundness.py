"""Soundness of the oracle's verdicts against exact geometry, and pins of
the exact geometry and MBR join it relies on.

Sec. 4.2: a true negative means the polygons share no cell and cannot
intersect; a true hit means a Full cell of one meets a cell of the other, so
they do intersect.  On every candidate pair of the tiny workload the oracle's
TH pairs must intersect exactly and its TN pairs must not.
"""

import numpy as np
import pytest

import oracle
import synth
from synth.grid import Grid
from synth.polygons import LATTICE, PolygonSet

Q = LATTICE * 1024  # a coarse unit for hand-made shapes


def sq(x, y, s):
    return np.array([[x, y], [x + s, y], [x + s, y + s], [x, y + s]], dtype=np.float64) * Q


def test_exact_intersection_hand_cases():
    a = sq(0, 0, 10)
    assert oracle.polygons_intersect(a, sq(10, 0, 5))          # shared edge
    assert oracle.polygons_intersect(a, sq(10, 10, 5))         # shared corner
    assert not oracle.polygons_intersect(a, sq(11, 0, 5))      # gap of one unit
    assert oracle.polygons_intersect(a, sq(2, 2, 3))           # nested
    assert oracle.polygons_intersect(sq(2, 2, 3), a)           # nested, other way
    assert oracle.polygons_intersect(a, sq(5, -5, 10))         # crossing
    tri = np.array([[12, 0], [20, 0], [12, 8]], dtype=np.float64) * Q
    assert not oracle.polygons_intersect(a, tri)
    tri2 = np.array([[10, 5], [20, 0], [20, 10]], dtype=np.float64) * Q
    assert oracle.polygons_intersect(a, tri2)                   # vertex on edge
    # concave: a U shape and a square inside its notch without contact
    u = np.array([[0, 0], [30, 0], [30, 30], [20, 30], [20, 10], [10, 10], [10, 30], [0, 30]],
                 dtype=np.float64) * Q
    assert not oracle.polygons_intersect(u, sq(12, 12, 5))
    assert oracle.polygons_intersect(u, sq(12, 8, 5))


def test_twice_area():
    assert oracle.twice_area(sq(0, 0, 10)) == 2 * (10 * 1024) ** 2
    tri = np.array([[0, 0], [4, 0], [0, 3]], dtype=np.float64) * Q
    assert oracle.twice_area(tri) == 12 * 1024 ** 2


def test_mbr_join_matches_brute_force():
    R, S, g = synth.configs.tiny()
    r, s = oracle.mbr_join(R, S)
    a, b = R.mbrs(), S.mbrs()
    meet = ((a[:, None, 0] <= b[None, :, 2]) & (b[None, :, 0] <= a[:, None, 2]) &
            (a[:, None, 1] <= b[None, :, 3]) & (b[None, :, 1] <= a[:, None, 3]))
    rr, ss = np.nonzero(meet)
    assert np.array_equal(r, rr.astype(np.uint32))
    assert np.array_equal(s, ss.astype(np.uint32))
    assert len(r) > 1000


@pytest.fixture(scope="module")
def tiny_filtered():
    R, S, g = synth.configs.tiny()
    LR = oracle.build_lists(g, R)
    LS = oracle.build_lists(g, S)
    r, s = oracle.mbr_join(R, S)
    v = oracle.filter_pairs(LR, LS, r, s)
    return R, S, g, LR, LS, r, s, v


def test_verdicts_sound_on_tiny(tiny_filtered):
    R, S, g, LR, LS, r, s, v = tiny_filtered
    counts = np.bincount(v, minlength=3)
    assert counts.min() > 50              # all three outcomes occur
    for p in range(len(r)):
        inter = oracle.polygons_intersect(R.polygon(int(r[p])), S.polygon(int(s[p])))
        if v[p] == oracle.TH:
            assert inter, p
        elif v[p] == oracle.TN:
            assert not inter, p


def test_swapped_roles(tiny_filtered):
    R, S, g, LR, LS, r, s, v = tiny_filtered
    v2 = oracle.filter_pairs(LS, LR, s, r)
    assert np.array_equal(v, v2)


def test_self_pairs(tiny_filtered):
    R, S, g, LR, LS, r, s, v = tiny_filtered
    ids = np.arange(len(R), dtype=np.uint32)
    vs = oracle.filter_pairs(LR, LR, ids, ids)
    hasF = np.diff(LR.offF) > 0
    assert np.array_equal(vs, np.where(hasF, oracle.TH, oracle.IND).astype(np.uint8))


def test_touching_polygons_are_not_negative():
    # two squares sharing an edge on an off-grid line: exact contact only
    g = Grid(0.0, 0.0, float((1 << 20) * 64) * LATTICE, 6)
    u = (1 << 20) * LATTICE
    a = np.array([[10.3, 10.3], [20.7, 10.3], [20.7, 20.1], [10.3, 20.1]]) * u
    b = np.array([[20.7, 12.0], [30.2, 12.0], [30.2, 25.0], [20.7, 25.0]]) * u
    a = np.round(a / LATTICE) * LATTICE
    b = np.round(b / LATTICE) * LATTICE
    b[:, 0] = np.where(np.isclose(b[:, 0], a[1, 0]), a[1, 0], b[:, 0])
    assert oracle.polygons_intersect(a, b)
    LA = oracle.build_lists(g, PolygonSet(a, np.array([0, 4], dtype=np.int64)))
    LB = oracle.build_lists(g, PolygonSet(b, np.array([0, 4], dtype=np.int64)))
    v = oracle.filter_pairs(LA, LB, [0], [0])
    assert v[0] != oracle.TN


def _pip(poly, x, y):
    return oracle.point_in_closed_polygon(poly, x * Q, y * Q)


def test_point_in_closed_polygon_hand_cases():
    """Closed point-in-polygon: the boundary counts as inside (R2's closed
    sets).  Hand cases on a U shape (concave, with a notch) and a square."""
    a = sq(0, 0, 10)
    assert _pip(a, 5, 5)                 # inside
    assert not _pip(a, 11, 5)            # outside, right
    assert not _pip(a, -1, 5)            # outside, left
    assert _pip(a, 10, 5)                # on an edge
    assert _pip(a, 5, 0)                 # on the bottom edge
    assert _pip(a, 0, 0) and _pip(a, 10, 10)    # on vertices
    assert not _pip(a, 11, 0)            # on the bottom edge's extension
    assert not _pip(a, 10, 11)           # on the right edge's extension
    assert not _pip(a, 15, 10)           # level with the top edge, right of it
    u = np.array([[0, 0], [30, 0], [30, 30], [20, 30], [20, 10], [10, 10], [10, 30], [0, 30]],
                 dtype=np.float64) * Q
    assert not _pip(u, 15, 20)           # in the notch
    assert _pip(u, 15, 10)               # on the notch's floor
    assert _pip(u, 20, 20)               # on the notch's wall
    assert _pip(u, 5, 20) and _pip(u, 25, 20) and _pip(u, 15, 5)
    assert not _pip(u, 15, 30)           # between the prongs at their tops
    assert _pip(u, 10, 30) and _pip(u, 20, 30)   # prong corners
    assert not _pip(u, 35, 30)           # level with the prong tops, right
    assert not _pip(u, -5, 10)           # level with the notch floor, left
    # a ray through a vertex: the point's ray towards +x passes a vertex
    d = np.array([[10, 0], [20, 10], [10, 20], [0, 10]], dtype=np.float64) * Q
    assert _pip(d, 5, 10) and _pip(d, 15, 10) and not _pip(d, -5, 10) and not _pip(d, 25, 10)
    assert _pip(d, 0, 10) and _pip(d, 20, 10)    # the vertices on that line


def _inside_union_of_rects(rects, x, y):
    return any(x0 <= x <= x1 and y0 <= y <= y1 for x0, y0, x1, y1 in rects)


def test_point_in_closed_polygon_closed_forms():
    """Against closed forms on every lattice point of a window: a U shape is
    the union of three closed rectangles; a convex polygon (counter-
    clockwise) holds a point iff no edge has it strictly on its right."""
    u = [[0, 0], [30, 0], [30, 30], [20, 30], [20, 10], [10, 10], [10, 30], [0, 30]]
    rects = [(0, 0, 30, 10), (0, 0, 10, 30), (20, 0, 30, 30)]
    up = np.array(u, dtype=np.float64) * Q
    for x in range(-2, 33):
        for y in range(-2, 33):
            assert _pip(up, x, y) == _inside_union_of_rects(rects, x, y), (x, y)
    rng = np.random.default_rng(5)
    for _ in range(20):
        # a convex polygon: the hull of random lattice points, counter-clockwise
        pts = rng.integers(0, 40, size=(12, 2))
        pts = sorted(set(map(tuple, pts.tolist())))

        def cross(o, a, b):
            return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])
        lower, upper = [], []
        for p in pts:
            while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
                lower.pop()
            lower.append(p)
        for p in reversed(pts):
            while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
                upper.pop()
            upper.append(p)
        hull = lower[:-1] + upper[:-1]
        if len(hull) < 3:
            continue
        hp = np.array(hull, dtype=np.float64) * Q
        for x in range(-1, 42, 2):
            for y in range(-1, 42, 2):
                want = all(cross(hull[k], hull[(k + 1) % len(hull)], (x, y)) >= 0
                           for k in range(len(hull)))
                assert _pip(hp, x, y) == want, (hull, x, y)
