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
