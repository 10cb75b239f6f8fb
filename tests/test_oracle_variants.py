"""Pins of the oracle's query variants (Sec. 4.3.2 within joins, Sec. 4.3.3
polygon-linestring joins, Sec. 5.3 different granularity).

Each variant is checked against the definition it implements, restated on
plain cell sets (Python sets, not intervals), on random small lists; and its
true negatives and true hits against exact geometry on the tiny workload.
The linestring cell builder is checked against an independent formulation of
"segment meets closed cell" (bounding boxes overlap and the cell's corners
are not all strictly on one side of the segment's line).
"""

import numpy as np
import pytest

import oracle
import synth
from synth.grid import Grid
from synth.polygons import LATTICE, PolygonSet

TN, TH, IND = 0, 1, 2


def runs(cells):
    """Sorted cell ids -> maximal half-open intervals (starts, ends)."""
    c = sorted(set(int(x) for x in cells))
    s, e = [], []
    for x in c:
        if e and e[-1] == x:
            e[-1] = x + 1
        else:
            s.append(x)
            e.append(x + 1)
    return s, e


def lists_of(sets_a, sets_f):
    """oracle.Lists from per-object A and F cell sets."""
    offA, sA, eA, offF, sF, eF = [0], [], [], [0], [], []
    for a, f in zip(sets_a, sets_f):
        s, e = runs(a)
        sA += s
        eA += e
        offA.append(len(sA))
        s, e = runs(f)
        sF += s
        eF += e
        offF.append(len(sF))
    u32 = lambda x: np.array(x, np.uint32)   # noqa: E731
    u64 = lambda x: np.array(x, np.uint64)   # noqa: E731
    return oracle.Lists(u64(offA), u32(sA), u32(eA), u64(offF), u32(sF), u32(eF))


def random_sets(rng, n, universe, p_fill=0.4):
    A, F = [], []
    for _ in range(n):
        a = set(np.nonzero(rng.random(universe) < rng.uniform(0.02, p_fill))[0].tolist())
        # F inside A: a random part of A, often contiguous blocks
        f = {x for x in a if rng.random() < 0.5}
        A.append(a)
        F.append(f)
    return A, F


# ------------------------------------------------------------------ within

def test_within_matches_set_definition():
    rng = np.random.default_rng(1)
    AR, FR = random_sets(rng, 40, 120)
    AS, FS = random_sets(rng, 40, 120, p_fill=0.9)
    # make some pairs true hits: A(r) inside F(s)
    for k in range(0, 40, 5):
        AR[k] = {x for x in FS[k] if rng.random() < 0.6} or set(list(FS[k])[:1]) or {3}
    LR, LS = lists_of(AR, FR), lists_of(AS, FS)
    r, s = np.meshgrid(np.arange(40), np.arange(40), indexing="ij")
    r, s = r.ravel(), s.ravel()
    got = oracle.filter_within(LR, LS, r, s)
    want = np.array([TN if not (AR[a] & AS[b]) else TH if AR[a] <= FS[b] else IND for a, b in zip(r, s)])
    assert np.array_equal(got, want)
    assert set(np.unique(want)) == {TN, TH, IND}


def test_within_sound_on_tiny():
    R, S, g = synth.configs.tiny()
    LR, LS = oracle.build_lists(g, R), oracle.build_lists(g, S)
    r, s = oracle.mbr_join(R, S)
    v = oracle.filter_within(LR, LS, r, s)
    for p in np.nonzero(v == TN)[0]:
        assert not oracle.polygons_intersect(R.polygon(int(r[p])), S.polygon(int(s[p])))
    for p in np.nonzero(v == TH)[0]:
        sp = S.polygon(int(s[p]))
        assert all(oracle.point_in_closed_polygon(sp, x, y) for x, y in R.polygon(int(r[p])))
    assert (v == TH).sum() > 0 and (v == TN).sum() > 0


W = 1 << 20
COARSE = Grid(0.0, 0.0, 64 * W * LATTICE, 6)


def sq(x, y, w):
    return np.array([[x, y], [x + w, y], [x + w, y + w], [x, y + w]], dtype=np.float64) * W * LATTICE


def test_within_hand_cases():
    outer = sq(4, 4, 30)
    shapes_r = [sq(10, 10, 5), sq(4, 4, 30), sq(40, 40, 5), sq(30, 30, 10)]
    want = [TH, IND, TN, IND]    # nested, identical, disjoint, partly outside
    Rp = PolygonSet(np.concatenate(shapes_r), np.arange(0, 17, 4))
    Sp = PolygonSet(outer, np.array([0, 4]))
    LR, LS = oracle.build_lists(COARSE, Rp), oracle.build_lists(COARSE, Sp)
    got = oracle.filter_within(LR, LS, np.arange(4), np.zeros(4))
    assert list(got) == want


# -------------------------------------------------------------- linestrings

def lines_set(rng, n, lo, hi, max_pts=6):
    xy, voff = [], [0]
    for _ in range(n):
        k = int(rng.integers(2, max_pts + 1))
        pts = rng.integers(lo, hi, size=(k, 2)).astype(np.float64)
        xy.append(pts)
        voff.append(voff[-1] + k)
    return PolygonSet(np.concatenate(xy), np.array(voff, np.int64))


def cells_by_corners(x0, y0, x1, y1, w, n):
    """Cells whose closed square meets segment (x0,y0)-(x1,y1), all in
    lattice units: boxes overlap and the corners are not all strictly on one
    side of the line through the segment."""
    out = set()
    for j in range(n):
        for i in range(n):
            bx0, by0, bx1, by1 = i * w, j * w, (i + 1) * w, (j + 1) * w
            if max(x0, x1) < bx0 or min(x0, x1) > bx1 or max(y0, y1) < by0 or min(y0, y1) > by1:
                continue
            if (x0, y0) == (x1, y1):
                out.add((i, j))
                continue
            sides = {np.sign((x1 - x0) * (cy - y0) - (y1 - y0) * (cx - x0))
                     for cx in (bx0, bx1) for cy in (by0, by1)}
            if not (sides == {1} or sides == {-1}):
                out.add((i, j))
    return out


def test_cells_match_corner_test():
    rng = np.random.default_rng(7)
    order, n = 5, 32
    g = Grid(0.0, 0.0, n * W * LATTICE, order)
    # vertices on a half-cell lattice (corners, edges and centres of cells)
    L = lines_set(rng, 30, 3, 2 * n - 3)
    L = PolygonSet(L.xy * (W // 2) * LATTICE, L.voff)
    C = oracle.build_cells(g, L)
    for k in range(len(L)):
        pts = np.round(L.polygon(k) / LATTICE).astype(np.int64)
        want = set()
        for a in range(len(pts) - 1):
            want |= cells_by_corners(int(pts[a, 0]), int(pts[a, 1]), int(pts[a + 1, 0]), int(pts[a + 1, 1]), W, n)
        ids = sorted(oracle.hilbert(order, np.array([c[0] for c in want]), np.array([c[1] for c in want])))
        assert list(C.cells(k)) == ids, k


def test_linestring_filter_matches_set_definition():
    rng = np.random.default_rng(3)
    AP, FP = random_sets(rng, 30, 150, p_fill=0.7)
    cells = [set(np.nonzero(rng.random(150) < 0.05)[0].tolist()) or {7} for _ in range(30)]
    LP = lists_of(AP, FP)
    off = np.concatenate([[0], np.cumsum([len(c) for c in cells])]).astype(np.uint64)
    ids = np.concatenate([sorted(c) for c in cells]).astype(np.uint32)
    CL = oracle.Cells(off, ids)
    p, l = np.meshgrid(np.arange(30), np.arange(30), indexing="ij")
    p, l = p.ravel(), l.ravel()
    got = oracle.filter_linestrings(LP, CL, p, l)
    want = np.array([TN if not (AP[a] & cells[b]) else TH if FP[a] & cells[b] else IND for a, b in zip(p, l)])
    assert np.array_equal(got, want)
    assert set(np.unique(want)) == {TN, TH, IND}


def test_linestring_filter_sound():
    R, _, g = synth.configs.tiny()
    rng = np.random.default_rng(11)
    # short random linestrings near the polygons, on the lattice
    starts = R.xy[rng.integers(0, len(R.xy), 400)]
    lo, hi = R.xy.min(axis=0), R.xy.max(axis=0)   # inside the grid's guarded interior
    xy, voff = [], [0]
    for st in starts:
        k = int(rng.integers(2, 5))
        steps = rng.normal(0, 0.01, size=(k - 1, 2))
        pts = np.clip(np.vstack([st, st + np.cumsum(steps, axis=0)]), lo, hi)
        xy.append(np.round(pts / LATTICE) * LATTICE)
        voff.append(voff[-1] + k)
    L = PolygonSet(np.concatenate(xy), np.array(voff, np.int64))
    LP, CL = oracle.build_lists(g, R), oracle.build_cells(g, L)
    # candidate pairs: MBRs meet
    p, l = oracle.mbr_join(R, L)
    v = oracle.filter_linestrings(LP, CL, p, l)
    for q in range(len(p)):
        hit = oracle.linestring_meets_polygon(L.polygon(int(l[q])), R.polygon(int(p[q])))
        if v[q] == TN:
            assert not hit
        if v[q] == TH:
            assert hit
    assert (v == TH).sum() > 0 and (v == TN).sum() > 0


# -------------------------------------------------------- different orders

def test_mixed_matches_set_definition():
    rng = np.random.default_rng(5)
    N, Lo = 5, 3                       # fine order 5 (1024 cells), coarse order 3 (64 cells)
    shift = 2 * (N - Lo)
    AF_, FF_ = random_sets(rng, 25, 4 ** N, p_fill=0.1)     # fine side
    AC, FC = random_sets(rng, 25, 4 ** Lo, p_fill=0.5)      # coarse side
    LF, LC = lists_of(AF_, FF_), lists_of(AC, FC)
    r, s = np.meshgrid(np.arange(25), np.arange(25), indexing="ij")
    r, s = r.ravel(), s.ravel()

    def want(fine, coarse):
        m = {c >> shift for c in AF_[fine]}
        return TN if not (m & AC[coarse]) else TH if m & FC[coarse] else IND

    got = oracle.filter_mixed(LF, N, LC, Lo, r, s)           # R fine
    assert np.array_equal(got, np.array([want(a, b) for a, b in zip(r, s)]))
    got = oracle.filter_mixed(LC, Lo, LF, N, s, r)           # S fine
    assert np.array_equal(got, np.array([want(a, b) for a, b in zip(r, s)]))


def test_mixed_sound_on_tiny():
    R, S, _ = synth.configs.tiny()
    # one data space at orders 8 and 10: a coarse cell side divisible by 4
    # and a guard ring of two coarse cells
    lo = np.round(np.minimum(R.xy.min(0), S.xy.min(0)) / LATTICE).astype(np.int64)
    hi = np.round(np.maximum(R.xy.max(0), S.xy.max(0)) / LATTICE).astype(np.int64)
    w8 = (int((hi - lo).max()) // 252 + 1 + 3) // 4 * 4
    x0, y0 = (lo - 2 * w8) * LATTICE
    g8 = Grid(float(x0), float(y0), float(w8 * 256) * LATTICE, 8)
    g = Grid(g8.x0, g8.y0, g8.side, 10)
    LR, LS = oracle.build_lists(g, R), oracle.build_lists(g8, S)
    r, s = oracle.mbr_join(R, S)
    v = oracle.filter_mixed(LR, g.order, LS, g8.order, r, s)
    for p in range(len(r)):
        if v[p] == IND:
            continue
        hit = oracle.polygons_intersect(R.polygon(int(r[p])), S.polygon(int(s[p])))
        assert hit == (v[p] == TH), p
    assert (v == TH).sum() > 0 and (v == TN).sum() > 0


def test_linestring_runs_give_the_cell_verdicts():
    """The GPU path streams a linestring's cells as maximal runs of
    consecutive ids.  A run [c0, c1 + 1) meets an interval exactly when one of
    its cells [c, c + 1) does, so Alg. 2's joins on the runs must give the
    oracle's cell-by-cell verdicts (Sec. 4.3.3) -- checked here with the
    oracle's own interval join on every candidate pair of a small workload."""
    P, L, g = synth.configs.linestring_scale(n_poly=1500, n_lines=1500)
    LP, CL = oracle.build_lists(g, P), oracle.build_cells(g, L)
    p, l = oracle.mbr_join(P, L)
    want = oracle.filter_linestrings(LP, CL, p, l)
    run_lists = [runs(CL.cells(k)) for k in range(len(CL))]
    shorter = sum(len(s) for s, _ in run_lists) < len(CL.ids)
    got = []
    for a, b in zip(p, l):
        rs = run_lists[b]
        if not oracle.interval_join(LP.A(a), rs)[0]:
            got.append(TN)
        else:
            got.append(TH if oracle.interval_join(LP.F(a), rs)[0] else IND)
    assert np.array_equal(np.array(got, np.uint8), want)
    assert set(np.unique(want)) == {TN, TH, IND} and shorter
