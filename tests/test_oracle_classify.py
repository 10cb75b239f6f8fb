"""Pins of the oracle's cell classification and list construction.

Sec. 4.1 defines the classes by coverage: Full = 100 % of the cell covered,
Partial = less than 100 %, Empty = 0 %; and Sec. 1 asks for pairs that share
at least one point.  The oracle reads both with closed sets: a cell whose
closed square touches the polygon only on the cell's border is Partial (it
is in the A-list), so touching polygons share a cell.

Independent checks:
  * exact coverage area of every cell, computed here by clipping the polygon
    to the cell in rational arithmetic: Full <=> area = w^2, area > 0 =>
    not Empty, and for area-0 cells, Partial <=> an edge touches the closed
    cell (an orientation-based test written here);
  * closed forms for rectangles and right triangles whose edges lie on grid
    lines or through cell centres;
  * the area sandwich |F| w^2 <= area(P) <= |A| w^2 (exact);
  * every vertex's cells are non-empty; random lattice points inside P lie
    in A cells; random points in F cells lie inside P (point-in-polygon
    written here);
  * list invariants: sorted, disjoint, maximal, F inside A, and the lists
    expand to exactly the Hilbert ids of the classified cells.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth.grid import Grid
from synth.polygons import LATTICE, PolygonSet, star_polygons

# order-6 grid with 2^20 lattice units per cell (cell side 2^-10)
W = 1 << 20
G6 = Grid(0.0, 0.0, float(W * 64) * LATTICE, 6)


def world(pts_cells):
    """Cell-unit coordinates (multiples of 1/2^20 allowed) -> world floats."""
    return np.array([[x * W * LATTICE, y * W * LATTICE] for x, y in pts_cells], dtype=np.float64)


def classes_by_cell(grid, xy):
    c = oracle.classify(grid, xy)
    return {(int(i), int(j)): int(k) for i, j, k in c}


# ---------------------------------------------------------------- helpers

def clip_area(poly, x0, y0, x1, y1):
    """Exact area of polygon ∩ box via successive half-plane clipping."""
    pts = [(Fraction(x), Fraction(y)) for x, y in poly]

    def clip(pts, inside, cut):
        out = []
        for k in range(len(pts)):
            a, b = pts[k - 1], pts[k]
            ia, ib = inside(a), inside(b)
            if ib:
                if not ia:
                    out.append(cut(a, b))
                out.append(b)
            elif ia:
                out.append(cut(a, b))
        return out

    def cut_x(c):
        return lambda a, b: (c, a[1] + (b[1] - a[1]) * (c - a[0]) / (b[0] - a[0]))

    def cut_y(c):
        return lambda a, b: (a[0] + (b[0] - a[0]) * (c - a[1]) / (b[1] - a[1]), c)

    for inside, cut in ((lambda p: p[0] >= x0, cut_x(x0)), (lambda p: p[0] <= x1, cut_x(x1)),
                        (lambda p: p[1] >= y0, cut_y(y0)), (lambda p: p[1] <= y1, cut_y(y1))):
        if not pts:
            return Fraction(0)
        pts = clip(pts, inside, cut)
    if len(pts) < 3:
        return Fraction(0)
    s = sum(pts[k - 1][0] * pts[k][1] - pts[k][0] * pts[k - 1][1] for k in range(len(pts)))
    return abs(s) / 2


def _orient(a, b, c):
    v = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    return (v > 0) - (v < 0)


def seg_touches_closed_box(a, b, x0, y0, x1, y1):
    """Separating-axis test: closed segment vs closed axis-aligned box."""
    if max(a[0], b[0]) < x0 or min(a[0], b[0]) > x1 or max(a[1], b[1]) < y0 or min(a[1], b[1]) > y1:
        return False
    s = {_orient(a, b, c) for c in ((x0, y0), (x1, y0), (x1, y1), (x0, y1))}
    return not (s == {1} or s == {-1})


def point_in_polygon(poly, p):
    """+1 inside, 0 on the boundary, -1 outside (winding by ray casting)."""
    n = len(poly)
    inside = False
    for k in range(n):
        a, b = poly[k], poly[(k + 1) % n]
        if _orient(a, b, p) == 0 and min(a[0], b[0]) <= p[0] <= max(a[0], b[0]) \
                and min(a[1], b[1]) <= p[1] <= max(a[1], b[1]):
            return 0
        if (a[1] > p[1]) != (b[1] > p[1]):
            # x of crossing > p.x ?
            num = (a[0] - p[0]) * (b[1] - a[1]) + (p[1] - a[1]) * (b[0] - a[0])
            if (num > 0) == (b[1] - a[1] > 0):
                inside = not inside
    return 1 if inside else -1


def lattice_poly(xy, grid):
    return [(round((x - grid.x0) / LATTICE), round((y - grid.y0) / LATTICE)) for x, y in xy]


def small_star_polys(seed, count, order_cells=64, lattice_to_grid_points=False):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(12, order_cells - 12, size=(count, 2))
    radii = rng.uniform(2.0, 9.0, size=count)
    nv = rng.integers(3, 12, size=count)
    ps = star_polygons(rng, centres * W * LATTICE, radii * W * LATTICE, nv, a=0.5)
    if lattice_to_grid_points:
        # put every vertex on a grid point or cell-edge midpoint: many exact
        # touches of grid lines and corners
        q = W * LATTICE / 2
        xy = np.round(ps.xy / q) * q
        good = []
        for k in range(len(ps)):
            p = xy[ps.voff[k]:ps.voff[k + 1]]
            L = [(round(x / LATTICE), round(y / LATTICE)) for x, y in p]
            c = (round(centres[k, 0] * W), round(centres[k, 1] * W))
            if len(set(L)) == len(L) and all(_orient(c, L[t], L[(t + 1) % len(L)]) > 0 for t in range(len(L))):
                good.append(p)
        voff = np.zeros(len(good) + 1, dtype=np.int64)
        np.cumsum([len(p) for p in good], out=voff[1:])
        ps = PolygonSet(np.concatenate(good), voff)
    return ps


# ------------------------------------------------------------- coverage pin

@pytest.mark.parametrize("aligned", [False, True])
def test_classes_match_exact_coverage(aligned):
    ps = small_star_polys(7 + aligned, 40, lattice_to_grid_points=aligned)
    assert len(ps) >= 20
    checked = 0
    for k in range(len(ps)):
        xy = ps.polygon(k)
        poly = lattice_poly(xy, G6)
        cls = classes_by_cell(G6, xy)
        xs = [p[0] for p in poly]
        ys = [p[1] for p in poly]
        # a window one cell wider than the polygon's MBR on every side
        for i in range(min(xs) // W - 1, max(xs) // W + 2):
            for j in range(min(ys) // W - 1, max(ys) // W + 2):
                box = (i * W, j * W, (i + 1) * W, (j + 1) * W)
                area = clip_area(poly, *box)
                c = cls.get((i, j), oracle.EMPTY)
                if area == W * W:
                    assert c == oracle.FULL, (k, i, j)
                elif area > 0:
                    assert c == oracle.PARTIAL, (k, i, j)
                else:
                    touch = any(seg_touches_closed_box(poly[t], poly[(t + 1) % len(poly)], *box)
                                for t in range(len(poly)))
                    assert c == (oracle.PARTIAL if touch else oracle.EMPTY), (k, i, j, touch)
                checked += 1
    assert checked > 1000


# ------------------------------------------------------------ closed forms

def a_f_counts(grid, xy):
    L = oracle.build_lists(grid, PolygonSet(xy, np.array([0, len(xy)], dtype=np.int64)))
    nA = int((L.eA.astype(np.int64) - L.sA).sum())
    nF = int((L.eF.astype(np.int64) - L.sF).sum())
    return nA, nF


@pytest.mark.parametrize("i0,j0,i1,j1", [(3, 3, 4, 4), (3, 5, 10, 9), (2, 2, 61, 61), (7, 20, 40, 21)])
def test_rectangle_on_grid_lines(i0, j0, i1, j1):
    xy = world([(i0, j0), (i1, j0), (i1, j1), (i0, j1)])
    nA, nF = a_f_counts(G6, xy)
    assert nF == (i1 - i0) * (j1 - j0)
    assert nA == (i1 - i0 + 2) * (j1 - j0 + 2)


@pytest.mark.parametrize("i0,j0,i1,j1", [(3, 3, 4, 4), (3, 5, 10, 9), (5, 6, 30, 50)])
def test_rectangle_through_cell_centres(i0, j0, i1, j1):
    h = 0.5
    xy = world([(i0 + h, j0 + h), (i1 + h, j0 + h), (i1 + h, j1 + h), (i0 + h, j1 + h)])
    nA, nF = a_f_counts(G6, xy)
    assert nF == (i1 - i0 - 1) * (j1 - j0 - 1)
    assert nA == (i1 - i0 + 1) * (j1 - j0 + 1)


@pytest.mark.parametrize("k", [1, 2, 3, 7, 20])
def test_right_triangle_on_grid_lines(k):
    # legs on x = 10 and y = 10 (cell units), hypotenuse through grid corners
    xy = world([(10, 10), (10 + k, 10), (10, 10 + k)])
    nA, nF = a_f_counts(G6, xy)
    assert nF == k * (k - 1) // 2
    assert nA == k * (k - 1) // 2 + 4 * k + 4


def test_tiny_polygon_inside_one_cell():
    xy = world([(20.25, 20.25), (20.75, 20.25), (20.5, 20.75)])
    nA, nF = a_f_counts(G6, xy)
    assert (nA, nF) == (1, 0)


def test_guard_ring_rejected():
    xy = world([(0.5, 10), (5, 10), (5, 15)])
    with pytest.raises(oracle.OracleError):
        oracle.build_lists(G6, PolygonSet(xy, np.array([0, 3], dtype=np.int64)))


# --------------------------------------------------------------- invariants

def _check_lists(s, e):
    s = s.astype(np.int64)
    e = e.astype(np.int64)
    assert np.all(s < e)
    assert np.all(e[:-1] < s[1:])         # sorted, disjoint and maximal


def _expand(s, e):
    return set(int(x) for a, b in zip(s, e) for x in range(int(a), int(b)))


def test_lists_expand_to_classified_cells():
    R, S, g = synth.configs.tiny(n=60)
    L = oracle.build_lists(g, R)
    for k in range(len(R)):
        c = oracle.classify(g, R.polygon(k))
        nz = c[c[:, 2] != oracle.EMPTY]
        full = c[c[:, 2] == oracle.FULL]
        ids_a = set(oracle.hilbert(g.order, nz[:, 0], nz[:, 1]).tolist())
        ids_f = set(oracle.hilbert(g.order, full[:, 0], full[:, 1]).tolist())
        sa, ea = L.A(k)
        sf, ef = L.F(k)
        _check_lists(sa, ea)
        _check_lists(sf, ef)
        assert _expand(sa, ea) == ids_a
        assert _expand(sf, ef) == ids_f
        assert ids_f <= ids_a
        assert len(sa) >= 1
        assert int(ea.max()) <= (1 << (2 * g.order)) - 1


def test_area_sandwich_and_points():
    R, S, g = synth.configs.tiny(n=80)
    w = g.cell_lattice
    rng = np.random.default_rng(5)
    L = oracle.build_lists(g, S)
    for k in range(len(S)):
        xy = S.polygon(k)
        nA = int((L.A(k)[1].astype(np.int64) - L.A(k)[0]).sum())
        nF = int((L.F(k)[1].astype(np.int64) - L.F(k)[0]).sum())
        a2 = oracle.twice_area(xy)
        assert a2 > 0
        assert 2 * nF * w * w <= a2 <= 2 * nA * w * w
        cls = classes_by_cell(g, xy)
        poly = lattice_poly(xy, g)
        # every vertex lies in cells that are not Empty (all cells whose
        # closed square contains it)
        for X, Y in poly:
            for i in {X // w, (X // w) - (X % w == 0)}:
                for j in {Y // w, (Y // w) - (Y % w == 0)}:
                    assert cls.get((i, j), oracle.EMPTY) != oracle.EMPTY
        xs = [p[0] for p in poly]
        ys = [p[1] for p in poly]
        for _ in range(150):
            p = (int(rng.integers(min(xs), max(xs) + 1)), int(rng.integers(min(ys), max(ys) + 1)))
            where = point_in_polygon(poly, p)
            c = cls.get((p[0] // w, p[1] // w), oracle.EMPTY)
            if where >= 0:
                assert c != oracle.EMPTY
            if c == oracle.FULL:
                assert where >= 0
