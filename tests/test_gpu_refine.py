"""Parity of the GPU refinement step with the oracle's exact geometry.

The refinement answers, for a candidate pair the filter left indecisive,
whether the two closed polygons share a point (Sec. 2: the pairs the
intermediate filter cannot decide go to exact geometry).  Every result here
is bit-exact against oracle.polygons_intersect, itself pinned by hand cases
(shared edge, shared corner, one-unit gap, nesting both ways, vertex on an
edge, a concave notch).

Cases:
  * the oracle's hand cases, both argument orders;
  * small rectilinear and triangular shapes on a coarse lattice, where
    shared edges, collinear overlaps, touching corners and nesting are
    common;
  * star polygons with 8 .. 400 vertices (edge chunks of either side
    gathered several times), and nested ones with no boundary contact;
  * pairs spanning 2^31 lattice units or more (the 128-bit pass) and the
    same shapes at small scale;
  * the tiny workload: every MBR candidate pair with no verdict input, and
    with the filter's verdicts as input (TN -> 0 and TH -> 1 without
    geometry);
  * the at-scale workload (200k x 200k polygons): all candidate pairs with
    the filter's verdicts, a random sample of indecisive pairs checked one by
    one, and every TN / TH pair checked against its verdict;
  * edge cases: no pairs, out-of-range ids, bad collections.
"""

import sys

import numpy as np
import pytest

import oracle
import synth
from synth.polygons import LATTICE, PolygonSet, star_polygons

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2307_01716_amd import april  # noqa: E402

Q = LATTICE * 1024


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def polys(ps: PolygonSet):
    P = april.april_polys_to_device(ps.xy, ps.voff, april.STRICT)
    torch.cuda.synchronize()
    return P


def from_list(shapes):
    lens = [len(p) for p in shapes]
    voff = np.zeros(len(shapes) + 1, np.int64)
    np.cumsum(lens, out=voff[1:])
    return PolygonSet(np.concatenate(shapes).astype(np.float64), voff)


def refine(PR, PS, r, s, verdict=None):
    n = len(r)
    out = torch.full((max(n, 1),), 77, dtype=torch.uint8, device="cuda")[:n]
    cnt = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    april.april_refine_pairs(PR, PS, cuda(np.asarray(r, np.uint32)), cuda(np.asarray(s, np.uint32)), out,
                             verdict=None if verdict is None else cuda(np.asarray(verdict, np.uint8)),
                             counts=cnt)
    torch.cuda.synchronize()
    return out.cpu().numpy(), cnt.cpu().numpy()


def want_of(R, S, r, s):
    return np.array([int(oracle.polygons_intersect(R.polygon(int(a)), S.polygon(int(b))))
                     for a, b in zip(r, s)], np.uint8)


def sq(x, y, s):
    return np.array([[x, y], [x + s, y], [x + s, y + s], [x, y + s]], dtype=np.float64) * Q


def hand_shapes():
    a = sq(0, 0, 10)
    u = np.array([[0, 0], [30, 0], [30, 30], [20, 30], [20, 10], [10, 10], [10, 30], [0, 30]],
                 dtype=np.float64) * Q
    others = [sq(10, 0, 5), sq(10, 10, 5), sq(11, 0, 5), sq(2, 2, 3), sq(5, -5, 10),
              np.array([[12, 0], [20, 0], [12, 8]], dtype=np.float64) * Q,
              np.array([[10, 5], [20, 0], [20, 10]], dtype=np.float64) * Q,
              sq(12, 12, 5), sq(12, 8, 5), sq(-20, -20, 50)]
    return [a, u], others


def test_hand_cases():
    left, right = hand_shapes()
    R, S = from_list(left), from_list(right)
    r, s = np.meshgrid(np.arange(len(left)), np.arange(len(right)), indexing="ij")
    r, s = r.ravel(), s.ravel()
    want = want_of(R, S, r, s)
    say(f"[refine] hand cases {len(r)} pairs, {int(want.sum())} intersect")
    assert 0 < want.sum() < len(want)
    got, cnt = refine(polys(R), polys(S), r, s)
    assert np.array_equal(got, want)
    assert list(cnt) == [int(want.sum()), len(r)]
    # roles swapped
    got2, _ = refine(polys(S), polys(R), s, r)
    assert np.array_equal(got2, want)


def coarse_shapes(rng, n, span=12):
    """Rectangles, right triangles and L shapes with corners on a coarse
    integer lattice: contacts along edges and at corners are frequent."""
    out = []
    for _ in range(n):
        x, y = rng.integers(0, span, 2)
        w, h = rng.integers(1, 6, 2)
        kind = rng.integers(0, 3)
        if kind == 0:
            p = [[x, y], [x + w, y], [x + w, y + h], [x, y + h]]
        elif kind == 1:
            p = [[x, y], [x + w, y], [x, y + h]] if rng.random() < 0.5 else [[x, y], [x + w, y + h], [x, y + h]]
        else:
            if w < 2 or h < 2:
                w, h = w + 1, h + 1
            p = [[x, y], [x + w, y], [x + w, y + 1], [x + 1, y + 1], [x + 1, y + h], [x, y + h]]
        out.append(np.array(p, dtype=np.float64) * Q)
    return from_list(out)


def test_coarse_lattice_contacts():
    rng = np.random.default_rng(5)
    R, S = coarse_shapes(rng, 60), coarse_shapes(rng, 60)
    r, s = np.meshgrid(np.arange(60), np.arange(60), indexing="ij")
    r, s = r.ravel(), s.ravel()
    want = want_of(R, S, r, s)
    say(f"[refine] coarse lattice {len(r)} pairs, {int(want.sum())} intersect")
    got, cnt = refine(polys(R), polys(S), r, s)
    assert np.array_equal(got, want)
    assert list(cnt) == [int(want.sum()), len(r)]


def test_star_polygons_many_chunks():
    rng = np.random.default_rng(8)
    n = 80
    def make(nv):
        c = 0.5 + 0.004 * rng.standard_normal((n, 2))
        rad = rng.uniform(0.0005, 0.003, n)
        return star_polygons(rng, c, rad, nv)
    R = make(rng.integers(8, 400, n))
    S = make(rng.integers(8, 400, n))
    r, s = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r, s = r.ravel(), s.ravel()
    want = want_of(R, S, r, s)
    say(f"[refine] star polygons {len(r)} pairs, {int(want.sum())} intersect")
    assert 0 < want.sum() < len(want)
    got, cnt = refine(polys(R), polys(S), r, s)
    assert np.array_equal(got, want)


def test_nested_stars_no_contact():
    """Many-vertex polygons nested inside each other without boundary
    contact: only the crossing-number test decides (several 64-edge blocks)."""
    rng = np.random.default_rng(12)
    n = 24
    c = 0.5 + 0.01 * rng.standard_normal((n, 2))
    outer = star_polygons(rng, c, np.full(n, 0.002), rng.integers(100, 600, n))
    inner = star_polygons(rng, c, np.full(n, 0.0005), rng.integers(100, 600, n))
    r, s = np.arange(n), np.arange(n)
    want = want_of(outer, inner, r, s)
    assert want.all()
    got, _ = refine(polys(outer), polys(inner), r, s)
    assert np.array_equal(got, want)
    got, _ = refine(polys(inner), polys(outer), s, r)
    assert np.array_equal(got, want)


def wide_cases():
    """Coarse shapes at three scales (the larger two span 2^31 lattice units
    or more), and one square of side 6 against small shapes across the
    128-bit boundary: nested, crossing a corner, far away, touching at a
    vertex, one lattice unit apart."""
    out = []
    for scale in (1.0, 2.0 ** 10, 2.0 ** 20):   # shape units of 2^-20, 1 and 2^10
        R, S = coarse_shapes(np.random.default_rng(31), 40), coarse_shapes(np.random.default_rng(32), 40)
        r, s = np.meshgrid(np.arange(40), np.arange(40), indexing="ij")
        out.append((f"x{scale:g}", PolygonSet(R.xy * scale, R.voff), PolygonSet(S.xy * scale, S.voff),
                    r.ravel(), s.ravel(), None))
    big = np.array([[-3.0, -3.0], [3.0, -3.0], [3.0, 3.0], [-3.0, 3.0]])
    box = lambda x, y, w: np.array([[x, y], [x + w, y], [x + w, y + w], [x, y + w]])   # noqa: E731
    smalls = [box(0.0, 0.0, 0.5), box(-3.5, -3.5, 1.0), box(1000.0, 1000.0, 1.0),
              np.array([[3.0, 0.0], [4.0, 0.0], [4.0, 1.0]]),
              np.array([[3.0 + LATTICE, 0.0], [4.0, 0.0], [4.0, 1.0]])]
    out.append(("big", from_list([big]), from_list(smalls), np.zeros(len(smalls), np.int64),
                np.arange(len(smalls)), [1, 1, 0, 1, 0]))
    return out


def test_wide_coordinates():
    """Pairs spanning 2^31 lattice units or more take the 128-bit pass, the
    same shapes at a small scale the 64-bit one; both match the oracle."""
    for name, R, S, r, s, expect in wide_cases():
        want = want_of(R, S, r, s)
        if expect is not None:
            assert list(want) == expect
        say(f"[refine] wide {name}: {int(want.sum())} of {len(r)} intersect")
        got, cnt = refine(polys(R), polys(S), r, s)
        assert np.array_equal(got, want)
        assert list(cnt) == [int(want.sum()), len(r)]


@pytest.fixture(scope="module")
def tiny():
    R, S, g = synth.configs.tiny()
    r, s = oracle.mbr_join(R, S)
    LR, LS = oracle.build_lists(g, R), oracle.build_lists(g, S)
    v = oracle.filter_pairs(LR, LS, r, s)
    want = want_of(R, S, r, s)
    return R, S, r, s, v, want


def test_tiny_all_pairs(tiny):
    R, S, r, s, v, want = tiny
    say(f"[refine] tiny all {len(r)} pairs")
    got, cnt = refine(polys(R), polys(S), r, s)
    assert np.array_equal(got, want)
    assert list(cnt) == [int(want.sum()), len(r)]


def test_tiny_with_verdicts(tiny):
    R, S, r, s, v, want = tiny
    say(f"[refine] tiny with verdicts, {int((v == 2).sum())} indecisive")
    got, cnt = refine(polys(R), polys(S), r, s, verdict=v)
    assert np.array_equal(got, want)
    assert list(cnt) == [int(want.sum()), int((v == april.INDECISIVE).sum())]
    # a planted verdict is taken as given: TH on a disjoint pair gives 1
    vv = v.copy()
    dis = np.nonzero(want == 0)[0][:5]
    vv[dis] = april.TH
    got, _ = refine(polys(R), polys(S), r, s, verdict=vv)
    assert np.all(got[dis] == 1)


def test_edge_cases(tiny):
    R, S, r, s, v, want = tiny
    PR, PS = polys(R), polys(S)
    say("[refine] no pairs")
    got, cnt = refine(PR, PS, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert len(got) == 0 and list(cnt) == [0, 0]
    say("[refine] out-of-range ids")
    rr = np.array([r[0], len(R), 3, 0xFFFFFFFF], np.uint32)
    ss = np.array([s[0], 0, len(S), 1], np.uint32)
    got, cnt = refine(PR, PS, rr, ss)
    assert got[0] == want[0]
    assert list(got[1:]) == [april.BAD_PAIR] * 3
    assert list(cnt) == [int(want[0]), 1]
    with pytest.raises(april.AprilError):
        april.april_polys_to_device(np.zeros((2, 2)), np.array([0, 2], np.uint64))
    with pytest.raises(april.AprilError):
        april.april_polys_to_device(np.full((3, 2), 0.3), np.array([0, 3], np.uint64), april.STRICT)


@pytest.fixture(scope="module")
def scale():
    say("[refine scale] generating 200k x 200k")
    R, S, g = synth.configs.scale()
    r, s = oracle.mbr_join(R, S)
    dR = april.april_lists_to_device(april.april_build_lists(g, R.xy, R.voff, april.STRICT))
    dS = april.april_lists_to_device(april.april_build_lists(g, S.xy, S.voff, april.STRICT))
    v = torch.empty(len(r), dtype=torch.uint8, device="cuda")
    rt, st = cuda(r), cuda(s)
    april.april_filter_pairs(dR, dS, rt, st, v, schedule=april.SCHED_BATCHED)
    torch.cuda.synchronize()
    return R, S, r, s, v.cpu().numpy()


def test_scale_with_verdicts(scale):
    R, S, r, s, v = scale
    say(f"[refine scale] {len(r)} pairs, {int((v == 2).sum())} indecisive")
    got, cnt = refine(polys(R), polys(S), r, s, verdict=v)
    assert np.all(got[v == april.TH] == 1)
    assert np.all(got[v == april.TN] == 0)
    assert set(np.unique(got)) <= {0, 1}
    assert list(cnt) == [int(got.sum()), int((v == april.INDECISIVE).sum())]
    ind = np.nonzero(v == april.INDECISIVE)[0]
    pick = np.random.default_rng(23).choice(ind, 3000, replace=False)
    want = want_of(R, S, r[pick], s[pick])
    say(f"[refine scale] sampled {len(pick)} indecisive pairs, {int(want.sum())} intersect")
    assert np.array_equal(got[pick], want)
    assert 0 < want.sum() < len(want)
