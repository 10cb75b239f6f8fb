"""Parity of the GPU query variants with the oracle (bit-exact verdicts and
counts): within joins (Sec. 4.3.2), polygon-linestring joins (Sec. 4.3.3)
and Alg. 2 across grid orders (Sec. 5.3).

Cases:
  * tiny workloads: every candidate pair against the oracle's own lists;
  * at scale (200k polygons; 200k linestrings; orders 16 and 14): every
    candidate pair against the oracle's filter run on the library's lists
    (the library's builders are pinned against the oracle's elsewhere);
  * mixed orders both ways (R finer, S finer), and one order, which must
    equal april_filter_pairs; orders 16 x 15 both ways, where thousands of
    coarse objects are loaded in pieces;
  * polygons whose lists are longer than a tile (loaded in pieces) against
    linestrings;
  * edge cases: no pairs, ids out of range, grids that do not match.
"""

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2307_01716_amd import april  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def run(fn, A, B, a, b):
    n = len(a)
    v = torch.full((max(n, 1),), 77, dtype=torch.uint8, device="cuda")[:n]
    c = torch.full((3,), -1, dtype=torch.int64, device="cuda")
    fn(A, B, cuda(np.asarray(a, np.uint32)), cuda(np.asarray(b, np.uint32)), v, c)
    torch.cuda.synchronize()
    return v.cpu().numpy(), c.cpu().numpy()


def host_lists(grid, ps):
    return april.april_build_lists(grid, ps.xy, ps.voff, april.STRICT)


def dev(h):
    d = april.april_lists_to_device(h)
    torch.cuda.synchronize()
    return d


def as_oracle(h):
    return oracle.Lists(*h.export())


def check(got, cnt, want):
    assert np.array_equal(got, want)
    assert np.array_equal(cnt, np.bincount(want, minlength=3)[:3])


# ------------------------------------------------------------------ within

def test_within_tiny():
    R, S, g = synth.configs.tiny()
    LR, LS = oracle.build_lists(g, R), oracle.build_lists(g, S)
    r, s = oracle.mbr_join(R, S)
    want = oracle.filter_within(LR, LS, r, s)
    say(f"[within] tiny {len(r)} pairs")
    got, cnt = run(april.april_filter_within, dev(host_lists(g, R)), dev(host_lists(g, S)), r, s)
    check(got, cnt, want)
    assert set(np.unique(want)) == {0, 1, 2}


@pytest.fixture(scope="module")
def scale():
    R, S, g = synth.configs.scale()
    hR, hS = host_lists(g, R), host_lists(g, S)
    r, s = april.april_mbr_join(R.mbrs(), S.mbrs())
    return R, S, g, hR, hS, r, s


def test_within_scale(scale):
    R, S, g, hR, hS, r, s = scale
    say(f"[within] scale {len(r)} pairs")
    want = oracle.filter_within(as_oracle(hR), as_oracle(hS), r, s)
    got, cnt = run(april.april_filter_within, dev(hR), dev(hS), r, s)
    check(got, cnt, want)


# -------------------------------------------------------------- linestrings

def linestring_pairs(P, L):
    return april.april_mbr_join(P.mbrs(), L.mbrs())


def test_linestrings_tiny():
    P, L, g = synth.configs.linestring_scale(n_poly=1500, n_lines=1500)
    LP, CL = oracle.build_lists(g, P), oracle.build_cells(g, L)
    hC = april.april_build_cells(g, L.xy, L.voff, april.STRICT)
    off, ids = hC.export()
    assert np.array_equal(off, CL.off) and np.array_equal(ids, CL.ids)
    p, l = linestring_pairs(P, L)
    want = oracle.filter_linestrings(LP, CL, p, l)
    say(f"[linestrings] small {len(p)} pairs")
    dC = april.april_cells_to_device(hC)
    got, cnt = run(april.april_filter_linestrings, dev(host_lists(g, P)), dC, p, l)
    check(got, cnt, want)
    assert set(np.unique(want)) == {0, 1, 2}


def test_linestrings_scale():
    P, L, g = synth.configs.linestring_scale()
    hP = host_lists(g, P)
    hC = april.april_build_cells(g, L.xy, L.voff, april.STRICT)
    p, l = linestring_pairs(P, L)
    e = hP.export()
    big = (np.maximum(np.diff(e[0]), np.diff(e[3])) >= 256)[p]
    say(f"[linestrings] scale {len(p)} pairs, {int(big.sum())} with the polygon in pieces")
    assert big.sum() > 1000
    off, ids = hC.export()
    want = oracle.filter_linestrings(as_oracle(hP), oracle.Cells(off, ids), p, l)
    got, cnt = run(april.april_filter_linestrings, dev(hP), april.april_cells_to_device(hC), p, l)
    check(got, cnt, want)


# -------------------------------------------------------- different orders

def test_mixed_tiny_both_ways_and_one_order():
    R, S, _ = synth.configs.tiny()
    gf, gc = synth.configs.two_orders(R, S, 10, 8)
    r, s = oracle.mbr_join(R, S)
    for name, gR, gS in (("R fine", gf, gc), ("S fine", gc, gf), ("one order", gf, gf)):
        LR, LS = oracle.build_lists(gR, R), oracle.build_lists(gS, S)
        want = oracle.filter_mixed(LR, gR.order, LS, gS.order, r, s)
        say(f"[mixed] tiny {name}: {len(r)} pairs")
        dR, dS = dev(host_lists(gR, R)), dev(host_lists(gS, S))
        got, cnt = run(april.april_filter_mixed, dR, dS, r, s)
        check(got, cnt, want)
        if gR.order == gS.order:
            ref, _ = run(lambda A, B, a, b, v, c: april.april_filter_pairs(A, B, a, b, v, c), dR, dS, r, s)
            assert np.array_equal(got, ref)


def test_mixed_scale(scale):
    R, S, _, _, _, r, s = scale
    gf, gc = synth.configs.two_orders(R, S, 16, 14)
    hR, hS = host_lists(gf, R), host_lists(gc, S)
    say(f"[mixed] scale orders 16 x 14: {len(r)} pairs")
    want = oracle.filter_mixed(as_oracle(hR), 16, as_oracle(hS), 14, r, s)
    got, cnt = run(april.april_filter_mixed, dev(hR), dev(hS), r, s)
    check(got, cnt, want)


def test_mixed_pieces_both_ways(scale):
    """Orders 16 x 15: thousands of coarse objects have lists longer than a
    tile, so the resident coarse side is cut into pieces.  Every pair whose
    coarse object needs pieces, plus a random sample of the others."""
    R, S, _, _, _, r, s = scale
    gf, gc = synth.configs.two_orders(R, S, 16, 15)
    rng = np.random.default_rng(12)
    for name, gR, gS in (("R fine", gf, gc), ("S fine", gc, gf)):
        hR, hS = host_lists(gR, R), host_lists(gS, S)
        coarse = hS if gR is gf else hR
        e = coarse.export()
        big = np.maximum(np.diff(e[0]), np.diff(e[3])) >= 256
        sel = big[s] if gR is gf else big[r]
        pick = np.nonzero(sel | (rng.random(len(r)) < 0.02))[0]
        assert sel.sum() > 1000
        say(f"[mixed] 16 x 15 {name}: {int(sel.sum())} pairs with a coarse object in pieces, {len(pick)} checked")
        want = oracle.filter_mixed(as_oracle(hR), gR.order, as_oracle(hS), gS.order, r[pick], s[pick])
        got, cnt = run(april.april_filter_mixed, dev(hR), dev(hS), r[pick], s[pick])
        check(got, cnt, want)


# ----------------------------------------------------------------- edges

def test_edge_cases():
    R, S, g = synth.configs.tiny()
    dR, dS = dev(host_lists(g, R)), dev(host_lists(g, S))
    r, s = oracle.mbr_join(R, S)
    for fn in (april.april_filter_within, april.april_filter_mixed):
        got, cnt = run(fn, dR, dS, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
        assert len(got) == 0 and list(cnt) == [0, 0, 0]
        rr = np.array([r[0], len(R), 5, 0xFFFFFFFF], np.uint32)
        ss = np.array([s[0], 0, len(S) + 3, 1], np.uint32)
        got, cnt = run(fn, dR, dS, rr, ss)
        assert list(got[1:]) == [april.BAD_PAIR] * 3 and cnt.sum() == 1
    P, L, gl = synth.configs.linestring_scale(n_poly=300, n_lines=300)
    dP = dev(host_lists(gl, P))
    dC = april.april_cells_to_device(april.april_build_cells(gl, L.xy, L.voff, april.STRICT))
    got, cnt = run(april.april_filter_linestrings, dP, dC, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert len(got) == 0 and list(cnt) == [0, 0, 0]
    got, cnt = run(april.april_filter_linestrings, dP, dC, np.array([0, 300, 7, 0xFFFFFFFF], np.uint32),
                   np.array([0, 0, 300, 1], np.uint32))
    assert list(got[1:]) == [april.BAD_PAIR] * 3 and cnt.sum() == 1
    from synth.polygons import LATTICE
    w = g.cell_lattice * LATTICE
    other = synth.Grid(g.x0 - w, g.y0 - w, g.side, g.order)   # origin one cell off
    dS2 = dev(host_lists(other, S))
    with pytest.raises(april.AprilError) as e:
        run(april.april_filter_within, dR, dS2, r[:4], s[:4])
    assert e.value.code == april.E_GRID
    with pytest.raises(april.AprilError) as e:
        run(april.april_filter_mixed, dR, dS2, r[:4], s[:4])
    assert e.value.code == april.E_GRID
