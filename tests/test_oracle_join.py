"""Pins of the oracle's IntervalJoin and of Alg. 2's verdict logic.

IntervalJoin (Alg. 2) must report an overlap exactly when the two interval
lists share a cell, i.e. when the sets of ids they cover intersect; this is
checked against the expanded sets on random, nested, touching, identical and
one-sided lists.  The count of elements read is pinned on hand cases.  The
verdict logic is pinned by the paper's cell-pair table (golden file), by
join-order invariance (golden file) and by symmetry.
"""

import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from synth.intervals import ListSet, complement_list, random_lists

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ids(s, e):
    return set(x for a, b in zip(s.tolist(), e.tolist()) for x in range(a, b))


@st.composite
def interval_list(draw, hi=200):
    k = draw(st.integers(0, 12))
    vals = sorted(draw(st.sets(st.integers(0, hi), min_size=2 * k, max_size=2 * k)))
    s = np.array(vals[0::2], dtype=np.uint32)
    e = np.array(vals[1::2], dtype=np.uint32)
    return s, e


@settings(max_examples=600, deadline=None)
@given(interval_list(), interval_list())
def test_join_equals_set_intersection(X, Y):
    hit, rx, ry = oracle.interval_join(X, Y)
    assert hit == bool(ids(*X) & ids(*Y))
    assert rx <= len(X[0]) and ry <= len(Y[0])
    # it is symmetric in its result
    assert oracle.interval_join(Y, X)[0] == hit


def test_touching_is_not_overlap():
    X = (np.array([0, 10], np.uint32), np.array([5, 20], np.uint32))
    Y = (np.array([5, 20], np.uint32), np.array([10, 30], np.uint32))
    assert oracle.interval_join(X, Y)[0] is False
    Y2 = (np.array([5, 19], np.uint32), np.array([10, 30], np.uint32))
    assert oracle.interval_join(X, Y2)[0] is True


def test_reads_on_hand_cases():
    # X = [0,2) [4,6) [8,10); Y = [10,12): the loop walks all of X against Y_0
    X = (np.array([0, 4, 8], np.uint32), np.array([2, 6, 10], np.uint32))
    Y = (np.array([10], np.uint32), np.array([12], np.uint32))
    assert oracle.interval_join(X, Y) == (False, 3, 1)
    # overlap on the first comparison
    Z = (np.array([1], np.uint32), np.array([3], np.uint32))
    assert oracle.interval_join(X, Z) == (True, 1, 1)
    # ties advance X: X_0 end 2 == Y_0 end 2 -> i moves; X_1 vs Y_0 ends 6 > 2 -> j moves
    Y3 = (np.array([1, 7], np.uint32), np.array([2, 8], np.uint32))
    # comparisons: (X0,Y0) overlap [0,2)x[1,2) -> True at once
    assert oracle.interval_join(X, Y3) == (True, 1, 1)
    Y4 = (np.array([2, 6], np.uint32), np.array([4, 8], np.uint32))
    # (X0,Y0): 2<=4 -> i=1; (X1,Y0): 6>4 -> j=1; (X1,Y1): 6<=8 -> i=2; (X2,Y1): 10>8 -> j=2 stop
    assert oracle.interval_join(X, Y4) == (False, 3, 2)
    # empty lists read nothing
    E = (np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert oracle.interval_join(X, E) == (False, 0, 0)


@pytest.mark.parametrize("k", [1, 2, 63, 64, 65, 1000, 100_000])
def test_long_lists(k):
    rng = np.random.default_rng(k)
    X = random_lists(rng, k, 0, 40 * k + 100)
    C = complement_list(*X)
    # the complement touches X everywhere and never overlaps it
    assert oracle.interval_join(X, C)[0] is False
    assert oracle.interval_join(X, X)[0] is True
    if k > 1:
        # shift one gap end by one cell: exactly one overlap appears
        t = int(rng.integers(0, len(C[0])))
        C2 = (C[0].copy(), C[1].copy())
        C2[1][t] += 1
        assert oracle.interval_join(X, C2)[0] is True


def _single(cell, full):
    s = np.array([cell], np.uint32)
    e = np.array([cell + 1], np.uint32)
    z = np.zeros(0, np.uint32)
    return (s, e), ((s, e) if full else (z, z))


def _lists_of(objs):
    A = ListSet.from_lists([o[0] for o in objs])
    F = ListSet.from_lists([o[1] for o in objs])
    return oracle.Lists(A.off, A.start, A.end, F.off, F.start, F.end)


def test_cell_matching_table():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "cell_matching.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 8
    code = {"TN": oracle.TN, "TH": oracle.TH, "IND": oracle.IND}
    for rc, sc, shared, want in rows:
        r = _single(100, rc == "full")
        s = _single(100 if shared == "yes" else 200, sc == "full")
        v = oracle.filter_pairs(_lists_of([r]), _lists_of([s]), [0], [0])
        assert v[0] == code[want], (rc, sc, shared)


def _verdict(order, Ar, Fr, As, Fs):
    """Alg. 2 with the three joins run in `order`: an empty AA-join ends
    with a true negative, a non-empty AF- or FA-join with a true hit."""
    for step in order:
        X, Y = {"AA": (Ar, As), "AF": (Ar, Fs), "FA": (Fr, As)}[step]
        hit = oracle.interval_join(X, Y)[0]
        if step == "AA" and not hit:
            return oracle.TN
        if step != "AA" and hit:
            return oracle.TH
    return oracle.IND


def test_join_order_invariance():
    orders = [ln.split() for ln in open(os.path.join(GOLDEN, "join_order.txt"))
              if ln.strip() and not ln.startswith("#")]
    assert len(orders) == 4
    rng = np.random.default_rng(3)
    seen = set()
    for _ in range(3000):
        objs = []
        for _side in range(2):
            A = random_lists(rng, int(rng.integers(1, 6)), 0, 60)
            # F: a random subset of A's cells, re-intervalized
            cells = sorted(c for c in ids(*A) if rng.random() < 0.5)
            if cells:
                runs = []
                st_ = cells[0]
                prev = cells[0]
                for c in cells[1:] + [None]:
                    if c is None or c != prev + 1:
                        runs.append((st_, prev + 1))
                        if c is not None:
                            st_ = c
                    if c is not None:
                        prev = c
                F = (np.array([a for a, _ in runs], np.uint32), np.array([b for _, b in runs], np.uint32))
            else:
                F = (np.zeros(0, np.uint32), np.zeros(0, np.uint32))
            objs.append((A, F))
        (Ar, Fr), (As, Fs) = objs
        v = [_verdict(o, Ar, Fr, As, Fs) for o in orders]
        assert len(set(v)) == 1
        got = oracle.filter_pairs(_lists_of([objs[0]]), _lists_of([objs[1]]), [0], [0])[0]
        assert got == v[0]
        # symmetry: swapping the roles of r and s keeps the verdict
        assert oracle.filter_pairs(_lists_of([objs[1]]), _lists_of([objs[0]]), [0], [0])[0] == got
        seen.add(int(got))
    assert seen == {oracle.TN, oracle.TH, oracle.IND}


def test_bytes_accounting():
    # r: A=[0,2)[4,6)  F=[4,6)      s: A=[5,7)  F=[]
    r = ((np.array([0, 4], np.uint32), np.array([2, 6], np.uint32)),
         (np.array([4], np.uint32), np.array([6], np.uint32)))
    s = ((np.array([5], np.uint32), np.array([7], np.uint32)),
         (np.zeros(0, np.uint32), np.zeros(0, np.uint32)))
    v, b = oracle.filter_pairs(_lists_of([r]), _lists_of([s]), [0], [0], want_bytes=True)
    # AA: (A0,S0) 2<=7 i=1; (A1,S0) overlap -> reads A(r) 2, A(s) 1
    # AF: F(s) empty -> no reads;  FA: (F0, S0) overlap -> F(r) 1, A(s) 1
    assert v[0] == oracle.TH
    assert b[0] == 8 + 16 * 4 + 8 * (2 + 1 + 0 + 1) + 1
