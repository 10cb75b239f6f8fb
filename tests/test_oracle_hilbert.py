"""Pins of the oracle's Hilbert numbering (Sec. 3.2: cells are ordered along
the Hilbert curve, ids in [0, 2^{2N} - 1]).

The oracle uses the quadrant-by-quadrant rotate/reflect conversion.  It is
checked against an independent construction (the curve of order n is built
as an explicit path from four transformed copies of the order n-1 path),
against the curve's defining properties (a bijection onto [0, 4^N) whose
consecutive cells are edge neighbours, starting at the lower-left corner and
ending at the lower-right one) and against the self-similarity that links
order N to order N-1, which reaches order 16.
"""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def path(n):
    """Cells of the order-n curve in curve order, built recursively.

    Order 1 visits (0,0), (0,1), (1,1), (1,0).  Order n puts the order n-1
    path, with side s = 2^(n-1), into the four quadrants: transposed in the
    lower-left, shifted up in the upper-left, shifted up and right in the
    upper-right, and reflected across the anti-diagonal into the
    lower-right, so that each copy ends next to where the next one starts.
    """
    if n == 1:
        return [(0, 0), (0, 1), (1, 1), (1, 0)]
    prev = path(n - 1)
    s = 1 << (n - 1)
    out = [(y, x) for x, y in prev]
    out += [(x, y + s) for x, y in prev]
    out += [(x + s, y + s) for x, y in prev]
    out += [(2 * s - 1 - y, s - 1 - x) for x, y in prev]
    return out


def test_order1_table():
    got = [int(oracle.hilbert(1, [x], [y])[0]) for x, y in [(0, 0), (0, 1), (1, 1), (1, 0)]]
    assert got == [0, 1, 2, 3]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_matches_recursive_construction(n):
    p = np.array(path(n), dtype=np.uint64)
    d = oracle.hilbert(n, p[:, 0], p[:, 1])
    assert np.array_equal(d, np.arange(len(p), dtype=np.uint64))


@pytest.mark.parametrize("n", [2, 5, 8])
def test_bijection_and_adjacency(n):
    side = 1 << n
    xs, ys = np.meshgrid(np.arange(side, dtype=np.uint64), np.arange(side, dtype=np.uint64))
    d = oracle.hilbert(n, xs.ravel(), ys.ravel())
    assert np.array_equal(np.sort(d), np.arange(side * side, dtype=np.uint64))
    inv = np.empty((side * side, 2), dtype=np.int64)
    inv[d.astype(np.int64), 0] = xs.ravel().astype(np.int64)
    inv[d.astype(np.int64), 1] = ys.ravel().astype(np.int64)
    step = np.abs(np.diff(inv, axis=0)).sum(axis=1)
    assert np.all(step == 1)
    assert tuple(inv[0]) == (0, 0)
    assert tuple(inv[-1]) == (side - 1, 0)


def test_order16_corners():
    n = 16
    last = (1 << n) - 1
    assert int(oracle.hilbert(n, [0], [0])[0]) == 0
    assert int(oracle.hilbert(n, [last], [0])[0]) == (1 << 32) - 1
    # the upper-left quadrant is the second quarter of the curve
    assert (1 << 30) <= int(oracle.hilbert(n, [0], [last])[0]) < (2 << 30)


@pytest.mark.parametrize("n", [9, 12, 16])
def test_self_similarity(n):
    """Order n on random cells equals order n-1 in the quadrant's frame."""
    rng = np.random.default_rng(n)
    s = 1 << (n - 1)
    x = rng.integers(0, 2 * s, 4000).astype(np.uint64)
    y = rng.integers(0, 2 * s, 4000).astype(np.uint64)
    d = oracle.hilbert(n, x, y).astype(np.int64)
    xi, yi = x.astype(np.int64), y.astype(np.int64)
    q = np.where(xi < s, np.where(yi < s, 0, 1), np.where(yi < s, 3, 2))
    lx = np.where(q == 0, yi, np.where(q == 1, xi, np.where(q == 2, xi - s, s - 1 - yi)))
    ly = np.where(q == 0, xi, np.where(q == 1, yi - s, np.where(q == 2, yi - s, 2 * s - 1 - xi)))
    sub = oracle.hilbert(n - 1, lx.astype(np.uint64), ly.astype(np.uint64)).astype(np.int64)
    assert np.array_equal(d, q * s * s + sub)
