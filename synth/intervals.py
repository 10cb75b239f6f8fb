"""Random sorted, disjoint, non-touching half-open interval lists.

Used to exercise the interval joins on inputs with no geometry behind them:
any lengths (0 .. 10^6), any overlap structure.  A list with k intervals is
built from 2k distinct sorted integers v_0 < v_1 < ... < v_{2k-1} drawn from
[lo, hi): interval i is [v_{2i}, v_{2i+1}).  Distinctness makes every end
strictly smaller than the next start, so the lists are maximal as well.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ListSet:
    """Interval lists of a collection in CSR/SoA form (the A or F lists).

    off   uint64 [n+1]  object k owns intervals off[k]:off[k+1]
    start uint32 [T]
    end   uint32 [T]
    """

    off: np.ndarray
    start: np.ndarray
    end: np.ndarray

    def __len__(self):
        return len(self.off) - 1

    def get(self, k):
        a, b = int(self.off[k]), int(self.off[k + 1])
        return self.start[a:b], self.end[a:b]

    @staticmethod
    def from_lists(lists):
        lens = np.array([len(s) for s, _ in lists], dtype=np.uint64)
        off = np.zeros(len(lists) + 1, dtype=np.uint64)
        np.cumsum(lens, out=off[1:])
        if len(lists):
            st = np.concatenate([np.asarray(s, dtype=np.uint32) for s, _ in lists])
            en = np.concatenate([np.asarray(e, dtype=np.uint32) for _, e in lists])
        else:
            st = np.zeros(0, np.uint32)
            en = np.zeros(0, np.uint32)
        return ListSet(off, st, en)


def random_lists(rng: np.random.Generator, k: int, lo: int = 0, hi: int = 2 ** 32 - 1):
    """One list of k intervals inside [lo, hi)."""
    if k == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    span = hi - lo
    assert span >= 2 * k
    if span <= 8 * k:
        v = np.sort(rng.choice(span, size=2 * k, replace=False)) + lo
    else:
        v = np.unique(rng.integers(lo, hi, size=2 * k + 16, dtype=np.int64))
        while len(v) < 2 * k:
            v = np.unique(np.concatenate([v, rng.integers(lo, hi, size=2 * k, dtype=np.int64)]))
        v = np.sort(rng.choice(v, size=2 * k, replace=False))
    v = v.astype(np.uint32)
    return v[0::2].copy(), v[1::2].copy()


def complement_list(start: np.ndarray, end: np.ndarray):
    """Gaps between consecutive intervals: touches the list everywhere, overlaps nowhere."""
    return end[:-1].copy(), start[1:].copy()


def sub_lists(rng: np.random.Generator, start: np.ndarray, end: np.ndarray, p: float = 0.5):
    """A list inside (start, end): each interval is kept with probability p,
    shrunk to a random non-empty sub-interval.  Used as an F-list for the
    A-list (start, end)."""
    start = np.asarray(start, dtype=np.int64)
    end = np.asarray(end, dtype=np.int64)
    keep = rng.random(len(start)) < p
    s0, e0 = start[keep], end[keep]
    a = s0 + (rng.random(len(s0)) * (e0 - s0)).astype(np.int64)
    b = a + 1 + (rng.random(len(s0)) * (e0 - a)).astype(np.int64)
    b = np.minimum(b, e0)
    return a.astype(np.uint32), b.astype(np.uint32)


def fragmented_sub_lists(rng: np.random.Generator, start: np.ndarray, end: np.ndarray, max_parts: int):
    """A list inside (start, end) with up to `max_parts` intervals inside each
    interval (so it can be much longer than the list it lies in): 2q distinct
    sorted points in [s, e] give q non-touching sub-intervals of [s, e)."""
    out_s, out_e = [], []
    for s, e in zip(np.asarray(start, np.int64), np.asarray(end, np.int64)):
        q = int(rng.integers(0, max_parts + 1))
        q = min(q, int(e - s + 1) // 2)
        if q == 0:
            continue
        v = np.sort(rng.choice(int(e - s + 1), size=2 * q, replace=False)) + s
        out_s.append(v[0::2])
        out_e.append(v[1::2])
    if not out_s:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    return np.concatenate(out_s).astype(np.uint32), np.concatenate(out_e).astype(np.uint32)
