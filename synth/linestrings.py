"""Seeded synthetic linestrings (roads, rivers) for polygon-linestring joins.

A linestring is a random walk of k vertices (k log-normal, median 12,
clamped to [2, 200]) from a start point drawn like the polygon centres of
the at-scale workload; each step has a uniform direction and a log-normal
length (median 3e-4).  Vertices are snapped to the 2^-30 lattice and kept
inside a given box.  Stored like polygons (xy, voff) but open: the last
vertex does not connect back to the first.
"""

from __future__ import annotations

import numpy as np

from .polygons import LATTICE, PolygonSet, snap


def random_walks(rng: np.random.Generator, starts: np.ndarray, lo, hi) -> PolygonSet:
    n = len(starts)
    k = np.clip(np.round(np.exp(np.log(12.0) + 0.8 * rng.standard_normal(n))), 2, 200).astype(np.int64)
    voff = np.zeros(n + 1, np.int64)
    np.cumsum(k, out=voff[1:])
    seg = np.repeat(np.arange(n), k)
    first = np.zeros(int(voff[-1]), bool)
    first[voff[:-1]] = True
    ang = rng.uniform(0, 2 * np.pi, len(seg))
    step = np.exp(np.log(3e-4) + 0.7 * rng.standard_normal(len(seg)))
    d = np.stack([np.cos(ang) * step, np.sin(ang) * step], axis=1)
    d[first] = 0.0
    # cumulative sum within each linestring
    c = np.cumsum(d, axis=0)
    base = c[voff[:-1]][seg]
    xy = starts[seg] + (c - base)
    xy = np.clip(xy, np.asarray(lo) + LATTICE, np.asarray(hi) - LATTICE)
    return PolygonSet(snap(xy), voff)
