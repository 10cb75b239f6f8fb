"""Space partitioning of a workload into k x k disjoint partitions (input).

The unit square is cut into k x k half-open partitions [i/k, (i+1)/k) x
[j/k, (j+1)/k) (indices clamped to 0..k-1 for coordinates outside it).  Each
object has one instance in every partition its closed MBR meets; instances
are grouped by partition.  Every partition gets its own grid of the given
order over the bounding box of its instances (both collections), drawn as
for a whole workload (`grid_covering`).  This module only describes the
layout; pair generation and list construction happen elsewhere.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .grid import Grid
from .polygons import LATTICE, PolygonSet


@dataclass
class Layout:
    k: int
    grids: list                 # k*k Grid objects (partition p = j*k + i)
    r_obj: np.ndarray           # R instance -> object id, grouped by partition
    r_off: np.ndarray           # k*k + 1 offsets of each partition's R instances
    s_obj: np.ndarray
    s_off: np.ndarray

    def part_of_point(self, x, y):
        i = np.clip(np.floor(np.asarray(x) * self.k), 0, self.k - 1).astype(np.int64)
        j = np.clip(np.floor(np.asarray(y) * self.k), 0, self.k - 1).astype(np.int64)
        return j * self.k + i

    def r_part(self):
        return np.repeat(np.arange(self.k * self.k), np.diff(self.r_off))

    def s_part(self):
        return np.repeat(np.arange(self.k * self.k), np.diff(self.s_off))


def _instances(mbrs: np.ndarray, k: int):
    i0 = np.clip(np.floor(mbrs[:, 0] * k), 0, k - 1).astype(np.int64)
    j0 = np.clip(np.floor(mbrs[:, 1] * k), 0, k - 1).astype(np.int64)
    i1 = np.clip(np.floor(mbrs[:, 2] * k), 0, k - 1).astype(np.int64)
    j1 = np.clip(np.floor(mbrs[:, 3] * k), 0, k - 1).astype(np.int64)
    ni, nj = i1 - i0 + 1, j1 - j0 + 1
    cnt = ni * nj
    obj = np.repeat(np.arange(len(mbrs)), cnt)
    t = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    pi = i0[obj] + t % ni[obj]
    pj = j0[obj] + t // ni[obj]
    part = pj * k + pi
    order = np.lexsort((obj, part))
    part, obj = part[order], obj[order]
    off = np.searchsorted(part, np.arange(k * k + 1))
    return obj, off


def _grid_for_boxes(lo, hi, order):
    """Grid of `order` around the lattice box [lo, hi], as synth.grid_covering."""
    loL = np.round(np.asarray(lo) / LATTICE).astype(np.int64)
    hiL = np.round(np.asarray(hi) / LATTICE).astype(np.int64)
    E = int(max(hiL[0] - loL[0], hiL[1] - loL[1]))
    w = E // ((1 << order) - 4) + 1
    return Grid((int(loL[0]) - 2 * w) * LATTICE, (int(loL[1]) - 2 * w) * LATTICE,
                float(w * (1 << order)) * LATTICE, order)


def layout(R: PolygonSet, S: PolygonSet, k: int = 16, order: int = 16) -> Layout:
    mR, mS = R.mbrs(), S.mbrs()
    r_obj, r_off = _instances(mR, k)
    s_obj, s_off = _instances(mS, k)
    grids = []
    for p in range(k * k):
        boxes = np.concatenate([mR[r_obj[r_off[p]:r_off[p + 1]]], mS[s_obj[s_off[p]:s_off[p + 1]]]])
        if len(boxes) == 0:
            grids.append(Grid(0.0, 0.0, float(1 << order) * LATTICE, order))
            continue
        grids.append(_grid_for_boxes(boxes[:, :2].min(axis=0), boxes[:, 2:].max(axis=0), order))
    return Layout(k, grids, r_obj, r_off, s_obj, s_off)
