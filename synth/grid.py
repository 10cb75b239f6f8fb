"""The square data space and its 2^N x 2^N raster grid, chosen for a workload.

The grid is an input of the filter (both collections of a join must use the
same one), so it is drawn here with the polygons.  It is described in
lattice units (multiples of 2^-30):

    origin (x0, y0)   lattice multiples
    cell side w       a positive integer number of lattice units
    side              w * 2^order lattice units

grid_covering() leaves a guard of at least one full cell plus a margin on
every side of the polygons' bounding box, so no polygon reaches the outer
ring of cells (this keeps the last Hilbert cell unused and every half-open
interval end below 2^32 at order 16).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .polygons import LATTICE, PolygonSet


@dataclass(frozen=True)
class Grid:
    x0: float      # origin, a multiple of 2^-30
    y0: float
    side: float    # side of the square data space; side*2^30 is divisible by 2^order
    order: int     # N: the grid has 2^N cells per side

    @property
    def cell_lattice(self) -> int:
        """Cell side in lattice units (an exact integer)."""
        w = self.side * 2.0 ** 30 / 2.0 ** self.order
        assert w == int(w) and w >= 1
        return int(w)

    def as_tuple(self):
        return (self.x0, self.y0, self.side, self.order)


def grid_covering(sets, order: int) -> Grid:
    """Smallest-cell grid of the given order whose interior ring holds every polygon.

    With E the larger side of the joint bounding box in lattice units, the cell
    side is w = floor(E / (2^order - 4)) + 1 and the origin sits 2w below and
    left of the box, so every vertex coordinate lies in [2w, (2^order - 2) w)
    lattice units from the origin: no polygon touches cell row or column 0
    or 2^order - 1.
    """
    if isinstance(sets, PolygonSet):
        sets = [sets]
    lo = np.array([np.inf, np.inf])
    hi = np.array([-np.inf, -np.inf])
    for s in sets:
        if len(s.xy):
            lo = np.minimum(lo, s.xy.min(axis=0))
            hi = np.maximum(hi, s.xy.max(axis=0))
    loL = np.round(lo / LATTICE).astype(np.int64)
    hiL = np.round(hi / LATTICE).astype(np.int64)
    E = int(max(hiL[0] - loL[0], hiL[1] - loL[1]))
    w = E // ((1 << order) - 4) + 1
    x0L = int(loL[0]) - 2 * w
    y0L = int(loL[1]) - 2 * w
    return Grid(x0L * LATTICE, y0L * LATTICE, float(w * (1 << order)) * LATTICE, order)
