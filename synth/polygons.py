"""Random simple star-shaped polygons on the 2^-30 lattice.

A polygon with centre c, radius r and n vertices takes vertex m at angle
    theta_m = 2*pi*(m + 0.5 + 0.8*(U_m - 0.5)) / n      (strictly increasing)
and distance rho_m = r*(1 - a*V_m) from c, with U, V uniform on [0,1).
Every coordinate is then rounded to a multiple of 2^-30, so every later
geometric predicate can be evaluated exactly in integers.  A polygon is kept
only if every triangle (c, v_m, v_{m+1}) is strictly counter-clockwise in
exact integer arithmetic; that makes it simple and star-shaped about c.
Polygons that fail are redrawn (this never happens for the sizes used here).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LATTICE = 2.0 ** -30  # coordinate quantum of every generated vertex


def snap(v: np.ndarray) -> np.ndarray:
    """Round to the nearest multiple of 2^-30 (exactly representable)."""
    return np.round(np.asarray(v, dtype=np.float64) * 2.0 ** 30) * LATTICE


@dataclass
class PolygonSet:
    """A collection of polygons in CSR form.

    xy    float64 [V, 2]  vertices, counter-clockwise, no closing duplicate
    voff  int64   [n+1]   polygon k owns xy[voff[k]:voff[k+1]]
    """

    xy: np.ndarray
    voff: np.ndarray

    def __len__(self) -> int:
        return len(self.voff) - 1

    def polygon(self, k: int) -> np.ndarray:
        return self.xy[self.voff[k]:self.voff[k + 1]]

    def mbrs(self) -> np.ndarray:
        """[n, 4] (xmin, ymin, xmax, ymax) of every polygon."""
        out = np.empty((len(self), 4))
        starts = self.voff[:-1]
        out[:, 0] = np.minimum.reduceat(self.xy[:, 0], starts)
        out[:, 1] = np.minimum.reduceat(self.xy[:, 1], starts)
        out[:, 2] = np.maximum.reduceat(self.xy[:, 0], starts)
        out[:, 3] = np.maximum.reduceat(self.xy[:, 1], starts)
        return out

    def subset(self, ids) -> "PolygonSet":
        ids = np.asarray(ids, dtype=np.int64)
        lens = np.diff(self.voff)[ids]
        voff = np.zeros(len(ids) + 1, dtype=np.int64)
        np.cumsum(lens, out=voff[1:])
        take = np.concatenate([np.arange(self.voff[k], self.voff[k + 1]) for k in ids]) \
            if len(ids) else np.zeros(0, dtype=np.int64)
        return PolygonSet(np.ascontiguousarray(self.xy[take]), voff)

    @staticmethod
    def concat(a: "PolygonSet", b: "PolygonSet") -> "PolygonSet":
        voff = np.concatenate([a.voff, b.voff[1:] + a.voff[-1]])
        return PolygonSet(np.concatenate([a.xy, b.xy]), voff)


def star_polygons(rng: np.random.Generator, centres: np.ndarray, radii: np.ndarray,
                  nverts: np.ndarray, a=0.3) -> PolygonSet:
    """Draw one star polygon per centre (see module docstring)."""
    centres = snap(np.asarray(centres, dtype=np.float64))
    radii = np.asarray(radii, dtype=np.float64)
    nverts = np.asarray(nverts, dtype=np.int64)
    n = len(nverts)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (n,))
    voff = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(nverts, out=voff[1:])
    V = int(voff[-1])
    xy = np.empty((V, 2), dtype=np.float64)
    todo = np.arange(n)
    for _attempt in range(20):
        if len(todo) == 0:
            break
        lens = nverts[todo]
        seg = np.repeat(np.arange(len(todo)), lens)
        base = np.repeat(voff[todo], lens)
        m = np.arange(len(seg)) - np.repeat(np.cumsum(lens) - lens, lens)
        U = rng.random(len(seg))
        Vr = rng.random(len(seg))
        nn = lens[seg].astype(np.float64)
        theta = 2.0 * np.pi * (m + 0.5 + 0.8 * (U - 0.5)) / nn
        rho = radii[todo][seg] * (1.0 - a[todo][seg] * Vr)
        cx = centres[todo, 0]
        cy = centres[todo, 1]
        x = snap(cx[seg] + rho * np.cos(theta))
        y = snap(cy[seg] + rho * np.sin(theta))
        # exact orientation of (c, v_m, v_{m+1}) with wrap-around; the
        # offsets from the centre are below 2^30 lattice units, so the
        # products stay below 2^62
        X = np.round((x - cx[seg]) * 2.0 ** 30).astype(np.int64)
        Y = np.round((y - cy[seg]) * 2.0 ** 30).astype(np.int64)
        nxt = np.arange(len(seg)) + 1
        ends = np.cumsum(lens) - 1
        nxt[ends] = ends - lens + 1
        cross = X * Y[nxt] - Y * X[nxt]
        bad_v = cross <= 0
        bad = np.zeros(len(todo), dtype=bool)
        np.logical_or.at(bad, seg[bad_v], True)
        good_v = ~bad[seg]
        xy[base[good_v] + m[good_v], 0] = x[good_v]
        xy[base[good_v] + m[good_v], 1] = y[good_v]
        todo = todo[bad]
    if len(todo):
        raise RuntimeError("could not draw simple star polygons for %d centres" % len(todo))
    return PolygonSet(xy, voff)
