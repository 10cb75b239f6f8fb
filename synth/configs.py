"""Recipes of the five synthetic workloads.

Each recipe is seeded and returns polygon collections R and S (and for the
served workload, a query stream) with the shapes the paper's real datasets
have: simple polygons without holes, tens of vertices for most objects and a
heavy tail of complex ones.  Seeds: R = 1000k+1, S = 1000k+2, queries =
1000k+3, shared mixture parameters = 1000k, for workload k = 1..5.
"""

from __future__ import annotations

import numpy as np

from .grid import Grid, grid_covering
from .polygons import LATTICE, PolygonSet, star_polygons


def tiny(k: int = 1, n: int = 1000):
    """|R| = |S| = n polygons, 8-64 vertices, centres uniform in [0,1)^2,
    radii uniform in [0.002, 0.02], grid order 10."""
    out = []
    for side in (1, 2):
        rng = np.random.default_rng(1000 * k + side)
        centres = rng.random((n, 2))
        radii = rng.uniform(0.002, 0.02, size=n)
        nv = rng.integers(8, 65, size=n)
        out.append(star_polygons(rng, centres, radii, nv, a=0.3))
    R, S = out
    return R, S, grid_covering([R, S], 10)


# mixture spread chosen so that the MBR join of two 200k collections yields
# about 5 million candidate pairs
SCALE_SIGMA = (0.012, 0.03)


def _mixture_rng(k):
    return np.random.default_rng(1000 * k)


def scale_collection(rng, n, mixture_seed_k, sigma=SCALE_SIGMA):
    """n polygons of the at-scale distribution: vertex count log-normal
    (median 30, clamped to [8, 5000]), centres from a shared 64-component
    Gaussian mixture, radius log-normal (median 0.001, clamped to
    [2e-4, 0.02])."""
    # the mixture (means, spreads, weights) is common to R and S
    mrng = _mixture_rng(mixture_seed_k)
    centres = gmm_centres_shared(mrng, rng, n, sigma)
    radii = np.clip(np.exp(np.log(0.001) + 0.6 * rng.standard_normal(n)), 2e-4, 0.02)
    nv = np.clip(np.round(np.exp(np.log(30.0) + 0.7 * rng.standard_normal(n))), 8, 5000).astype(np.int64)
    return star_polygons(rng, centres, radii, nv, a=0.3)


def gmm_centres_shared(mrng, rng, n, sigma, k=64, lo=0.05, hi=0.95):
    """Centres from a mixture whose parameters come from `mrng` (shared by
    both collections) and whose draws come from `rng`."""
    means = mrng.uniform(lo, hi, size=(k, 2))
    sig = mrng.uniform(sigma[0], sigma[1], size=k)
    w = mrng.uniform(0.5, 1.5, size=k)
    w = w / w.sum()
    out = np.empty((n, 2))
    todo = np.arange(n)
    while len(todo):
        comp = rng.choice(k, size=len(todo), p=w)
        pts = means[comp] + sig[comp, None] * rng.standard_normal((len(todo), 2))
        ok = np.all((pts >= 0.0) & (pts < 1.0), axis=1)
        out[todo[ok]] = pts[ok]
        todo = todo[~ok]
    return out


def scale(k: int = 2, n: int = 200_000, order: int = 16):
    """The at-scale workload: two collections of n polygons, grid order 16."""
    R = scale_collection(np.random.default_rng(1000 * k + 1), n, k)
    S = scale_collection(np.random.default_rng(1000 * k + 2), n, k)
    return R, S, grid_covering([R, S], order)


def large_collection(rng, n, mixture_seed_k, a=0.02):
    """n complex polygons: 20k-100k vertices, radius uniform in [0.02, 0.1]."""
    mrng = _mixture_rng(mixture_seed_k)
    centres = gmm_centres_shared(mrng, rng, n, SCALE_SIGMA)
    radii = rng.uniform(0.02, 0.1, size=n)
    nv = rng.integers(20_000, 100_001, size=n)
    return star_polygons(rng, centres, radii, nv, a=a)


def skewed(k: int = 3, n: int = 200_000, n_large: int = 2000, a_large: float = 0.02,
           order: int = 16):
    """The skewed workload: the at-scale collections plus n_large complex
    polygons on each side (appended after the small ones)."""
    out = []
    for side in (1, 2):
        rng = np.random.default_rng(1000 * k + side)
        small = scale_collection(rng, n, k)
        big = large_collection(rng, n_large, k, a=a_large)
        out.append(PolygonSet.concat(small, big))
    R, S = out
    return R, S, grid_covering([R, S], order)


def serving(k: int = 5, n_s: int = 1_000_000, n_queries: int = 10_000, order: int = 16):
    """The served workload: S of n_s at-scale polygons, and a stream of query
    polygons with 10..10^4 vertices (log-uniform), radius 5e-4..0.05
    (log-uniform), centres from S's mixture.  Returns (S, queries, grid);
    the grid covers S and the queries."""
    S = scale_collection(np.random.default_rng(1000 * k + 2), n_s, k)
    Q = query_stream(k, n_queries)
    return S, Q, grid_covering([S, Q], order)


def query_stream(k: int, n: int, r_range=(5e-4, 0.05), v_range=(10, 10_000)):
    rng = np.random.default_rng(1000 * k + 3)
    mrng = _mixture_rng(k)
    centres = gmm_centres_shared(mrng, rng, n, SCALE_SIGMA)
    radii = np.exp(rng.uniform(np.log(r_range[0]), np.log(r_range[1]), n))
    nv = np.round(np.exp(rng.uniform(np.log(v_range[0]), np.log(v_range[1]), n))).astype(np.int64)
    return star_polygons(rng, centres, radii, nv, a=0.3)


def partitioned(k: int = 4, n: int = 500_000, parts: int = 16, order: int = 16):
    """The partitioned workload: two at-scale collections of n polygons, the
    unit square cut into parts x parts partitions with a grid of `order` each."""
    from .partitions import layout
    R = scale_collection(np.random.default_rng(1000 * k + 1), n, k)
    S = scale_collection(np.random.default_rng(1000 * k + 2), n, k)
    return R, S, layout(R, S, parts, order)


def linestring_scale(k: int = 6, n_poly: int = 200_000, n_lines: int = 200_000, order: int = 16):
    """Polygon-linestring workload: the at-scale polygon collection and
    n_lines random-walk linestrings starting like the polygon centres."""
    from .linestrings import random_walks
    P = scale_collection(np.random.default_rng(1000 * k + 1), n_poly, 2)
    rng = np.random.default_rng(1000 * k + 2)
    starts = gmm_centres_shared(_mixture_rng(2), rng, n_lines, SCALE_SIGMA)
    lo, hi = P.xy.min(axis=0), P.xy.max(axis=0)
    L = random_walks(rng, starts, lo, hi)
    return P, L, grid_covering([P, L], order)


def two_orders(R, S, fine: int = 16, coarse: int = 14):
    """One data space at two grid orders: a coarse grid over both sets
    (guard ring of two coarse cells, cell side divisible by 2^(fine-coarse))
    and the fine grid with the same origin and side."""
    lo = np.round(np.minimum(R.xy.min(0), S.xy.min(0)) / LATTICE).astype(np.int64)
    hi = np.round(np.maximum(R.xy.max(0), S.xy.max(0)) / LATTICE).astype(np.int64)
    q = 1 << (fine - coarse)
    w = (int((hi - lo).max()) // ((1 << coarse) - 4) + 1 + q - 1) // q * q
    x0, y0 = (lo - 2 * w) * LATTICE
    gc = Grid(float(x0), float(y0), float(w * (1 << coarse)) * LATTICE, coarse)
    return Grid(gc.x0, gc.y0, gc.side, fine), gc
