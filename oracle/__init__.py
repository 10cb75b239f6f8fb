"""CPU oracle of the APRIL intermediate filter -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never calls it and shares no code with it.
The arithmetic lives in oracle.c (plain C, built with gcc); this module only
marshals numpy arrays in and out.

Functions (each follows the paper passage named in oracle.c):
    hilbert(order, x, y)              Hilbert position of cells (Sec. 3.2)
    classify(grid, poly)              per-cell Full/Partial/Empty (Sec. 4.1)
    build_lists(grid, polys)          A- and F-lists (Sec. 4.1)
    interval_join(X, Y)               IntervalJoin of Alg. 2
    filter_pairs(LR, LS, r, s)        Alg. 2 verdicts + bytes moved per pair
    mbr_join(R, S)                    candidate pairs (closed MBRs meet)
    polygons_intersect(a, b)          exact closed-polygon intersection
    twice_area(poly)                  exact shoelace area x2 (lattice units^2)
    filter_within(LR, LS, r, s)       within-join filter (Sec. 4.3.2)
    build_cells(grid, lines)          linestring cell lists (Sec. 4.3.3)
    filter_linestrings(LP, CL, p, l)  polygon-linestring filter (Sec. 4.3.3)
    filter_mixed(LR, NR, LS, NS, r, s) Alg. 2 across grid orders (Sec. 5.3)
    point_in_closed_polygon, linestring_meets_polygon   exact geometry

Parity is pinned for every function by tests/test_oracle_*.py against
closed forms, brute force and invariants; see those files.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TN, TH, IND = 0, 1, 2
EMPTY, PARTIAL, FULL = 0, 1, 2


def build() -> str:
    """Compile oracle.c into liboracle.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC", "-pthread",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    L = C.CDLL(_LIB)
    P = C.c_void_p
    i64, u64, i32, d = C.c_int64, C.c_uint64, C.c_int, C.c_double
    L.orc_hilbert.restype = u64
    L.orc_hilbert.argtypes = [i32, u64, u64]
    L.orc_hilbert_many.argtypes = [i32, P, P, i64, P]
    L.orc_classify.argtypes = [d, d, d, i32, P, i64, C.POINTER(P), C.POINTER(i64)]
    L.orc_classify_cells.argtypes = [d, d, d, i32, P, i64, P, i64, P]
    L.orc_free.argtypes = [P]
    L.orc_build.argtypes = [d, d, d, i32, P, P, i64, i32, C.POINTER(P)]
    L.orc_lists_sizes.argtypes = [P, C.POINTER(i64), C.POINTER(i64)]
    L.orc_lists_export.argtypes = [P] * 7
    L.orc_lists_free.argtypes = [P]
    L.orc_interval_join.argtypes = [P, P, u64, P, P, u64, C.POINTER(u64), C.POINTER(u64)]
    L.orc_filter.argtypes = [P] * 14 + [i64, P, P, i32]
    L.orc_mbr_join.argtypes = [P, P, i64, P, P, i64, i32, C.POINTER(P), C.POINTER(i64)]
    L.orc_pairs_export.argtypes = [P, P, P]
    L.orc_pairs_free.argtypes = [P]
    L.orc_polygons_intersect.argtypes = [P, i64, P, i64]
    L.orc_twice_area.argtypes = [P, i64, C.POINTER(i64), C.POINTER(u64)]
    L.orc_filter_within.argtypes = [P] * 11 + [i64, P]
    L.orc_build_cells.argtypes = [d, d, d, i32, P, P, i64, C.POINTER(P)]
    L.orc_cells_size.restype = i64
    L.orc_cells_size.argtypes = [P]
    L.orc_cells_export.argtypes = [P, P, P]
    L.orc_cells_free.argtypes = [P]
    L.orc_filter_linestrings.argtypes = [P] * 10 + [i64, P]
    L.orc_filter_mixed.argtypes = [P] * 6 + [i32] + [P] * 6 + [i32, P, P, i64, P]
    L.orc_point_in_closed_polygon.argtypes = [P, i64, d, d]
    L.orc_linestring_meets_polygon.argtypes = [P, i64, P, i64]
    _lib = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc < 0:
        raise OracleError({-1: "invalid input", -2: "outside the grid / guard ring",
                           -3: "out of memory"}.get(rc, str(rc)))
    return rc


def _grid_args(grid):
    x0, y0, side, order = grid.as_tuple() if hasattr(grid, "as_tuple") else grid
    return float(x0), float(y0), float(side), int(order)


def default_threads() -> int:
    """Host threads for the oracle's parallel loops: the CPUs this process
    may run on, at most 16 (a GPU host's share per GPU)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def hilbert(order: int, x, y) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint64).ravel())
    y = np.ascontiguousarray(np.asarray(y, dtype=np.uint64).ravel())
    out = np.empty(len(x), dtype=np.uint64)
    _load().orc_hilbert_many(order, _p(x), _p(y), len(x), _p(out))
    return out


def classify(grid, xy: np.ndarray) -> np.ndarray:
    """[k, 3] int64 rows (i, j, class) over the polygon's cell window."""
    L = _load()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    ptr = C.c_void_p()
    n = C.c_int64()
    _check(L.orc_classify(*_grid_args(grid), _p(xy), len(xy), C.byref(ptr), C.byref(n)))
    try:
        buf = (C.c_int64 * (3 * n.value)).from_address(ptr.value) if n.value else []
        out = np.array(buf, dtype=np.int64).reshape(-1, 3)
    finally:
        L.orc_free(ptr)
    return out


def classify_cells(grid, xy: np.ndarray, ij: np.ndarray) -> np.ndarray:
    """Classes (0 Empty, 1 Partial, 2 Full) of the given cells, rows of ij =
    (i, j), each decided by brute force over all of the polygon's edges."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    ij = np.ascontiguousarray(ij, dtype=np.int64).reshape(-1, 2)
    out = np.empty(len(ij), dtype=np.uint8)
    _check(_load().orc_classify_cells(*_grid_args(grid), _p(xy), len(xy), _p(ij), len(ij), _p(out)))
    return out


@dataclass
class Lists:
    """A- and F-lists of a collection: CSR offsets + SoA uint32 endpoints."""

    offA: np.ndarray
    sA: np.ndarray
    eA: np.ndarray
    offF: np.ndarray
    sF: np.ndarray
    eF: np.ndarray

    def __len__(self):
        return len(self.offA) - 1

    def A(self, k):
        a, b = int(self.offA[k]), int(self.offA[k + 1])
        return self.sA[a:b], self.eA[a:b]

    def F(self, k):
        a, b = int(self.offF[k]), int(self.offF[k + 1])
        return self.sF[a:b], self.eF[a:b]


def build_lists(grid, polys, nthreads: int = 0) -> Lists:
    L = _load()
    xy = np.ascontiguousarray(polys.xy, dtype=np.float64)
    voff = np.ascontiguousarray(polys.voff, dtype=np.int64)
    n = len(voff) - 1
    h = C.c_void_p()
    _check(L.orc_build(*_grid_args(grid), _p(xy), _p(voff), n, nthreads or default_threads(),
                       C.byref(h)))
    try:
        na, nf = C.c_int64(), C.c_int64()
        L.orc_lists_sizes(h, C.byref(na), C.byref(nf))
        out = Lists(np.empty(n + 1, np.uint64), np.empty(na.value, np.uint32),
                    np.empty(na.value, np.uint32), np.empty(n + 1, np.uint64),
                    np.empty(nf.value, np.uint32), np.empty(nf.value, np.uint32))
        L.orc_lists_export(h, _p(out.offA), _p(out.sA), _p(out.eA), _p(out.offF),
                           _p(out.sF), _p(out.eF))
    finally:
        L.orc_lists_free(h)
    return out


def interval_join(X, Y):
    """(overlap?, elements of X read, elements of Y read) -- Alg. 2 IntervalJoin."""
    xs = np.ascontiguousarray(X[0], dtype=np.uint32)
    xe = np.ascontiguousarray(X[1], dtype=np.uint32)
    ys = np.ascontiguousarray(Y[0], dtype=np.uint32)
    ye = np.ascontiguousarray(Y[1], dtype=np.uint32)
    rx, ry = C.c_uint64(), C.c_uint64()
    hit = _load().orc_interval_join(_p(xs), _p(xe), len(xs), _p(ys), _p(ye), len(ys),
                                    C.byref(rx), C.byref(ry))
    return bool(hit), rx.value, ry.value


def filter_pairs(LR: Lists, LS: Lists, r, s, nthreads: int = 0, want_bytes=False):
    """Alg. 2 over candidate pairs; returns verdicts (uint8) [and bytes moved]."""
    r = np.ascontiguousarray(r, dtype=np.uint32)
    s = np.ascontiguousarray(s, dtype=np.uint32)
    assert len(r) == len(s)
    if len(r):
        assert int(r.max()) < len(LR) and int(s.max()) < len(LS)
    v = np.empty(len(r), np.uint8)
    b = np.empty(len(r), np.uint64) if want_bytes else None
    _load().orc_filter(_p(LR.offA), _p(LR.sA), _p(LR.eA), _p(LR.offF), _p(LR.sF), _p(LR.eF),
                       _p(LS.offA), _p(LS.sA), _p(LS.eA), _p(LS.offF), _p(LS.sF), _p(LS.eF),
                       _p(r), _p(s), len(r), _p(v), _p(b) if b is not None else None,
                       nthreads or default_threads())
    return (v, b) if want_bytes else v


def filter_pairs_timed(LR: Lists, LS: Lists, r, s, nthreads: int):
    """Like filter_pairs; returns (verdicts, threads used) for timing runs."""
    r = np.ascontiguousarray(r, dtype=np.uint32)
    s = np.ascontiguousarray(s, dtype=np.uint32)
    v = np.empty(len(r), np.uint8)
    used = _load().orc_filter(_p(LR.offA), _p(LR.sA), _p(LR.eA), _p(LR.offF), _p(LR.sF),
                              _p(LR.eF), _p(LS.offA), _p(LS.sA), _p(LS.eA), _p(LS.offF),
                              _p(LS.sF), _p(LS.eF), _p(r), _p(s), len(r), _p(v), None, nthreads)
    return v, used


def mbr_join(R, S, nthreads: int = 0):
    """All (r, s) with intersecting closed MBRs, sorted by (r, s)."""
    L = _load()
    xr = np.ascontiguousarray(R.xy, dtype=np.float64)
    xs = np.ascontiguousarray(S.xy, dtype=np.float64)
    vr = np.ascontiguousarray(R.voff, dtype=np.int64)
    vs = np.ascontiguousarray(S.voff, dtype=np.int64)
    h = C.c_void_p()
    n = C.c_int64()
    rc = L.orc_mbr_join(_p(xr), _p(vr), len(vr) - 1, _p(xs), _p(vs), len(vs) - 1,
                        nthreads or default_threads(), C.byref(h), C.byref(n))
    try:
        _check(rc)
        r = np.empty(n.value, np.uint32)
        s = np.empty(n.value, np.uint32)
        L.orc_pairs_export(h, _p(r), _p(s))
    finally:
        L.orc_pairs_free(h)
    return r, s


def polygons_intersect(a: np.ndarray, b: np.ndarray) -> bool:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return bool(_check(_load().orc_polygons_intersect(_p(a), len(a), _p(b), len(b))))


def twice_area(xy: np.ndarray) -> int:
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    hi, lo = C.c_int64(), C.c_uint64()
    _load().orc_twice_area(_p(xy), len(xy), C.byref(hi), C.byref(lo))
    return (hi.value << 64) + lo.value


def _partition_local_pairs(layout, R, S, p, nthreads):
    """Partition p's candidate pairs (Sec. 5.2) as local indices (i, j) into
    its R and S instances: MBR pairs of its instances kept only where the
    lower-left corner of the two MBRs' intersection lies in p."""
    k = layout.k
    ro = layout.r_obj[layout.r_off[p]:layout.r_off[p + 1]]
    so = layout.s_obj[layout.s_off[p]:layout.s_off[p + 1]]
    if len(ro) == 0 or len(so) == 0:
        return ro, so, None, None
    Rp, Sp = R.subset(ro), S.subset(so)
    i, j = mbr_join(Rp, Sp, nthreads)
    br, bs = Rp.mbrs()[i], Sp.mbrs()[j]
    cx = np.maximum(br[:, 0], bs[:, 0])
    cy = np.maximum(br[:, 1], bs[:, 1])
    pi = np.clip(np.floor(cx * k), 0, k - 1).astype(np.int64)
    pj = np.clip(np.floor(cy * k), 0, k - 1).astype(np.int64)
    keep = (pj * k + pi) == p
    return ro, so, i[keep], j[keep]


def partitioned_pairs(layout, R, S, nthreads: int = 0):
    """Partition-local candidate pairs of all partitions as instance indices
    (R instance layout.r_off[p] + i, S instance layout.s_off[p] + j), sorted."""
    out_r, out_s = [], []
    for p in range(layout.k * layout.k):
        ro, so, i, j = _partition_local_pairs(layout, R, S, p, nthreads)
        if i is None or len(i) == 0:
            continue
        out_r.append(i.astype(np.int64) + int(layout.r_off[p]))
        out_s.append(j.astype(np.int64) + int(layout.s_off[p]))
    if not out_r:
        z = np.zeros(0, np.int64)
        return z, z
    r, s = np.concatenate(out_r), np.concatenate(out_s)
    order = np.lexsort((s, r))
    return r[order], s[order]


def partitioned_filter(layout, R, S, nthreads: int = 0):
    """Partitioned join (Sec. 5.2), partition by partition: lists of each
    partition's instances on its own grid, the partition's MBR pairs kept only
    where the lower-left corner of the MBR intersection lies in it, Alg. 2 on
    them.  Returns (r, s, verdict) with global object ids, sorted by (r, s)."""
    out = []
    for p in range(layout.k * layout.k):
        ro, so, i, j = _partition_local_pairs(layout, R, S, p, nthreads)
        if i is None or len(i) == 0:
            continue
        Rp, Sp = R.subset(ro), S.subset(so)
        g = layout.grids[p]
        v = filter_pairs(build_lists(g, Rp, nthreads), build_lists(g, Sp, nthreads), i, j, nthreads)
        out.append((ro[i], so[j], v))
    if not out:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros(0, np.uint8)
    r = np.concatenate([o[0] for o in out])
    s = np.concatenate([o[1] for o in out])
    v = np.concatenate([o[2] for o in out])
    order = np.lexsort((s, r))
    return r[order], s[order], v[order]


# ------------------------------------------------ query variants (Sec. 4.3, 5.3)

def _pairs(r, s):
    r = np.ascontiguousarray(r, dtype=np.uint32)
    s = np.ascontiguousarray(s, dtype=np.uint32)
    assert len(r) == len(s)
    return r, s


def filter_within(LR: Lists, LS: Lists, r, s):
    """Within join filter (Sec. 4.3.2): is r within s?  0 TN, 1 TH, 2 IND."""
    r, s = _pairs(r, s)
    v = np.empty(len(r), np.uint8)
    _check(_load().orc_filter_within(_p(LR.offA), _p(LR.sA), _p(LR.eA), _p(LS.offA), _p(LS.sA), _p(LS.eA),
                                     _p(LS.offF), _p(LS.sF), _p(LS.eF), _p(r), _p(s), len(r), _p(v)))
    return v


@dataclass
class Cells:
    """Linestring approximations: per linestring the sorted cell ids."""
    off: np.ndarray
    ids: np.ndarray

    def __len__(self):
        return len(self.off) - 1

    def cells(self, k):
        return self.ids[int(self.off[k]):int(self.off[k + 1])]


def build_cells(grid, lines) -> Cells:
    """Cell lists of linestrings (Sec. 4.3.3); `lines` has .xy and .voff
    like a polygon set (vertices in order, not closed)."""
    L = _load()
    xy = np.ascontiguousarray(lines.xy, dtype=np.float64)
    voff = np.ascontiguousarray(lines.voff, dtype=np.int64)
    h = C.c_void_p()
    _check(L.orc_build_cells(*_grid_args(grid), _p(xy), _p(voff), len(voff) - 1, C.byref(h)))
    try:
        n = L.orc_cells_size(h)
        out = Cells(np.empty(len(voff), np.uint64), np.empty(n, np.uint32))
        L.orc_cells_export(h, _p(out.off), _p(out.ids))
    finally:
        L.orc_cells_free(h)
    return out


def filter_linestrings(LP: Lists, CL: Cells, p, l):
    """Polygon-linestring filter (Sec. 4.3.3).  0 TN, 1 TH, 2 IND."""
    p, l = _pairs(p, l)
    v = np.empty(len(p), np.uint8)
    _check(_load().orc_filter_linestrings(_p(LP.offA), _p(LP.sA), _p(LP.eA), _p(LP.offF), _p(LP.sF), _p(LP.eF),
                                          _p(CL.off), _p(CL.ids), _p(p), _p(l), len(p), _p(v)))
    return v


def filter_mixed(LR: Lists, NR: int, LS: Lists, NS: int, r, s):
    """Alg. 2 across grid orders NR and NS on one data space (Sec. 5.3)."""
    r, s = _pairs(r, s)
    v = np.empty(len(r), np.uint8)
    _check(_load().orc_filter_mixed(_p(LR.offA), _p(LR.sA), _p(LR.eA), _p(LR.offF), _p(LR.sF), _p(LR.eF), NR,
                                    _p(LS.offA), _p(LS.sA), _p(LS.eA), _p(LS.offF), _p(LS.sF), _p(LS.eF), NS,
                                    _p(r), _p(s), len(r), _p(v)))
    return v


def point_in_closed_polygon(poly: np.ndarray, x: float, y: float) -> bool:
    poly = np.ascontiguousarray(poly, dtype=np.float64)
    return bool(_check(_load().orc_point_in_closed_polygon(_p(poly), len(poly), float(x), float(y))))


def linestring_meets_polygon(line: np.ndarray, poly: np.ndarray) -> bool:
    line = np.ascontiguousarray(line, dtype=np.float64)
    poly = np.ascontiguousarray(poly, dtype=np.float64)
    return bool(_check(_load().orc_linestring_meets_polygon(_p(line), len(line), _p(poly), len(poly))))
