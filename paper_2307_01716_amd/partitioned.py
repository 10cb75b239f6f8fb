"""Partitioned joins (Sec. 5.2): partition-local lists and candidate pairs.

Given a partition layout (every object has one instance per partition it
meets, every partition its own grid), this builds one collection of
instances per side with april_build_lists_partitioned and the candidate
pairs of every partition with april_mbr_join, keeping a pair only in the
partition that holds the lower-left corner of the two MBRs' intersection, so
every globally intersecting MBR pair is filtered exactly once.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import april


def build_instances(layout, polys, side: str, flags=april.STRICT) -> april.Lists:
    obj = layout.r_obj if side == "r" else layout.s_obj
    part = layout.r_part() if side == "r" else layout.s_part()
    inst = polys.subset(obj)
    grids = (april.april_grid_t * len(layout.grids))(*[april._grid(g) for g in layout.grids])
    xy = np.ascontiguousarray(inst.xy, np.float64)
    vo = np.ascontiguousarray(inst.voff, np.uint64)
    gof = np.ascontiguousarray(part, np.uint32)
    h = C.c_void_p()
    april._check(april.lib().april_build_lists_partitioned(
        grids, len(layout.grids), april._np(gof), april._np(xy), april._np(vo), len(vo) - 1, flags,
        C.byref(h)))
    return april.Lists(h.value)


def pairs(layout, R, S, with_all_count: bool = False):
    """Partition-local candidate pairs as instance indices (r_inst, s_inst);
    with `with_all_count` also the number of partition-local MBR pairs
    before the reference-point rule (each global pair once per partition
    both MBRs meet)."""
    mR, mS = R.mbrs(), S.mbrs()
    out_r, out_s = [], []
    n_all = 0
    for p in range(layout.k * layout.k):
        r0, r1 = int(layout.r_off[p]), int(layout.r_off[p + 1])
        s0, s1 = int(layout.s_off[p]), int(layout.s_off[p + 1])
        if r1 == r0 or s1 == s0:
            continue
        br, bs = mR[layout.r_obj[r0:r1]], mS[layout.s_obj[s0:s1]]
        i, j = april.april_mbr_join(br, bs)
        n_all += len(i)
        # reference point: lower-left corner of the MBR intersection
        keep = layout.part_of_point(np.maximum(br[i, 0], bs[j, 0]), np.maximum(br[i, 1], bs[j, 1])) == p
        out_r.append(i[keep].astype(np.uint64) + r0)
        out_s.append(j[keep].astype(np.uint64) + s0)
    r = np.concatenate(out_r).astype(np.uint32) if out_r else np.zeros(0, np.uint32)
    s = np.concatenate(out_s).astype(np.uint32) if out_s else np.zeros(0, np.uint32)
    return (r, s, n_all) if with_all_count else (r, s)
