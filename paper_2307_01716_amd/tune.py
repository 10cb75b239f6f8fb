"""Autotuner of the batched schedule.

Sweeps the batched schedule's knobs on a workload that is already resident
on the device -- LDS tile per wavefront, streamed chunk per lane, the length above which
streamed lists are range-searched first, the lane-per-pair threshold and the
resident wavefronts per SIMD -- timing each setting with HIP events, and
returns the fastest.  Results can be written to
a JSON table keyed by device and a workload signature, and read back by
callers that want to skip the sweep.
"""

from __future__ import annotations

import itertools
import json
import os

import numpy as np

from . import april

GRID = {
    "tile": (128, 256, 512),
    "chunk": (1, 2),
    "search_min": (512, 4096),
    "thread_max": (8,),
    "waves_per_simd": (0, 4, 6),
}


def _call_cfg(cfg: dict) -> dict:
    """Knobs as april_filter_pairs takes them: waves per SIMD (0 = as many as
    fit) becomes a count of resident wavefronts."""
    out = {k: v for k, v in cfg.items() if k != "waves_per_simd"}
    wps = cfg.get("waves_per_simd", 0)
    if wps:
        out["waves"] = wps * 4 * april.april_device_info()["compute_units"]
    return out


def signature(n_pairs: int, lists_r, lists_s) -> str:
    ir, is_ = lists_r.info(), lists_s.info()
    return f"P{n_pairs}-R{ir.n_objects}x{ir.n_a}x{ir.n_f}-S{is_.n_objects}x{is_.n_a}x{is_.n_f}"


def time_config(dR, dS, r, s, verdict, counts, workspace, reps=3, **cfg) -> float:
    import torch

    stream = torch.cuda.current_stream()

    kw = _call_cfg(cfg)

    def run():
        april.april_filter_pairs(dR, dS, r, s, verdict, counts, schedule=april.SCHED_BATCHED,
                                 workspace=workspace, stream=stream, **kw)

    run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def sweep(dR, dS, r, s, verdict, counts, workspace, grid=None, reps=3, log=None):
    """Time every setting of `grid`; returns (best_cfg, best_ms, table)."""
    grid = grid or GRID
    keys = list(grid)
    table = []
    for vals in itertools.product(*[grid[k] for k in keys]):
        cfg = dict(zip(keys, vals))
        if cfg["thread_max"] >= cfg["tile"]:
            continue
        ms = time_config(dR, dS, r, s, verdict, counts, workspace, reps=reps, **cfg)
        table.append({**cfg, "ms": ms})
        if log:
            log(f"  tune {cfg} -> {ms:.3f} ms")
    best = min(table, key=lambda t: t["ms"])
    cfg = {k: best[k] for k in keys}
    return cfg, best["ms"], table


def call_config(cfg: dict) -> dict:
    """The keyword arguments of april_filter_pairs for a swept setting."""
    return _call_cfg(cfg)


def save(path: str, device: str, sig: str, cfg: dict, ms: float, table) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault(device, {})[sig] = {"config": cfg, "ms": ms, "sweep": table}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load(path: str, device: str, sig: str):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(device, {}).get(sig)
    return ent["config"] if ent else None
