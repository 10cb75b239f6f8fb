"""Autotuner of the batched schedule.

Sweeps the batched schedule's knobs on a workload that is already resident
on the device, timing each setting with HIP events:
  tile             intervals per list in a wavefront's LDS tile;
  chunk            streamed intervals per lane per step;
  waves_per_simd   resident wavefronts per SIMD (0 = as many as fit);
  thread_max       the lane bin: pairs whose four lists all hold at most
                   this many intervals run one lane per pair;
  wg_min           the workgroup bin: pairs in which neither object fits a
                   tile and the shorter one spans at least wg_min intervals
                   run on a whole workgroup (0xFFFFFFFF: no workgroup bin);
  search_min       streamed lists longer than this are range-searched first.
The sweep is coordinate-wise: tile x chunk x waves together (they trade LDS
for residency), then each bin threshold, then the search threshold, each
stage keeping the best setting so far.  The winner is stored in a JSON table
keyed by device (name and compute units) and a workload signature (pair
count and list totals), so that callers can skip the sweep next time.
"""

from __future__ import annotations

import itertools
import json
import os

import numpy as np

from . import april

NO_WG = 0xFFFFFFFF

# stage 1 together, then one knob at a time; 0 = the library's default
STAGES = [
    {"tile": (128, 256, 512), "chunk": (1, 2, 4), "waves_per_simd": (0, 4, 6)},
    {"thread_max": (0, 4, 16)},
    {"wg_min": (0, 1, NO_WG)},   # default 4 tiles; every pair that fits no tile; none
    {"search_min": (0, 4096)},
]

# default table next to this module (device -> signature -> setting)
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x.json")


def _call_cfg(cfg: dict) -> dict:
    """Knobs as april_filter_pairs takes them: waves per SIMD (0 = as many as
    fit) becomes a count of resident wavefronts."""
    out = {k: v for k, v in cfg.items() if k != "waves_per_simd" and v}
    wps = cfg.get("waves_per_simd", 0)
    if wps:
        out["waves"] = wps * 4 * april.april_device_info()["compute_units"]
    return out


def device_key() -> str:
    d = april.april_device_info()
    return f"{d['arch'].split(':')[0]}-{d['compute_units']}cu"


def signature(n_pairs: int, lists_r, lists_s) -> str:
    """Pair count and list totals, rounded to 2 significant digits: the same
    workload regenerated, or one close to it, maps to the same entry."""
    ir, is_ = lists_r.info(), lists_s.info()

    def r2(x):
        x = int(x)
        if x < 100:
            return str(x)
        e = len(str(x)) - 2
        return f"{round(x / 10 ** e)}e{e}"
    return (f"P{r2(n_pairs)}-R{r2(ir.n_objects)}x{r2(ir.n_a)}x{r2(ir.n_f)}"
            f"-S{r2(is_.n_objects)}x{r2(is_.n_a)}x{r2(is_.n_f)}")


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


def _valid(cfg: dict) -> bool:
    tile = cfg.get("tile") or 256
    return (cfg.get("thread_max") or 8) < tile


def sweep(dR, dS, r, s, verdict, counts, workspace, stages=None, reps=3, log=None):
    """Coordinate-wise sweep; returns (best_cfg, best_ms, table of every
    timed setting)."""
    stages = stages or STAGES
    best = {k: 0 for st in stages for k in st}
    best_ms = None
    table = []
    for st in stages:
        keys = list(st)
        for vals in itertools.product(*[st[k] for k in keys]):
            cfg = {**best, **dict(zip(keys, vals))}
            if not _valid(cfg):
                continue
            ms = time_config(dR, dS, r, s, verdict, counts, workspace, reps=reps, **cfg)
            table.append({**cfg, "ms": ms})
            if log:
                log(f"  tune {cfg} -> {ms:.3f} ms")
            if best_ms is None or ms < best_ms:
                best, best_ms = cfg, ms
    return best, best_ms, table


def call_config(cfg: dict) -> dict:
    """The keyword arguments of april_filter_pairs for a swept setting."""
    return _call_cfg(cfg)


def save(path: str, device: str, sig: str, cfg: dict, ms: float, table=None) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    ent = {"config": cfg, "ms": round(ms, 4)}
    if table is not None:
        ent["settings_timed"] = len(table)
    data.setdefault(device, {})[sig] = ent
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)


def load(path: str, device: str, sig: str):
    """The stored setting for (device, signature), or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(device, {}).get(sig)
    return dict(ent["config"]) if ent else None
