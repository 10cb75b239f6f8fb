"""Summaries of rocprofv3 output for the filter kernels.

Reads the CSV files that `rocprofv3 --kernel-trace --stats` and
`rocprofv3 --pmc ...` write, and turns them into short text summaries:

* kernel statistics (calls, average / min / max duration per kernel);
* per-dispatch counters of the filter kernels;
* VALU instructions per launch (SQ_INSTS_VALU), against the device's peak
  issue rate, keyed like the traffic records;
* HBM traffic per launch from FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
  each scaled by what the same counter reads for a device-to-device copy of
  known size (the copies `bench.py --copy-calibration` makes before its
  timed region), together with a digest of the kernel's sources and the
  launch configuration, so that a reader (bench.py) can tell whether the
  figure still describes the kernel it runs.

Command line:
    python -m paper_2307_01716_amd.profiling stats TRACE_DIR
    python -m paper_2307_01716_amd.profiling traffic --fetch DIR --write DIR \
        --kernel k_batched --config tile=512,chunk=2 --pairs N --alg-bytes B \
        --command "..." --out FILE
    python -m paper_2307_01716_amd.profiling valu --pmc DIR --kernel k_batched \
        --pairs N --command "..." --out FILE
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import OrderedDict

PKG = os.path.dirname(os.path.abspath(__file__))
# sources that define each kernel's code and its launch defaults
# (the batched schedule's defaults live in batched.hip, so a change to the
# plain kernel in filter.hip leaves the batched records valid)
KERNEL_SOURCES = {"k_batched": ["csrc/batched.hip", "csrc/device.hpp"],
                  "k_filter_plain": ["csrc/filter.hip", "csrc/device.hpp"],
                  "k_filter_vbyte": ["csrc/compressed.hip", "csrc/vbyte.hpp", "csrc/device.hpp"]}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
# Peak VALU issue rate of the device: 256 CUs x 4 SIMDs, each issuing one
# wave64 VALU instruction every 4 cycles (16 lanes wide) at 2.4 GHz, i.e.
# 39.3 T 32-bit lane operations per second.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def source_digest(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """Kernel name without return type, namespaces and argument list."""
    n = name.replace("void ", "")
    for ns in ("april::(anonymous namespace)::", "april::"):
        n = n.replace(ns, "")
    depth, out = 0, []
    for ch in n:   # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _one(pattern: str) -> str:
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise FileNotFoundError(pattern)
    return files[0]


def kernel_stats(trace_dir: str):
    """Rows of the --stats kernel table: (name, calls, avg_ns, min_ns, max_ns, pct)."""
    path = _one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["AverageNs"]),
                         float(r["MinNs"]), float(r["MaxNs"]), float(r["Percentage"])))
    return rows


def dispatch_times(trace_dir: str, kernel: str):
    """Durations (ns) of every dispatch of `kernel` in dispatch order, from
    the --kernel-trace CSV."""
    path = _one(os.path.join(trace_dir, "**", "*kernel_trace.csv"))
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if short_name(r["Kernel_Name"]).startswith(kernel):
                rows.append((int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    return [d for _, d in sorted(rows)]


def counters(pmc_dir: str):
    """{dispatch id: (kernel, {counter: value summed over dimensions})}."""
    path = _one(os.path.join(pmc_dir, "**", "*counter_collection.csv"))
    out = OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            name, vals = out.setdefault(d, (short_name(r["Kernel_Name"]), {}))
            vals[r["Counter_Name"]] = vals.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def _per_kernel(pmc_dir: str, counter: str, kernel: str):
    got = [v[counter] for _, (n, v) in counters(pmc_dir).items() if n.startswith(kernel) and counter in v]
    if not got:
        raise ValueError(f"no {counter} for {kernel} in {pmc_dir}")
    return got


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int = 1 << 30, parts=None):
    """HBM bytes per launch of `kernel` from FETCH_SIZE / WRITE_SIZE runs, each
    scaled by the counter's reading for a copy of `copy_bytes` (which reads
    and writes copy_bytes).  With `parts` (kernel name prefixes), a launch is
    one dispatch of each, and their per-dispatch averages are summed."""
    kib = copy_bytes / 1024.0
    cf = _per_kernel(fetch_dir, "FETCH_SIZE", COPY_KERNEL)
    cw = _per_kernel(write_dir, "WRITE_SIZE", COPY_KERNEL)
    # the calibration copies are the large ones
    cf = [x for x in cf if x > kib / 8]
    cw = [x for x in cw if x > kib / 8]
    f_factor = kib / (sum(cf) / len(cf))
    w_factor = kib / (sum(cw) / len(cw))
    fk = wk = 0.0
    per_part = {}
    n = None
    for part in parts or [kernel]:
        kf = _per_kernel(fetch_dir, "FETCH_SIZE", part)
        kw = _per_kernel(write_dir, "WRITE_SIZE", part)
        per_part[part] = {"fetch_kib_raw": sum(kf) / len(kf), "write_kib_raw": sum(kw) / len(kw),
                          "dispatches": len(kf)}
        fk += sum(kf) / len(kf)
        wk += sum(kw) / len(kw)
        n = len(kf) if n is None else min(n, len(kf))
    fetch = fk * 1024.0 * f_factor
    write = wk * 1024.0 * w_factor
    out = {"fetch_kib_raw": fk, "write_kib_raw": wk,
           "copy_fetch_kib": sum(cf) / len(cf), "copy_write_kib": sum(cw) / len(cw),
           "fetch_factor": f_factor, "write_factor": w_factor,
           "fetch_bytes": fetch, "write_bytes": write, "traffic_bytes": fetch + write,
           "dispatches": n}
    if parts:
        out["parts"] = per_part
    return out


def valu(pmc_dir: str, kernel: str, parts=None):
    """VALU instructions (SQ_INSTS_VALU, wave64 instructions) per launch of
    `kernel` (with `parts`: the sum of their per-dispatch averages)."""
    total, n, per_part = 0.0, None, {}
    for part in parts or [kernel]:
        x = _per_kernel(pmc_dir, "SQ_INSTS_VALU", part)
        per_part[part] = sum(x) / len(x)
        total += sum(x) / len(x)
        n = len(x) if n is None else min(n, len(x))
    out = {"insts_per_launch": total, "dispatches": n}
    if parts:
        out["parts"] = per_part
    return out


def _record(path: str, kernel: str, config: dict, pairs: int):
    """The record in `path`, if it was taken on the current sources of
    `kernel`, with `config` and `pairs`; else None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != source_digest(kernel):
        return None
    if rec.get("config") != config or rec.get("pairs") != pairs:
        return None
    return rec


def read_traffic(path: str, kernel: str, config: dict, pairs: int):
    """Traffic bytes per launch recorded in `path`, if that record was taken
    on the current sources of `kernel`, with `config` and `pairs`; else None."""
    rec = _record(path, kernel, config, pairs)
    return rec["traffic"]["traffic_bytes"] if rec else None


def read_valu(path: str, kernel: str, config: dict, pairs: int, kernel_ms: float):
    """VALU issue of a launch taking `kernel_ms`, from the instruction count
    recorded in `path` (same conditions as read_traffic), against the
    device's peak issue rate; None without a valid record."""
    rec = _record(path, kernel, config, pairs)
    if not rec:
        return None
    insts = rec["valu"]["insts_per_launch"]
    rate = insts / (kernel_ms / 1e3)
    return {"insts_per_launch": insts, "insts_per_pair": insts / pairs, "issue_rate": rate,
            "peak": VALU_ISSUE_PEAK, "unit": "wave64 VALU instructions/s", "frac": rate / VALU_ISSUE_PEAK}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("trace_dir")
    v = sub.add_parser("valu")
    v.add_argument("--pmc", required=True, help="a --pmc SQ_INSTS_VALU output folder")
    v.add_argument("--kernel", default="k_batched")
    v.add_argument("--parts", default="")
    v.add_argument("--config", default="")
    v.add_argument("--pairs", type=int, required=True)
    v.add_argument("--command", default="")
    v.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", default="k_batched")
    t.add_argument("--parts", default="", help="kernel name prefixes of one launch, comma-separated "
                                               "(default: the kernel alone)")
    t.add_argument("--config", default="")
    t.add_argument("--pairs", type=int, required=True)
    t.add_argument("--alg-bytes", type=int, default=0)
    t.add_argument("--command", default="")
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("pmc_dirs", nargs="+")
    c.add_argument("--kernel", default="k_")
    args = ap.parse_args()
    if args.cmd == "stats":
        print(f"{'kernel':44s} {'calls':>6s} {'avg us':>10s} {'min us':>10s} {'max us':>10s} {'%':>6s}")
        for n, calls, avg, mn, mx, pct in kernel_stats(args.trace_dir):
            print(f"{n[:44]:44s} {calls:6d} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f} {pct:6.2f}")
    elif args.cmd == "counters":
        for d in args.pmc_dirs:
            for disp, (n, v) in counters(d).items():
                if n.startswith(args.kernel) or n == COPY_KERNEL:
                    print(f"{os.path.basename(d.rstrip('/'))} dispatch {disp} {n}: " +
                          " ".join(f"{k}={x:.6g}" for k, x in sorted(v.items())))
    elif args.cmd == "valu":
        cfg = {k: int(x) for k, x in (kv.split("=") for kv in args.config.split(","))} if args.config else {}
        va = valu(args.pmc, args.kernel, parts=[p for p in args.parts.split(",") if p] or None)
        rec = {"kernel": args.kernel, "config": cfg, "pairs": args.pairs,
               "source_sha256": source_digest(args.kernel), "valu": va, "command": args.command}
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
            f.write("\n")
        print(json.dumps(rec, indent=1, sort_keys=True))
    else:
        cfg = {k: int(v) for k, v in (kv.split("=") for kv in args.config.split(","))} if args.config else {}
        tr = traffic(args.fetch, args.write, args.kernel,
                     parts=[p for p in args.parts.split(",") if p] or None)
        rec = {"kernel": args.kernel, "config": cfg, "pairs": args.pairs, "alg_bytes": args.alg_bytes,
               "source_sha256": source_digest(args.kernel), "traffic": tr, "command": args.command}
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
            f.write("\n")
        print(json.dumps(rec, indent=1, sort_keys=True))


if __name__ == "__main__":
    main()
