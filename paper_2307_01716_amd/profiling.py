"""Summaries of rocprofv3 output for the filter kernels.

Reads the CSV files that `rocprofv3 --kernel-trace --stats` and
`rocprofv3 --pmc ...` write, and turns them into short text summaries:

* kernel statistics (calls, average / min / max duration per kernel);
* per-dispatch counters of the filter kernels;
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


def read_traffic(path: str, kernel: str, config: dict, pairs: int):
    """Traffic bytes per launch recorded in `path`, if that record was taken
    on the current sources of `kernel`, with `config` and `pairs`; else None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != source_digest(kernel):
        return None
    if rec.get("config") != config or rec.get("pairs") != pairs:
        return None
    return rec["traffic"]["traffic_bytes"]


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("trace_dir")
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
