#!/usr/bin/env python3
"""Throughput of the APRIL intermediate filter on one MI355X.

Workload: the at-scale join -- |R| = |S| = 200,000 seeded star polygons
(vertex count log-normal, median 30; centres from a 64-component Gaussian
mixture; radius log-normal, median 0.001), grid order 16, all ~4.7M
candidate pairs of the MBR filter.  Lists are built by the library, pairs by
the library's MBR join; both are resident in HBM before timing starts.

A step is one april_filter_pairs call over every candidate pair.  W untimed
warm-up steps, then K timed steps between device synchronizations; HIP
events on the launch stream give the per-launch kernel time.  The roofline
uses the bytes Alg. 2 itself moves (april_alg2_bytes, summed over the pairs)
per launch, against MI355X's 8 TB/s HBM peak.

The CPU baseline is the oracle (plain C, all host threads up to 16) timed on
a bounded sample: every candidate pair among the objects whose MBR centres
lie in a square window holding about 2% of each collection, repeated until
about 10 s of CPU time has passed.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--schedule", choices=["both", "plain", "batched"], default="both")
    ap.add_argument("--no-tune", action="store_true", help="batched: library defaults, no sweep")
    ap.add_argument("--config", default="",
                    help="batched: fixed tuning instead of a sweep, e.g. tile=256,waves_per_simd=6")
    ap.add_argument("--no-graph", action="store_true", help="batched: eager launches")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB three times (reference dispatches for HBM counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-random-order", action="store_true",
                    help="skip the extra timing of the batched kernel on pairs in random order "
                         "(profiles of the in-order launches)")
    ap.add_argument("--workload", choices=["scale", "skewed"], default="scale",
                    help="scale: 200k x 200k polygons (default); skewed: the same plus 2000 "
                         "complex polygons (20k-100k vertices) per side")
    ap.add_argument("--serve", action="store_true",
                    help="served selection queries instead of the batch filter (own JSON line)")
    ap.add_argument("--serve-objects", type=int, default=1_000_000)
    ap.add_argument("--gpu-build-cells", type=int, default=0,
                    help="served queries spanning this many grid cells or more are built on the GPU "
                         "(0: library default 2^18; 4294967295: never)")
    ap.add_argument("--partitioned", action="store_true",
                    help="partitioned join, raw and compressed lists (own JSON line)")
    ap.add_argument("--part-objects", type=int, default=500_000)
    ap.add_argument("--variants", action="store_true",
                    help="within join, polygon-linestring join and mixed grid orders (own JSON line)")
    ap.add_argument("--build", action="store_true",
                    help="list construction on the GPU against the host builder (own JSON line)")
    ap.add_argument("--refine", action="store_true",
                    help="exact refinement after the filter, against refining every candidate "
                         "pair (own JSON line)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="offered arrivals per load level last about this long (at most 10^4 queries)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--tune-table", default=os.path.join(HERE, "paper_2307_01716_amd", "tuning", "mi355x.json"),
                    help="stored batched settings (device x workload signature) used instead of a sweep")
    ap.add_argument("--retune", action="store_true", help="sweep even when the table has the workload")
    ap.add_argument("--tune-out", default="", help="store swept settings in this table")
    ap.add_argument("--no-skewed", action="store_true",
                    help="skip the skewed workload's leg of the default run")
    ap.add_argument("--skewed-no-plain", action="store_true",
                    help="skewed leg: batched form only")
    return ap.parse_args()


def cpu_baseline(R, S, g, seconds):
    """Oracle filter on a spatial-window sample; returns the cpu_baseline dict."""
    import oracle

    cores = min(16, len(os.sched_getaffinity(0)))
    mR, mS = R.mbrs(), S.mbrs()
    cR = (mR[:, :2] + mR[:, 2:]) / 2
    cS = (mS[:, :2] + mS[:, 2:]) / 2
    # a square window around the densest mixture region holding ~2% of R
    target = max(1, len(R) // 50)
    centre = np.median(cR[np.argsort(np.linalg.norm(cR - cR.mean(0), axis=1))[: len(R) // 10]], axis=0)
    d = np.max(np.abs(cR - centre), axis=1)
    half = float(np.sort(d)[target - 1])
    inR = np.nonzero(d <= half)[0]
    inS = np.nonzero(np.max(np.abs(cS - centre), axis=1) <= half)[0]
    Rs, Ss = R.subset(inR), S.subset(inS)
    t0 = time.time()
    LR = oracle.build_lists(g, Rs, cores)
    LS = oracle.build_lists(g, Ss, cores)
    r, s = oracle.mbr_join(Rs, Ss, cores)
    build_s = time.time() - t0
    reps, t_filter, used = 0, 0.0, cores
    while t_filter < seconds or reps == 0:
        t1 = time.perf_counter()
        _, used = oracle.filter_pairs_timed(LR, LS, r, s, cores)
        t_filter += time.perf_counter() - t1
        reps += 1
    value = reps * len(r) / t_filter
    # one thread, one pass over the same sample (median of three)
    t1s = []
    for _ in range(3):
        t1 = time.perf_counter()
        oracle.filter_pairs_timed(LR, LS, r, s, 1)
        t1s.append(time.perf_counter() - t1)
    single = len(r) / float(np.median(t1s))
    return {"value": value, "unit": "pairs/s", "cores": int(used), "kind": "oracle",
            "single_thread_value": single, "cpu": cpu_model(),
            "sample": (f"all {len(r)} candidate pairs among the {len(inR)} R and {len(inS)} S "
                       f"objects whose MBR centres lie in a {2 * half:.4f}-wide square window; "
                       f"filter repeated {reps}x ({t_filter:.1f} s); list build {build_s:.1f} s "
                       "not timed")}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gpu_lists(april, g, P, max_vertices=16_000_000):
    """Lists of polygon set P built on the GPU in chunks of consecutive
    polygons (each chunk's build scratch then fits the device), read back and
    joined into one host collection."""
    parts = []
    v = P.voff
    k = 0
    n = len(v) - 1
    while k < n:
        e = int(np.searchsorted(v, v[k] + max_vertices, side="right")) - 1
        e = max(e, k + 1)
        e = min(e, n)
        sub = P.subset(np.arange(k, e))
        d = april.april_build_lists_gpu(g, sub.xy, sub.voff, april.STRICT)
        parts.append(april.april_lists_download(d).export())
        d.free()
        k = e
    offA, sA, eA, offF, sF, eF = [], [], [], [], [], []
    ba = bf = 0
    for i, (oa, sa, ea, of, sf, ef) in enumerate(parts):
        offA.append(oa[(1 if i else 0):] + np.uint64(ba))
        offF.append(of[(1 if i else 0):] + np.uint64(bf))
        sA.append(sa), eA.append(ea), sF.append(sf), eF.append(ef)
        ba += len(sa)
        bf += len(sf)
    cat = np.concatenate
    return april.april_lists_from_arrays(g, cat(offA), cat(sA), cat(eA), cat(offF), cat(sF), cat(eF),
                                         validate=False)


def calibration_copies():
    """Three 1 GiB device-to-device copies: reference dispatches of known
    size for the HBM byte counters (FETCH_SIZE, WRITE_SIZE)."""
    import torch
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: 3 x 1 GiB device-to-device copies")


def autotune(tune, dR, dS, r, s, verdict, counts, ws, sig, args):
    """Sweep the batched schedule's knobs; keep the library defaults unless
    the best setting is more than 2% faster; store the result under
    --tune-out (keyed by device and workload signature)."""
    t0 = time.time()
    cfg, best_ms, table = tune.sweep(dR, dS, r, s, verdict, counts, ws, reps=3, log=log)
    dflt_ms = tune.time_config(dR, dS, r, s, verdict, counts, ws, reps=3)
    log(f"autotune: {len(table)} settings in {time.time() - t0:.1f}s; best {cfg} "
        f"({best_ms:.3f} ms); library defaults {dflt_ms:.3f} ms")
    if best_ms > 0.98 * dflt_ms:   # within run-to-run noise: keep the defaults
        cfg, best_ms = {}, dflt_ms
    if args.tune_out:
        tune.save(args.tune_out, tune.device_key(), sig, cfg, best_ms, table)
    return cfg, "sweep"


def skewed_leg(args, stream):
    """The skewed workload: batched (hipGraph replay) and plain forms on all
    ~30M pairs, the workgroup bin's share and the schedule's tail, measured
    HBM traffic when a record for the current kernel exists."""
    import torch

    import synth
    from paper_2307_01716_amd import april, profiling, tune

    t0 = time.time()
    R, S, g = synth.configs.skewed()
    log(f"skewed: generated R={len(R)} S={len(S)} in {time.time() - t0:.1f}s")
    t0 = time.time()
    hR, hS = gpu_lists(april, g, R), gpu_lists(april, g, S)
    log(f"skewed: lists built on the GPU (A={hR.info().n_a + hS.info().n_a}) in {time.time() - t0:.1f}s")
    r_np, s_np = april.april_mbr_join(R.mbrs(), S.mbrs())
    P = len(r_np)
    # the bins, from the list lengths (as the library's binning pass decides)
    oR, oS = hR.export(), hS.export()
    mr = np.maximum(np.diff(oR[0].astype(np.int64)), np.diff(oR[3].astype(np.int64)))[r_np]
    ms = np.maximum(np.diff(oS[0].astype(np.int64)), np.diff(oS[3].astype(np.int64)))[s_np]
    del oR, oS, R, S
    dR = april.april_lists_to_device(hR, stream=stream)
    dS = april.april_lists_to_device(hS, stream=stream)
    r = torch.from_numpy(r_np.view(np.int32)).cuda()
    s = torch.from_numpy(s_np.view(np.int32)).cuda()
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.zeros(3, dtype=torch.int64, device="cuda")
    ws = torch.empty(april.april_filter_workspace_size(P), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    sig = tune.signature(P, dR, dS)
    cfg = tune.load(args.tune_table, tune.device_key(), sig)
    src = "tuning table"
    if cfg is None or args.retune:
        cfg, src = {}, "library defaults"
        if not args.no_tune:
            cfg, src = autotune(tune, dR, dS, r, s, verdict, counts, ws, sig, args)
    kw = tune.call_config(cfg)
    tile = cfg.get("tile") or (256 if (hR.info().n_a + hS.info().n_a) <= 256 * (len(hR) + len(hS)) else 512)
    wg_min = cfg.get("wg_min") or 4096
    in_wg = (mr >= tile) & (ms >= tile) & (np.minimum(mr, ms) >= wg_min)
    log(f"skewed: {P} pairs; setting {cfg} ({src}); workgroup bin {int(in_wg.sum())} pairs")

    def run(flags=0):
        april.april_filter_pairs(dR, dS, r, s, verdict, counts, schedule=april.SCHED_BATCHED,
                                 workspace=ws, stream=stream, flags=flags, **kw)

    run()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(stream)
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            april.april_filter_pairs(dR, dS, r, s, verdict, counts, schedule=april.SCHED_BATCHED,
                                     workspace=ws, stream=torch.cuda.current_stream(), **kw)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 2)
    ts = []
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        graph.replay()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ms_b = float(np.mean(ts))
    c = counts.cpu().numpy()
    assert int(c.sum()) == P
    batched_v = verdict.clone()
    # the schedule's tail: wavefront end times of one eager launch
    run(april.WAVE_TIMES)
    torch.cuda.synchronize()
    t = ws[april.WAVE_TIMES_OFFSET:april.WAVE_TIMES_OFFSET + 24].cpu().numpy().view(np.uint64)
    span = float(t[2] - t[0])
    tail_frac = float(t[2] - t[1]) / span if span > 0 else 0.0
    out = {"workload": "skewed: 200k x 200k star polygons plus 2000 x 2000 with 20k-100k vertices "
                       "(radius 0.02-0.1), grid 2^16, all MBR candidate pairs",
           "pairs": P, "verdicts": {"TN": int(c[0]), "TH": int(c[1]), "IND": int(c[2])},
           "batched": {"kernel_ms": ms_b, "kernel_ms_median": float(np.median(ts)),
                       "kernel_ms_p10": float(np.percentile(ts, 10)),
                       "kernel_ms_p90": float(np.percentile(ts, 90)), "steps": steps,
                       "pairs_per_s": P / (ms_b / 1e3), "hipgraph": True, "tuning": cfg,
                       "tuning_source": src, "workgroup_bin_pairs": int(in_wg.sum()),
                       "tail_ms": tail_frac * ms_b, "tail_frac": tail_frac}}
    log(f"skewed batched: {ms_b:.2f} ms ({P / ms_b / 1e3:.0f} M pairs/s); tail {tail_frac * ms_b:.2f} ms "
        f"({tail_frac:.1%}); TN/TH/IND = {c.tolist()}")
    kname = "k_batched"
    tr = profiling.read_traffic(os.path.join(HERE, "profiles", f"{kname}_skewed_traffic.txt"), kname, cfg, P)
    if tr is not None:
        out["batched"]["traffic_bytes"] = tr
        out["batched"]["hbm_GBps"] = tr / (ms_b / 1e3) / 1e9
        out["batched"]["hbm_frac"] = out["batched"]["hbm_GBps"] / HBM_PEAK_GBS
    else:
        out["batched"]["traffic_bytes"] = None
    out["batched"]["valu"] = profiling.read_valu(os.path.join(HERE, "profiles", f"{kname}_skewed_valu.txt"),
                                                 kname, cfg, P, ms_b)
    if not args.skewed_no_plain:
        ts = []
        for k in range(2):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            april.april_filter_pairs(dR, dS, r, s, verdict, counts, schedule=april.SCHED_PLAIN, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        assert torch.equal(verdict, batched_v), "skewed: batched and plain verdicts differ"
        out["plain"] = {"kernel_ms": float(np.mean(ts)), "pairs_per_s": P / (np.mean(ts) / 1e3), "steps": 2}
        out["batched"]["speedup_vs_plain"] = out["plain"]["kernel_ms"] / ms_b
        log(f"skewed plain: {out['plain']['kernel_ms']:.1f} ms; batched speedup "
            f"{out['batched']['speedup_vs_plain']:.1f}x")
    del dR, dS, ws, r, s, verdict
    torch.cuda.empty_cache()
    return out


def serve_bench(args):
    """Served selection queries on one GPU: S device-resident, query lists
    built by builder threads (large queries on the GPU), filtered in
    continuous batches.  Saturation throughput (all queries offered at once),
    then Poisson arrivals at 0.5, 0.8 and 0.95 of it; per level p50/p99 of
    submit-to-done latency (the library's steady clock), of its list-build
    part, and pairs/s."""
    import torch

    import synth
    from paper_2307_01716_amd import april

    assert torch.cuda.is_available(), "no HIP device"
    t0 = time.time()
    S, Q, g = synth.configs.serving(n_s=args.serve_objects, n_queries=11_000)
    log(f"generated S={len(S)} queries={len(Q)} in {time.time() - t0:.1f}s")
    t0 = time.time()
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    dS = april.april_lists_to_device(hS)
    torch.cuda.synchronize()
    info = hS.info()
    log(f"S lists: A={info.n_a} F={info.n_f} intervals, built and uploaded in {time.time() - t0:.1f}s")
    srv = april.Server(dS, S.mbrs(), gpu_build_cells=args.gpu_build_cells)
    warm, n_sat = 1000, 4000
    nq = len(Q)

    def collect(tickets):
        out = []
        for t in tickets:
            out.append(srv.wait(t, 600))
            srv.release(t)
        return out

    collect([srv.submit(Q.polygon(k)) for k in range(warm)])
    log(f"warm-up: {warm} queries")
    t0 = time.perf_counter()
    res = collect([srv.submit(Q.polygon(warm + k)) for k in range(n_sat)])
    t_sat = time.perf_counter() - t0
    sat_qps = n_sat / t_sat
    sat_pairs = sum(len(r.s_ids) for r in res)
    log(f"saturation: {n_sat} queries in {t_sat:.2f}s = {sat_qps:.0f} queries/s, "
        f"{sat_pairs / t_sat / 1e6:.1f} M pairs/s, {sat_pairs / n_sat:.0f} pairs/query")
    rng = np.random.default_rng(7)
    levels = []
    nxt = warm + n_sat
    for load in (0.5, 0.8, 0.95):
        rate = load * sat_qps
        n = int(min(10_000, max(200, rate * args.serve_seconds)))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
        tickets = []
        t0 = time.perf_counter()
        for k in range(n):
            while time.perf_counter() - t0 < arrivals[k]:
                pass
            tickets.append(srv.submit(Q.polygon((nxt + k) % nq)))
        res = collect(tickets)
        wall = time.perf_counter() - t0
        nxt += n
        lat = np.array([r.t_done - r.t_submit for r in res]) * 1e3
        bld = np.array([r.t_built - r.t_submit for r in res]) * 1e3
        dvc = np.array([r.t_done - r.t_built for r in res]) * 1e3   # waiting for a slot + device
        pairs = sum(len(r.s_ids) for r in res)
        lv = {"load": load, "queries": n, "offered_qps": rate, "achieved_qps": n / wall,
              "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
              "build_p50_ms": float(np.percentile(bld, 50)), "build_p99_ms": float(np.percentile(bld, 99)),
              "device_p50_ms": float(np.percentile(dvc, 50)), "device_p99_ms": float(np.percentile(dvc, 99)),
              "pairs_per_s": pairs / wall, "pairs_per_query": pairs / n}
        levels.append(lv)
        log(f"load {load}: {n} queries at {rate:.0f}/s offered: latency p50 {lv['p50_ms']:.2f} ms "
            f"p99 {lv['p99_ms']:.2f} ms (lists built p50 {lv['build_p50_ms']:.2f} ms, "
            f"p99 {lv['build_p99_ms']:.2f} ms; slot wait + device p50 {lv['device_p50_ms']:.2f} ms, "
            f"p99 {lv['device_p99_ms']:.2f} ms); {lv['pairs_per_s'] / 1e6:.1f} M pairs/s")
    st = srv.stats()
    srv.close()
    out = {"metric": "served selection queries (p50/p99 latency per offered load)",
           "value": sat_pairs / t_sat, "unit": "pairs/s", "n_gpus": 1, "steps": len(levels),
           "warmup": warm, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"served: S = {len(S)} star polygons device-resident, grid 2^16; "
                                  "queries 10..10^4 vertices, radius 5e-4..0.05 (log-uniform)",
                      "slots": st["slots"], "cap_pairs": st["cap_pairs"],
                      "gpu_build_cells": args.gpu_build_cells or (1 << 18)},
           "served": {"saturation_qps": sat_qps, "saturation_pairs_per_s": sat_pairs / t_sat,
                      "levels": levels}}
    print(json.dumps(out), flush=True)


def partitioned_bench(args):
    """Partitioned join on one GPU: |R| = |S| = n at-scale polygons, the unit
    square cut into 16 x 16 partitions with a grid of order 16 each, every
    object an instance in each partition its MBR meets, pairs kept in the
    partition holding their reference point.  The same pairs are filtered on
    raw and on delta + VByte lists (batched schedule, one launch over all
    partitions); HIP events time each launch."""
    import torch

    import synth
    from paper_2307_01716_amd import april, partitioned, profiling, tune

    assert torch.cuda.is_available(), "no HIP device"
    t0 = time.time()
    R, S, lay = synth.configs.partitioned(n=args.part_objects)
    log(f"generated R={len(R)} S={len(S)}, {lay.k}x{lay.k} partitions, "
        f"{len(lay.r_obj)} + {len(lay.s_obj)} instances in {time.time() - t0:.1f}s")
    t0 = time.time()
    hR = partitioned.build_instances(lay, R, "r")
    hS = partitioned.build_instances(lay, S, "s")
    log(f"built instance lists in {time.time() - t0:.1f}s")
    t0 = time.time()
    r_np, s_np, n_all = partitioned.pairs(lay, R, S, with_all_count=True)
    P = len(r_np)
    log(f"pairs: {P} after the reference-point rule, {n_all} partition-local before "
        f"({time.time() - t0:.1f}s)")
    stream = torch.cuda.current_stream()
    r = torch.from_numpy(r_np.view(np.int32)).cuda()
    s = torch.from_numpy(s_np.view(np.int32)).cuda()
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.zeros(3, dtype=torch.int64, device="cuda")
    ws = torch.empty(april.april_filter_workspace_size(P), dtype=torch.uint8, device="cuda")
    forms, ref = {}, None
    for codec, name, grid in ((april.CODEC_RAW, "raw", {"tile": (256, 512), "chunk": (1, 2, 4)}),
                              (april.CODEC_VBYTE, "vbyte", {"tile": (256, 512, 1024),
                                                            "search_min": (64, 1024)})):
        dR = april.april_lists_to_device(hR, codec=codec, stream=stream)
        dS = april.april_lists_to_device(hS, codec=codec, stream=stream)
        torch.cuda.synchronize()
        nbytes = dR.info().device_bytes + dS.info().device_bytes
        best = None
        if args.no_tune:   # fixed settings (as profiled): the library defaults
            grid = {"tile": (512,)}
        for vals in __import__("itertools").product(*grid.values()):
            cfg = dict(zip(grid, vals))
            ms = tune.time_config(dR, dS, r, s, verdict, counts, ws, reps=5, **cfg)
            log(f"  {name} {cfg}: {ms:.3f} ms")
            if best is None or ms < best[1]:
                best = (cfg, ms)
        cfg, _ = best
        ms = tune.time_config(dR, dS, r, s, verdict, counts, ws, reps=args.steps, **cfg)
        c = counts.cpu().numpy()
        if ref is None:
            ref = verdict.clone()
        assert torch.equal(verdict, ref), "raw and compressed verdicts differ"
        forms[name] = {"kernel_ms": ms, "pairs_per_s": P / (ms / 1e3), "device_bytes": int(nbytes),
                       "tuning": cfg, "verdicts": {"TN": int(c[0]), "TH": int(c[1]), "IND": int(c[2])}}
        # Alg. 2's bytes: raw intervals, or the consumed prefixes of the
        # compressed streams (Sec. 5.1)
        by = torch.empty(P, dtype=torch.int64, device="cuda")
        april.april_alg2_bytes(dR, dS, r, s, by, stream=stream)
        torch.cuda.synchronize()
        forms[name]["alg_bytes"] = int(by.sum().item())
        forms[name]["alg_GBps"] = forms[name]["alg_bytes"] / (ms / 1e3) / 1e9
        forms[name]["alg_frac"] = forms[name]["alg_GBps"] / HBM_PEAK_GBS
        del by
        # measured HBM traffic and VALU issue, from the committed rocprofv3
        # records when they were taken on these sources and this launch
        kname = "k_batched" if codec == april.CODEC_RAW else "k_filter_vbyte"
        stem = os.path.join(HERE, "profiles", f"{kname}_partitioned500k")
        tr = profiling.read_traffic(stem + "_traffic.txt", kname, cfg, P)
        forms[name]["traffic_bytes"] = tr
        if tr is not None:
            forms[name]["hbm_frac"] = tr / (ms / 1e3) / 1e9 / HBM_PEAK_GBS
        forms[name]["valu"] = profiling.read_valu(stem + "_valu.txt", kname, cfg, P, ms)
        log(f"{name}: {ms:.3f} ms, {P / ms / 1e6:.3f} G pairs/s, lists {nbytes / 1e9:.2f} GB on device")
        del dR, dS
        torch.cuda.synchronize()
    out = {"metric": "candidate pairs filtered/s (partitioned join, delta + VByte lists decoded in-kernel)",
           "value": forms["vbyte"]["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "ms_per_step": forms["vbyte"]["kernel_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"partitioned: {len(R)} x {len(S)} star polygons, {lay.k}x{lay.k} "
                                  "partitions, grid 2^16 each",
                      "pairs": P, "pairs_before_dedup": int(n_all),
                      "instances": [int(len(lay.r_obj)), int(len(lay.s_obj))]},
           "forms": forms,
           "compression": forms["raw"]["device_bytes"] / forms["vbyte"]["device_bytes"],
           "roofline": {"bound": "hbm", "achieved": forms["vbyte"]["alg_GBps"], "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": forms["vbyte"]["alg_frac"],
                        "traffic": forms["vbyte"]["traffic_bytes"]}}
    print(json.dumps(out), flush=True)


def variants_bench(args):
    """The filter's query variants at scale, each over all its candidate
    pairs with lists resident in HBM; W untimed launches, then K timed ones,
    HIP events on the launch stream:
      within       r within s on the at-scale join (4.7M pairs);
      linestrings  200k polygons x 200k random-walk linestrings;
      mixed        R at grid order 16 against S at order 14 (one data space).
    The same pairs through april_filter_pairs (one order) are timed beside
    for reference.  The CPU baseline is the oracle's within filter on a
    bounded sample."""
    import torch

    import synth
    from paper_2307_01716_amd import april

    assert torch.cuda.is_available(), "no HIP device"
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    def dev(h):
        return april.april_lists_to_device(h, stream=stream)

    forms = {}
    R, S, g = synth.configs.scale()
    hR = april.april_build_lists(g, R.xy, R.voff, april.STRICT)
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    r_np, s_np = april.april_mbr_join(R.mbrs(), S.mbrs())
    P = len(r_np)
    r = torch.from_numpy(r_np.view(np.int32)).cuda()
    s = torch.from_numpy(s_np.view(np.int32)).cuda()
    v = torch.empty(P, dtype=torch.uint8, device="cuda")
    c = torch.zeros(3, dtype=torch.int64, device="cuda")
    dR, dS = dev(hR), dev(hS)
    for name, fn in (("within", lambda: april.april_filter_within(dR, dS, r, s, v, c, stream=stream)),
                     ("one-order filter (plain)", lambda: april.april_filter_pairs(dR, dS, r, s, v, c,
                                                                                    stream=stream))):
        ms = timed(fn)
        cc = c.cpu().numpy()
        forms[name] = {"ms": ms, "pairs": P, "pairs_per_s": P / (ms / 1e3),
                       "verdicts": {"TN": int(cc[0]), "TH": int(cc[1]), "IND": int(cc[2])}}
        log(f"{name}: {ms:.3f} ms, {P / ms / 1e6:.3f} G pairs/s, TN/TH/IND = {cc.tolist()}")
    gf, gc = synth.configs.two_orders(R, S, 16, 14)
    mR = dev(april.april_build_lists(gf, R.xy, R.voff, april.STRICT))
    mS = dev(april.april_build_lists(gc, S.xy, S.voff, april.STRICT))
    ms = timed(lambda: april.april_filter_mixed(mR, mS, r, s, v, c, stream=stream))
    cc = c.cpu().numpy()
    forms["mixed 16 x 14"] = {"ms": ms, "pairs": P, "pairs_per_s": P / (ms / 1e3),
                              "verdicts": {"TN": int(cc[0]), "TH": int(cc[1]), "IND": int(cc[2])},
                              "device_bytes_S": int(mS.info().device_bytes),
                              "device_bytes_S_order16": int(dS.info().device_bytes)}
    log(f"mixed 16 x 14: {ms:.3f} ms, {P / ms / 1e6:.3f} G pairs/s, TN/TH/IND = {cc.tolist()}; "
        f"S lists {mS.info().device_bytes / 1e6:.0f} MB at order 14 vs {dS.info().device_bytes / 1e6:.0f} MB")
    del mR, mS
    Pp, L, gl = synth.configs.linestring_scale()
    dP = dev(april.april_build_lists(gl, Pp.xy, Pp.voff, april.STRICT))
    hC = april.april_build_cells(gl, L.xy, L.voff, april.STRICT)
    dC = april.april_cells_to_device(hC, stream=stream)
    p_np, l_np = april.april_mbr_join(Pp.mbrs(), L.mbrs())
    pl = torch.from_numpy(p_np.view(np.int32)).cuda()
    ll = torch.from_numpy(l_np.view(np.int32)).cuda()
    vl = torch.empty(len(p_np), dtype=torch.uint8, device="cuda")
    ms = timed(lambda: april.april_filter_linestrings(dP, dC, pl, ll, vl, c, stream=stream))
    cc = c.cpu().numpy()
    forms["linestrings"] = {"ms": ms, "pairs": int(len(p_np)), "pairs_per_s": len(p_np) / (ms / 1e3),
                            "cells": int(hC.info()[1]),
                            "verdicts": {"TN": int(cc[0]), "TH": int(cc[1]), "IND": int(cc[2])}}
    log(f"linestrings: {ms:.3f} ms for {len(p_np)} pairs, {len(p_np) / ms / 1e6:.3f} G pairs/s, "
        f"TN/TH/IND = {cc.tolist()}")
    out = {"metric": "candidate pairs filtered/s (within join at scale)", "value": forms["within"]["pairs_per_s"],
           "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": forms["within"]["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "scale: 200k x 200k star polygons, grid 2^16, all MBR candidate pairs; "
                                  "linestrings: 200k polygons x 200k random walks"},
           "forms": forms}
    if not args.no_cpu_baseline:
        import oracle
        LRo, LSo = oracle.Lists(*hR.export()), oracle.Lists(*hS.export())
        sample = np.arange(0, P, 10)
        t0 = time.perf_counter()
        oracle.filter_within(LRo, LSo, r_np[sample], s_np[sample])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(sample) / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
                               "sample": f"every 10th within pair ({len(sample)}), one thread ({dt:.1f} s)"}
        log(f"cpu baseline (within): {len(sample) / dt / 1e6:.2f} M pairs/s on one thread")
    print(json.dumps(out), flush=True)


def build_bench(args):
    """List construction (Sec. 6) on the GPU against the library's host
    builder, on the at-scale collection R (200k polygons) and on 200 complex
    polygons (20k-100k vertices, as in the skewed workload).  A step is
    one april_build_lists_gpu call (upload, build, lists resident in HBM; the
    call synchronizes); W untimed calls, then K timed ones, wall clock.  The
    host builder (all host threads) is timed once per collection.  The CPU
    baseline is the oracle's builder on a bounded sample of R."""
    import torch

    import synth
    from paper_2307_01716_amd import april

    assert torch.cuda.is_available(), "no HIP device"
    R, S, g = synth.configs.scale()
    cases = [("scale R: 200k star polygons, grid 2^16", R, g)]
    big = synth.configs.large_collection(np.random.default_rng(3001), 200, 3)
    cases.append(("complex: 200 polygons of 20k-100k vertices (the skewed workload's large ones), grid 2^16",
                  big, synth.grid.grid_covering([big], 16)))
    forms = {}
    for name, ps, grid in cases:
        nv = int(ps.voff[-1])
        stream = torch.cuda.current_stream()
        for _ in range(args.warmup):
            april.april_build_lists_gpu(grid, ps.xy, ps.voff, april.STRICT, stream=stream).free()
        torch.cuda.synchronize()
        times = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            L = april.april_build_lists_gpu(grid, ps.xy, ps.voff, april.STRICT, stream=stream)
            times.append(time.perf_counter() - t0)
            inf = L.info()
            L.free()
        ms = float(np.median(times)) * 1e3
        t0 = time.perf_counter()
        H = april.april_build_lists(grid, ps.xy, ps.voff, april.STRICT)
        host_ms = (time.perf_counter() - t0) * 1e3
        assert H.info().n_a == inf.n_a and H.info().n_f == inf.n_f, "GPU and host lists differ in size"
        del H
        forms[name] = {"ms": ms, "polygons": len(ps), "vertices": nv, "intervals": int(inf.n_a + inf.n_f),
                       "polygons_per_s": len(ps) / (ms / 1e3), "vertices_per_s": nv / (ms / 1e3),
                       "host_builder_ms": host_ms, "speedup_vs_host": host_ms / ms}
        log(f"{name}: GPU {ms:.1f} ms ({len(ps) / ms / 1e3:.2f} M polygons/s, {nv / ms / 1e3:.1f} M vertices/s); "
            f"host builder {host_ms:.0f} ms ({host_ms / ms:.1f}x)")
    first = forms[cases[0][0]]
    out = {"metric": "polygons built/s (A- and F-lists on the GPU, lists resident in HBM)",
           "value": first["polygons_per_s"], "unit": "polygons/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": first["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "i64", "data": "synthetic",
           "config": {"workload": cases[0][0]}, "forms": forms}
    if not args.no_cpu_baseline:
        import oracle
        sample = R.subset(np.arange(0, len(R), 100))
        t0 = time.perf_counter()
        oracle.build_lists(g, sample)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(sample) / dt, "unit": "polygons/s",
                               "cores": int(min(16, len(os.sched_getaffinity(0)))), "kind": "oracle",
                               "sample": f"every 100th polygon of R ({len(sample)}), the oracle's builder "
                                         f"({dt:.1f} s)"}
        log(f"cpu baseline: {len(sample) / dt:.0f} polygons/s")
    print(json.dumps(out), flush=True)


def refine_bench(args):
    """Refinement on the at-scale workload (or --workload skewed).  The batched filter's verdicts are
    computed once (untimed); then three timed forms, each K launches after W
    warm-up ones, HIP events on the launch stream:
      refine_ind     april_refine_pairs on the indecisive pairs only;
      filter_refine  the filter plus a refinement call that takes its
                     verdicts (only indecisive pairs are tested);
      refine_all     every candidate pair tested exactly, no filter.
    The CPU baseline is the oracle's exact test, one pair per call, on
    indecisive pairs for about --cpu-seconds."""
    import torch

    import synth
    from paper_2307_01716_amd import april

    assert torch.cuda.is_available(), "no HIP device"
    t0 = time.time()
    R, S, g = synth.configs.scale() if args.workload == "scale" else synth.configs.skewed()
    r_np, s_np = april.april_mbr_join(R.mbrs(), S.mbrs())
    P = len(r_np)
    stream = torch.cuda.current_stream()
    dR = april.april_lists_to_device(april.april_build_lists(g, R.xy, R.voff, april.STRICT), stream=stream)
    dS = april.april_lists_to_device(april.april_build_lists(g, S.xy, S.voff, april.STRICT), stream=stream)
    pR = april.april_polys_to_device(R.xy, R.voff, april.STRICT, stream=stream)
    pS = april.april_polys_to_device(S.xy, S.voff, april.STRICT, stream=stream)
    r = torch.from_numpy(r_np.view(np.int32)).cuda()
    s = torch.from_numpy(s_np.view(np.int32)).cuda()
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    fcounts = torch.zeros(3, dtype=torch.int64, device="cuda")
    ws = torch.empty(april.april_filter_workspace_size(P), dtype=torch.uint8, device="cuda")
    april.april_filter_pairs(dR, dS, r, s, verdict, fcounts, schedule=april.SCHED_BATCHED, workspace=ws)
    torch.cuda.synchronize()
    v_np = verdict.cpu().numpy()
    ind = np.nonzero(v_np == april.INDECISIVE)[0]
    ri, si = r[torch.from_numpy(ind).cuda()], s[torch.from_numpy(ind).cuda()]
    nv_r, nv_s = np.diff(R.voff), np.diff(S.voff)
    edge_pairs_ind = int(np.sum(nv_r[r_np[ind]] * nv_s[s_np[ind]]))
    edge_pairs_all = int(np.sum(nv_r[r_np].astype(np.int64) * nv_s[s_np]))
    log(f"setup {time.time() - t0:.1f}s: {P} pairs, {len(ind)} indecisive "
        f"({edge_pairs_ind / 1e6:.1f}M edge pairs; all pairs {edge_pairs_all / 1e9:.2f}G)")
    out_ind = torch.empty(len(ind), dtype=torch.uint8, device="cuda")
    out_all = torch.empty(P, dtype=torch.uint8, device="cuda")
    rc = torch.zeros(2, dtype=torch.int64, device="cuda")

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    forms = {}
    log("refine indecisive: timing")
    ms = timed(lambda: april.april_refine_pairs(pR, pS, ri, si, out_ind, counts=rc, stream=stream))
    hits_ind = int(rc[0].item())
    forms["refine_ind"] = {"ms": ms, "pairs": len(ind), "pairs_per_s": len(ind) / (ms / 1e3),
                           "edge_pairs_per_s": edge_pairs_ind / (ms / 1e3), "intersecting": hits_ind}
    log(f"refine indecisive: {ms:.3f} ms, {len(ind) / ms / 1e3:.2f} M pairs/s, {hits_ind} intersect")

    def pipeline():
        april.april_filter_pairs(dR, dS, r, s, verdict, fcounts, schedule=april.SCHED_BATCHED, workspace=ws,
                                 stream=stream)
        april.april_refine_pairs(pR, pS, r, s, out_all, verdict=verdict, counts=rc, stream=stream)
    log("filter + refine: timing")
    ms = timed(pipeline)
    c = rc.cpu().numpy()
    res_filter = out_all.clone()
    forms["filter_refine"] = {"ms": ms, "pairs_per_s": P / (ms / 1e3), "intersecting": int(c[0]),
                              "tested": int(c[1])}
    log(f"filter + refine: {ms:.3f} ms, {P / ms / 1e6:.3f} G pairs/s, {int(c[0])} intersect")
    if args.workload == "scale":
        log("refine all: timing")
        ms = timed(lambda: april.april_refine_pairs(pR, pS, r, s, out_all, counts=rc, stream=stream))
        c = rc.cpu().numpy()
        assert torch.equal(out_all, res_filter), "refinement with and without the filter disagree"
        forms["refine_all"] = {"ms": ms, "pairs_per_s": P / (ms / 1e3),
                               "edge_pairs_per_s": edge_pairs_all / (ms / 1e3), "intersecting": int(c[0]),
                               "tested": int(c[1])}
        log(f"refine all: {ms:.3f} ms, {P / ms / 1e6:.3f} G pairs/s; the filter saves "
            f"{forms['refine_all']['ms'] / forms['filter_refine']['ms']:.2f}x")
    else:
        # every candidate pair tested exactly includes the pairs of two
        # 20k-100k-vertex polygons, whose culled edges are tested all-pairs:
        # not bounded in minutes, so only the filtered forms are timed here
        log("refine all: not timed on the skewed workload (pairs of two complex polygons)")
    out = {"metric": "candidate pairs resolved/s (intermediate filter + exact refinement of indecisive pairs)",
           "value": forms["filter_refine"]["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": forms["filter_refine"]["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i64",
           "data": "synthetic",
           "config": {"workload": ("scale: 200k x 200k star polygons, grid 2^16, all MBR candidate pairs"
                                   if args.workload == "scale" else
                                   "skewed: scale plus 2000 polygons of 20k-100k vertices per side, "
                                   "grid 2^16, all MBR candidate pairs"),
                      "pairs": P, "indecisive": int(len(ind))},
           "forms": forms,
           "filter_speedup": (forms["refine_all"]["ms"] / forms["filter_refine"]["ms"]
                              if "refine_all" in forms else None)}
    if not args.no_cpu_baseline:
        import oracle
        order = np.random.default_rng(3).permutation(ind)
        done, t_cpu, hits = 0, 0.0, 0
        while t_cpu < args.cpu_seconds and done < len(order):
            blk = order[done:done + 2000]
            t1 = time.perf_counter()
            for p in blk:
                hits += oracle.polygons_intersect(R.polygon(int(r_np[p])), S.polygon(int(s_np[p])))
            t_cpu += time.perf_counter() - t1
            done += len(blk)
        out["cpu_baseline"] = {"value": done / t_cpu, "unit": "indecisive pairs/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{done} random indecisive pairs, one exact test per call "
                                         f"({t_cpu:.1f} s)"}
        log(f"cpu baseline: {done / t_cpu / 1e3:.1f} K indecisive pairs/s on one thread")
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the filter runs on a single MI355X; see the design notes on sharding)",
              file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.refine:
        refine_bench(args)
        return
    if args.build:
        build_bench(args)
        return
    if args.variants:
        variants_bench(args)
        return
    if args.partitioned:
        if args.copy_calibration:
            calibration_copies()
        partitioned_bench(args)
        return
    import torch

    import synth
    from paper_2307_01716_amd import april

    assert torch.cuda.is_available(), "no HIP device"
    dev = april.april_device_info()
    log(f"device: {dev['name']} {dev['arch']} CUs={dev['compute_units']}")
    if args.workload == "skewed":
        if args.copy_calibration:
            calibration_copies()
        sk = skewed_leg(args, torch.cuda.current_stream())
        b = sk["batched"]
        print(json.dumps({"metric": "candidate pairs filtered/s (skewed workload, batched, hipGraph replay)",
                          "value": b["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": b["steps"],
                          "warmup": args.warmup, "ms_per_step": b["kernel_ms"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
                          "config": {"workload": sk["workload"], "pairs": sk["pairs"]}, "forms": {"skewed": sk}}),
              flush=True)
        return

    t0 = time.time()
    R, S, g = synth.configs.scale()
    log(f"generated R={len(R)} S={len(S)} in {time.time() - t0:.1f}s")
    t0 = time.time()
    hR = april.april_build_lists(g, R.xy, R.voff, april.STRICT)
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    log(f"built lists (A={hR.info().n_a + hS.info().n_a}, F={hR.info().n_f + hS.info().n_f}) "
        f"in {time.time() - t0:.1f}s")
    t0 = time.time()
    r_np, s_np = april.april_mbr_join(R.mbrs(), S.mbrs())
    P = len(r_np)
    log(f"MBR join: {P} candidate pairs in {time.time() - t0:.1f}s")

    stream = torch.cuda.current_stream()
    dR = april.april_lists_to_device(hR, stream=stream)
    dS = april.april_lists_to_device(hS, stream=stream)
    r = torch.from_numpy(r_np.view(np.int32)).cuda()
    s = torch.from_numpy(s_np.view(np.int32)).cuda()
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.zeros(3, dtype=torch.int64, device="cuda")
    by = torch.empty(P, dtype=torch.int64, device="cuda")
    april.april_alg2_bytes(dR, dS, r, s, by, stream=stream)
    torch.cuda.synchronize()
    alg_bytes = int(by.sum().item())
    del by
    log(f"Alg. 2 bytes per launch: {alg_bytes / 1e9:.3f} GB ({alg_bytes / P:.0f} B/pair)")

    def timed(fn, steps, warmup):
        """W untimed calls, then K timed ones; per-call HIP event times (ms)
        on the launch stream and the wall time of the K calls."""
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return np.array([a.elapsed_time(b) for a, b in ev]), wall

    def form(name, launch_ms, wall):
        ms = wall * 1e3 / args.steps
        c = counts.cpu().numpy()
        assert int(c.sum()) == P, f"{name}: counts do not cover every pair"
        d = {"ms_per_step": ms, "kernel_ms": float(launch_ms.mean()),
             "kernel_ms_median": float(np.median(launch_ms)),
             "kernel_ms_p10": float(np.percentile(launch_ms, 10)),
             "kernel_ms_p90": float(np.percentile(launch_ms, 90)),
             "pairs_per_s": P / (ms / 1e3),
             "alg_GBps": alg_bytes / (launch_ms.mean() / 1e3) / 1e9,
             "verdicts": {"TN": int(c[0]), "TH": int(c[1]), "IND": int(c[2])}}
        log(f"{name}: {ms:.3f} ms/step, kernel {d['kernel_ms']:.3f} ms (p10 {d['kernel_ms_p10']:.3f} "
            f"p90 {d['kernel_ms_p90']:.3f}); {d['pairs_per_s'] / 1e9:.3f} G pairs/s; "
            f"{d['alg_GBps']:.0f} GB/s algorithmic; TN/TH/IND = {c.tolist()}")
        return d

    if args.copy_calibration:
        calibration_copies()

    forms = {}
    if args.schedule in ("both", "plain"):
        def plain():
            april.april_filter_pairs(dR, dS, r, s, verdict, counts, schedule=april.SCHED_PLAIN,
                                     stream=stream)
        forms["plain"] = form("plain", *timed(plain, args.steps, args.warmup))
        plain_verdict = verdict.clone()

    if args.schedule in ("both", "batched"):
        from paper_2307_01716_amd import tune
        ws = torch.empty(april.april_filter_workspace_size(P), dtype=torch.uint8, device="cuda")
        cfg, kw, tune_src = {}, {}, "library defaults"
        sig = tune.signature(P, dR, dS)
        stored = tune.load(args.tune_table, tune.device_key(), sig)
        if args.config:
            cfg = {k: int(v) for k, v in (kv.split("=") for kv in args.config.split(","))}
            tune_src = "--config"
        elif stored is not None and not args.retune:
            cfg, tune_src = stored, "tuning table"
        elif not args.no_tune:
            cfg, tune_src = autotune(tune, dR, dS, r, s, verdict, counts, ws, sig, args)
        kw = tune.call_config(cfg)
        log(f"batched setting {cfg} ({tune_src})")

        def batched_eager():
            april.april_filter_pairs(dR, dS, r, s, verdict, counts, schedule=april.SCHED_BATCHED,
                                     workspace=ws, stream=stream, **kw)

        if args.no_graph:
            fn = batched_eager
        else:
            batched_eager()
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            cap = torch.cuda.Stream()
            cap.wait_stream(stream)
            with torch.cuda.stream(cap):
                with torch.cuda.graph(graph, stream=cap):
                    april.april_filter_pairs(dR, dS, r, s, verdict, counts,
                                             schedule=april.SCHED_BATCHED, workspace=ws,
                                             stream=torch.cuda.current_stream(), **kw)
            torch.cuda.synchronize()
            fn = graph.replay
        forms["batched"] = form("batched", *timed(fn, args.steps, args.warmup))
        forms["batched"]["tuning"] = cfg
        forms["batched"]["tuning_source"] = tune_src
        forms["batched"]["hipgraph"] = not args.no_graph
        if not args.no_random_order:
            # the same pairs in a seeded random order (no spatial locality
            # between consecutive pairs); verdicts must follow the permutation
            perm = torch.from_numpy(np.random.default_rng(0).permutation(P)).to(r.device)
            rp, sp = r[perm].contiguous(), s[perm].contiguous()
            vp = torch.empty_like(verdict)

            def batched_random():
                april.april_filter_pairs(dR, dS, rp, sp, vp, counts, schedule=april.SCHED_BATCHED,
                                         workspace=ws, stream=stream, **kw)

            rnd_ms, _ = timed(batched_random, max(3, args.steps // 4), 1)
            assert torch.equal(vp, verdict[perm]), "random-order verdicts differ"
            forms["batched"]["random_order_kernel_ms"] = float(np.median(rnd_ms))
            log(f"batched, pairs in random order: {forms['batched']['random_order_kernel_ms']:.3f} ms")
            del rp, sp, vp, perm
        if "plain" in forms:
            assert torch.equal(verdict, plain_verdict), "batched and plain verdicts differ"
            forms["batched"]["speedup_vs_plain"] = (forms["plain"]["kernel_ms"] /
                                                    forms["batched"]["kernel_ms"])
            log(f"batched / plain speedup: {forms['batched']['speedup_vs_plain']:.2f}x")

    main_form = "batched" if "batched" in forms else "plain"
    f = forms[main_form]
    # HBM traffic per launch from the committed rocprofv3 counters, when they
    # were taken on this kernel's current sources with this configuration
    from paper_2307_01716_amd import profiling
    kname = "k_batched" if main_form == "batched" else "k_filter_plain"
    tr_cfg = f.get("tuning", {}) if main_form == "batched" else {}
    traffic = profiling.read_traffic(os.path.join(HERE, "profiles", f"{kname}_scale200k_traffic.txt"),
                                     kname, tr_cfg, P) if args.workload == "scale" else None
    if "plain" in forms:
        forms["plain"]["traffic_bytes"] = profiling.read_traffic(
            os.path.join(HERE, "profiles", "k_filter_plain_scale200k_traffic.txt"), "k_filter_plain", {}, P)
    # VALU issue (the kernels' instruction counts from the same records)
    if args.workload == "scale":
        for fname, kn, kc in (("batched", "k_batched", forms.get("batched", {}).get("tuning", {})),
                              ("plain", "k_filter_plain", {})):
            if fname in forms:
                forms[fname]["valu"] = profiling.read_valu(
                    os.path.join(HERE, "profiles", f"{kn}_scale200k_valu.txt"), kn, kc, P,
                    forms[fname]["kernel_ms"])
    out = {
        "metric": "candidate pairs filtered/s (" + (
            "batched persistent schedule, hipGraph replay" if main_form == "batched"
            else "plain, one wavefront per pair") + ")",
        "value": f["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": ("scale: 200k x 200k star polygons, grid 2^16, all MBR candidate pairs"
                                if args.workload == "scale" else
                                "skewed: 200k x 200k star polygons plus 2000 x 2000 with 20k-100k vertices "
                                "(radius 0.02-0.1), grid 2^16, all MBR candidate pairs"),
                   "pairs": P, "schedule": main_form, "verdicts": f["verdicts"]},
        "forms": forms,
        "alg_bytes_per_launch": alg_bytes,
        "roofline": {"bound": "hbm", "achieved": f["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": f["alg_GBps"] / HBM_PEAK_GBS, "traffic": traffic},
    }
    # the oracle's brute-force list builder cannot sample the skewed workload
    # (its large polygons cover up to 10^8 cells each)
    if not args.no_cpu_baseline and args.workload == "scale":
        t0 = time.time()
        out["cpu_baseline"] = cpu_baseline(R, S, g, args.cpu_seconds)
        log(f"cpu baseline: {out['cpu_baseline']['value'] / 1e6:.2f} M pairs/s "
            f"on {out['cpu_baseline']['cores']} threads ({time.time() - t0:.1f}s)")
    if not args.no_skewed and args.workload == "scale":
        del dR, dS
        torch.cuda.synchronize()
        out["forms"]["skewed"] = skewed_leg(args, stream)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
