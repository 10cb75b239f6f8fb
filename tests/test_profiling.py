"""Host logic of the profile summaries that bench.py reads (no GPU needed).

* kernel names lose return type, namespaces and argument lists but keep
  template arguments;
* a traffic record counts only while it was taken on the kernel's current
  sources, with the same launch configuration and workload size;
* the copy calibration scales FETCH_SIZE / WRITE_SIZE by what a copy of known
  size reads for them;
* VALU records sum the instruction counts of a launch's kernels, and their
  issue fraction is instructions per second over 256 x 4 SIMDs issuing one
  wave64 instruction per 4 cycles at 2.4 GHz.
"""

import csv
import json
import os

from paper_2307_01716_amd import profiling


def test_short_name():
    n = "void april::(anonymous namespace)::k_batched<512, 2>(april::(anonymous namespace)::BatchArgs)"
    assert profiling.short_name(n) == "k_batched<512, 2>"
    assert profiling.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"
    assert profiling.short_name("april::(anonymous namespace)::k_bin(april::X, unsigned int)") == "k_bin"


def _write_counters(d, name, rows):
    os.makedirs(d / name, exist_ok=True)
    with open(d / name / f"{name}_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for disp, kern, ctr, val in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": kern, "Counter_Name": ctr, "Counter_Value": val})


def test_traffic_calibration(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    kern = "void april::(anonymous namespace)::k_batched<512, 2>(april::(anonymous namespace)::BatchArgs)"
    # a 1 GiB copy reads FETCH_SIZE = 0.5 GiB and WRITE_SIZE = 1 GiB (in KiB);
    # counters come per dimension and are summed
    _write_counters(tmp_path, "fetch", [(1, copy, "FETCH_SIZE", 262144), (1, copy, "FETCH_SIZE", 262144),
                                        (2, kern, "FETCH_SIZE", 1000.0), (3, kern, "FETCH_SIZE", 3000.0)])
    _write_counters(tmp_path, "write", [(1, copy, "WRITE_SIZE", 1048576), (2, kern, "WRITE_SIZE", 10.0),
                                        (3, kern, "WRITE_SIZE", 30.0)])
    t = profiling.traffic(str(tmp_path / "fetch"), str(tmp_path / "write"), "k_batched")
    assert abs(t["fetch_factor"] - 2.0) < 1e-12 and abs(t["write_factor"] - 1.0) < 1e-12
    assert t["fetch_bytes"] == 2000.0 * 1024 * 2.0      # mean of the two launches, KiB, scaled
    assert t["write_bytes"] == 20.0 * 1024
    assert t["dispatches"] == 2


def test_read_traffic_requires_matching_sources(tmp_path):
    rec = {"kernel": "k_batched", "config": {}, "pairs": 10, "alg_bytes": 0,
           "source_sha256": profiling.source_digest("k_batched"),
           "traffic": {"traffic_bytes": 123.0}, "command": ""}
    p = tmp_path / "t.txt"
    p.write_text(json.dumps(rec))
    assert profiling.read_traffic(str(p), "k_batched", {}, 10) == 123.0
    assert profiling.read_traffic(str(p), "k_batched", {"tile": 256}, 10) is None
    assert profiling.read_traffic(str(p), "k_batched", {}, 11) is None
    rec["source_sha256"] = "0" * 64
    p.write_text(json.dumps(rec))
    assert profiling.read_traffic(str(p), "k_batched", {}, 10) is None
    assert profiling.read_traffic(str(tmp_path / "missing.txt"), "k_batched", {}, 10) is None


def test_committed_records_name_their_command():
    here = os.path.dirname(os.path.abspath(__file__))
    for name in ("k_batched_scale200k_traffic.txt", "k_filter_plain_scale200k_traffic.txt"):
        with open(os.path.join(here, "..", "profiles", name)) as f:
            rec = json.load(f)
        assert "rocprofv3 --pmc FETCH_SIZE" in rec["command"] and "rocprofv3 --pmc WRITE_SIZE" in rec["command"]
        assert rec["traffic"]["traffic_bytes"] > 0


def test_valu_record_and_issue_fraction(tmp_path):
    k1 = "void april::(anonymous namespace)::k_bin(april::(anonymous namespace)::BatchArgs, unsigned int)"
    k2 = "void april::(anonymous namespace)::k_batched<512, 4>(april::(anonymous namespace)::BatchArgs)"
    _write_counters(tmp_path, "sq", [(1, k1, "SQ_INSTS_VALU", 100.0), (2, k2, "SQ_INSTS_VALU", 1000.0),
                                     (3, k1, "SQ_INSTS_VALU", 300.0), (4, k2, "SQ_INSTS_VALU", 3000.0)])
    v = profiling.valu(str(tmp_path / "sq"), "k_batched", parts=["k_bin", "k_batched"])
    assert v["insts_per_launch"] == 200.0 + 2000.0 and v["dispatches"] == 2
    assert profiling.VALU_ISSUE_PEAK == 614.4e9
    rec = {"kernel": "k_batched", "config": {}, "pairs": 10, "command": "",
           "source_sha256": profiling.source_digest("k_batched"), "valu": {"insts_per_launch": 614.4e6}}
    p = tmp_path / "v.txt"
    p.write_text(json.dumps(rec))
    got = profiling.read_valu(str(p), "k_batched", {}, 10, kernel_ms=2.0)   # 614.4e6 in 2 ms
    assert abs(got["frac"] - 0.5) < 1e-12 and got["insts_per_pair"] == 61.44e6
    assert profiling.read_valu(str(p), "k_batched", {}, 11, kernel_ms=2.0) is None
