"""Parity of the HIP filter with the oracle (bit-exact verdicts and counts).

Cases:
  * random interval lists with no geometry behind them: lengths 0 .. 10^5
    around the kernel's tile edges, dense and sparse overlap, lists that
    touch everywhere without overlapping (full scans ending in a true
    negative) and the same with one overlap planted near the end;
  * the tiny workload end to end (the library's own lists vs the oracle's,
    verdicts, counts, Alg. 2 byte counts);
  * the at-scale workload (200k x 200k polygons, ~4.7M pairs): the oracle's
    own lists of all 400k polygons equal the library's, and every verdict of
    every schedule (also the benchmark's hipGraph launch and compressed
    lists) equals the oracle's Alg. 2 on its lists;
  * edge cases: no pairs, out-of-range indices, duplicated pairs;
  * lists that went through list files (save, load, upload in both codecs).
"""

import sys

import numpy as np
import pytest

import oracle
import synth
from synth.intervals import ListSet, complement_list, fragmented_sub_lists, random_lists, sub_lists

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2307_01716_amd import april  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).cuda()


def device_lists(grid, lists: oracle.Lists):
    h = april.april_lists_from_arrays(grid, lists.offA, lists.sA, lists.eA, lists.offF, lists.sF,
                                      lists.eF, validate=True)
    d = april.april_lists_to_device(h)
    torch.cuda.synchronize()
    return d


def gpu_filter(LRd, LSd, r, s, **kw):
    P = len(r)
    v = torch.full((max(P, 1),), 77, dtype=torch.uint8, device="cuda")[:P]
    c = torch.full((3,), -1, dtype=torch.int64, device="cuda")
    april.april_filter_pairs(LRd, LSd, cuda(r), cuda(s), v, c, **kw)
    torch.cuda.synchronize()
    return v.cpu().numpy(), c.cpu().numpy()


GRID = (0.0, 0.0, float(1 << 16) * 2.0 ** -30 * (1 << 16), 16)

# schedules under test: plain, batched with defaults, and batched tunings
# that push pairs through every bin and code path (lane-per-pair bin, wave
# bin with either side resident, big pairs with the resident lists cut into
# pieces on one wave or on a workgroup, range search on every streamed list)
SCHEDULES = {
    "plain": dict(schedule=april.SCHED_PLAIN),
    "batched": dict(schedule=april.SCHED_BATCHED),
    "batched-small-tiles": dict(schedule=april.SCHED_BATCHED, tile=128, chunk=1, thread_max=100,
                                search_min=64),
    "batched-wide": dict(schedule=april.SCHED_BATCHED, tile=512, chunk=4, thread_max=1,
                         search_min=1),
    # every pair in which neither object fits a tile runs on a workgroup
    "batched-workgroup": dict(schedule=april.SCHED_BATCHED, tile=128, chunk=1, wg_min=1,
                              search_min=64),
    # no workgroup bin: such pairs run on one wave, piece by piece
    "batched-no-workgroup": dict(schedule=april.SCHED_BATCHED, tile=128, wg_min=0xFFFFFFFF),
}


def _random_collection(rng, n, kind):
    A, F = [], []
    for k in range(n):
        if kind == "edges":
            L = int(rng.choice([0, 1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513,
                                1000, 4095, 4097]))
        elif kind == "long":
            L = int(rng.choice([1, 3, 10_000, 65_536, 100_000]))
        elif kind == "fragmented":
            L = int(rng.choice([1, 2, 5, 40, 300]))
        else:
            L = int(rng.integers(0, 300))
        lo = int(rng.integers(0, 1 << 20))
        span = max(4 * L + 8, int(rng.integers(2 * L + 2, 64 * L + 64)))
        if kind == "fragmented":
            # few A intervals holding many F intervals each: F longer than A
            span = max(span, 4000 * L)
            a = random_lists(rng, max(L, 1), lo, lo + span)
            f = fragmented_sub_lists(rng, *a, max_parts=int(rng.choice([0, 3, 60, 400])))
        else:
            a = random_lists(rng, max(L, 1), lo, lo + span)
            f = sub_lists(rng, *a, p=float(rng.random()))    # F inside A, as for polygons
        A.append(a)
        F.append(f)
    a = ListSet.from_lists(A)
    f = ListSet.from_lists(F)
    return oracle.Lists(a.off, a.start, a.end, f.off, f.start, f.end)


@pytest.mark.parametrize("sched", list(SCHEDULES))
@pytest.mark.parametrize("kind,n,P", [("mixed", 400, 20_000), ("edges", 300, 20_000),
                                      ("long", 12, 150), ("fragmented", 60, 3000)])
def test_random_lists(kind, n, P, sched):
    rng = np.random.default_rng({"mixed": 1, "edges": 2, "long": 3, "fragmented": 4}[kind])
    say(f"[random lists] kind={kind} n={n} P={P} schedule={sched}")
    LR = _random_collection(rng, n, kind)
    LS = _random_collection(rng, n, kind)
    r = rng.integers(0, n, P).astype(np.uint32)
    s = rng.integers(0, n, P).astype(np.uint32)
    want = oracle.filter_pairs(LR, LS, r, s)
    got, cnt = gpu_filter(device_lists(GRID, LR), device_lists(GRID, LS), r, s, **SCHEDULES[sched])
    assert np.array_equal(got, want)
    assert np.array_equal(cnt, np.bincount(want, minlength=3))


@pytest.mark.parametrize("sched", list(SCHEDULES))
@pytest.mark.parametrize("k", [1, 2, 63, 64, 65, 255, 256, 257, 1000, 30_000, 300_000])
def test_touching_lists(k, sched):
    """X against its gaps: no overlap anywhere (a full merge), then the same
    with one gap widened by one cell at a random place (one overlap)."""
    rng = np.random.default_rng(k)
    say(f"[touching] k={k} schedule={sched}")
    X = random_lists(rng, k + 1, 0, 8 * k + 64)
    C = complement_list(*X)
    C2 = (C[0].copy(), C[1].copy())
    C3 = (C[0].copy(), C[1].copy())
    if k >= 1:
        C2[1][-1] += 1            # overlap at the very end of the merge
        t = int(rng.integers(0, k))
        C3[0][t] -= 1             # overlap somewhere inside
    z = (np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    # object 0: X with F = X; objects of S: gaps (A) with F = gaps
    LR = ListSet.from_lists([X]), ListSet.from_lists([X])
    LS = ListSet.from_lists([C, C2, C3, X]), ListSet.from_lists([z, C2, z, z])
    LRo = oracle.Lists(LR[0].off, LR[0].start, LR[0].end, LR[1].off, LR[1].start, LR[1].end)
    LSo = oracle.Lists(LS[0].off, LS[0].start, LS[0].end, LS[1].off, LS[1].start, LS[1].end)
    r = np.zeros(4, np.uint32)
    s = np.arange(4, dtype=np.uint32)
    want = oracle.filter_pairs(LRo, LSo, r, s)
    assert want[0] == oracle.TN and want[1] == oracle.TH and want[3] == oracle.TH
    got, cnt = gpu_filter(device_lists(GRID, LRo), device_lists(GRID, LSo), r, s, **SCHEDULES[sched])
    assert np.array_equal(got, want)
    # roles swapped: the long list on the other side
    got2, _ = gpu_filter(device_lists(GRID, LSo), device_lists(GRID, LRo), s, r, **SCHEDULES[sched])
    assert np.array_equal(got2, want)


@pytest.fixture(scope="module")
def tiny():
    R, S, g = synth.configs.tiny()
    LR = oracle.build_lists(g, R)
    LS = oracle.build_lists(g, S)
    r, s = oracle.mbr_join(R, S)
    v, b = oracle.filter_pairs(LR, LS, r, s, want_bytes=True)
    return R, S, g, LR, LS, r, s, v, b


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_tiny_end_to_end(tiny, sched):
    R, S, g, LR, LS, r, s, v, b = tiny
    say(f"[tiny] pairs={len(r)} schedule={sched}")
    hR = april.april_build_lists(g, R.xy, R.voff, april.STRICT)
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    dR = april.april_lists_to_device(hR)
    dS = april.april_lists_to_device(hS)
    got, cnt = gpu_filter(dR, dS, r, s, **SCHEDULES[sched])
    assert np.array_equal(got, v)
    assert np.array_equal(cnt, np.bincount(v, minlength=3))
    by = torch.zeros(len(r), dtype=torch.int64, device="cuda")
    april.april_alg2_bytes(dR, dS, cuda(r), cuda(s), by)
    torch.cuda.synchronize()
    assert np.array_equal(by.cpu().numpy().astype(np.uint64), b)


def test_tiny_from_list_files(tiny, tmp_path):
    """Lists saved to list files, loaded and uploaded in both codecs give the
    oracle's verdicts."""
    R, S, g, LR, LS, r, s, v, b = tiny
    for name, P in (("r", R), ("s", S)):
        april.april_lists_save(april.april_build_lists(g, P.xy, P.voff, april.STRICT), tmp_path / name)
    hR, hS = april.april_lists_load(tmp_path / "r"), april.april_lists_load(tmp_path / "s")
    for codec in (april.CODEC_RAW, april.CODEC_VBYTE):
        say(f"[tiny] from list files, codec={codec}")
        dR, dS = april.april_lists_to_device(hR, codec), april.april_lists_to_device(hS, codec)
        # compressed lists run on the batched schedule only
        for sched in ("plain", "batched") if codec == april.CODEC_RAW else ("batched",):
            got, cnt = gpu_filter(dR, dS, r, s, **SCHEDULES[sched])
            assert np.array_equal(got, v)
            assert np.array_equal(cnt, np.bincount(v, minlength=3))


def test_tiny_counts_in_pinned_host_memory(tiny):
    """The totals may go to pinned host memory: after the stream is
    synchronized it holds the bincount of the oracle's verdicts, for every
    schedule and codec, and zeros for an empty call."""
    R, S, g, LR, LS, r, s, v, b = tiny
    dR, dS = device_lists(g, LR), device_lists(g, LS)
    vR = april.april_lists_to_device(april.april_lists_download(dR), april.CODEC_VBYTE)
    vS = april.april_lists_to_device(april.april_lists_download(dS), april.CODEC_VBYTE)
    for lists, sched, codec in (((dR, dS), "plain", "raw"), ((dR, dS), "batched", "raw"),
                                ((vR, vS), "batched", "vbyte")):
        say(f"[tiny] counts to pinned host memory, {sched}, {codec}")
        host = torch.full((3,), -1, dtype=torch.int64).pin_memory()
        verdict = torch.empty(len(r), dtype=torch.uint8, device="cuda")
        april.april_filter_pairs(*lists, cuda(r), cuda(s), verdict, host, **SCHEDULES[sched])
        torch.cuda.synchronize()
        assert np.array_equal(host.numpy(), np.bincount(v, minlength=3))
        assert np.array_equal(verdict.cpu().numpy(), v)
    host = torch.full((3,), -1, dtype=torch.int64).pin_memory()
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    april.april_filter_pairs(dR, dS, empty, empty, torch.empty(0, dtype=torch.uint8, device="cuda"), host)
    torch.cuda.synchronize()
    assert host.tolist() == [0, 0, 0]


def test_tiny_waves_and_duplicates(tiny):
    R, S, g, LR, LS, r, s, v, b = tiny
    dR, dS = device_lists(g, LR), device_lists(g, LS)
    rng = np.random.default_rng(9)
    perm = rng.integers(0, len(r), 3 * len(r))          # shuffled, with repeats
    for waves in (1, 7, 64, 100_000):
        say(f"[tiny] waves={waves}")
        got, cnt = gpu_filter(dR, dS, r[perm], s[perm], waves=waves)
        assert np.array_equal(got, v[perm])
        assert np.array_equal(cnt, np.bincount(v[perm], minlength=3))


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_empty_and_bad_pairs(tiny, sched):
    R, S, g, LR, LS, r, s, v, b = tiny
    kw = SCHEDULES[sched]
    dR, dS = device_lists(g, LR), device_lists(g, LS)
    say(f"[edge] no pairs schedule={sched}")
    got, cnt = gpu_filter(dR, dS, np.zeros(0, np.uint32), np.zeros(0, np.uint32), **kw)
    assert len(got) == 0 and np.array_equal(cnt, [0, 0, 0])
    say("[edge] out-of-range indices")
    rr = np.array([0, len(R), 5, 0xFFFFFFFF], np.uint32)
    ss = np.array([0, 0, len(S) + 3, 1], np.uint32)
    got, cnt = gpu_filter(dR, dS, rr, ss, **kw)
    want0 = oracle.filter_pairs(LR, LS, rr[:1], ss[:1])[0]
    assert got[0] == want0
    assert list(got[1:]) == [april.BAD_PAIR] * 3
    assert cnt.sum() == 1
    with pytest.raises(april.AprilError) as e:
        gpu_filter(dR, dS, rr, ss, flags=april.VALIDATE, **kw)
    assert e.value.code == april.E_INVALID
    got, cnt = gpu_filter(dR, dS, r[:50], s[:50], flags=april.VALIDATE, **kw)
    assert np.array_equal(got, v[:50])


def test_grid_mismatch(tiny):
    R, S, g, LR, LS, r, s, v, b = tiny
    dR = device_lists(g, LR)
    other = synth.Grid(g.x0, g.y0, g.side * 2, g.order)
    dS = device_lists(other, LS)
    with pytest.raises(april.AprilError) as e:
        gpu_filter(dR, dS, r[:4], s[:4])
    assert e.value.code == april.E_GRID


@pytest.fixture(scope="module")
def scale():
    say("[scale] generating 200k x 200k")
    R, S, g = synth.configs.scale()
    r, s = april.april_mbr_join(R.mbrs(), S.mbrs())
    hR = april.april_build_lists(g, R.xy, R.voff, april.STRICT)
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    dR = april.april_lists_to_device(hR)
    dS = april.april_lists_to_device(hS)
    torch.cuda.synchronize()
    return R, S, g, r, s, hR, hS, dR, dS


@pytest.fixture(scope="module")
def scale_oracle(scale):
    """The oracle end to end on the whole at-scale workload: its own lists of
    all 400k polygons (brute-force classification) and Alg. 2 on every
    candidate pair."""
    R, S, g, r, s, hR, hS, dR, dS = scale
    say("[scale] oracle lists of all 400k polygons")
    LR = oracle.build_lists(g, R)
    LS = oracle.build_lists(g, S)
    say(f"[scale] oracle filter over all {len(r)} pairs")
    return LR, LS, oracle.filter_pairs(LR, LS, r, s)


def test_scale_lists_equal_oracle(scale, scale_oracle):
    """The library's host lists of every at-scale polygon equal the oracle's."""
    R, S, g, r, s, hR, hS, dR, dS = scale
    LR, LS, _ = scale_oracle
    for h, L in ((hR, LR), (hS, LS)):
        got = h.export()
        want = (L.offA, L.sA, L.eA, L.offF, L.sF, L.eF)
        for a, b in zip(got, want):
            assert np.array_equal(a, b)


def test_scale_pairs_equal_oracle(scale):
    """The library's MBR join gives the oracle's candidate pairs (as a set)."""
    R, S, g, r, s, hR, hS, dR, dS = scale
    ro, so = oracle.mbr_join(R, S)
    k = np.lexsort((s, r))
    assert np.array_equal(r[k], ro) and np.array_equal(s[k], so)


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_scale_every_pair_against_oracle(scale, scale_oracle, sched):
    """Every one of the ~4.7M at-scale verdicts, under each schedule, equals
    the oracle's, and so do the counts; then the same with R and S swapped."""
    R, S, g, r, s, hR, hS, dR, dS = scale
    want = scale_oracle[2]
    say(f"[scale] {sched} over {len(r)} pairs")
    got, cnt = gpu_filter(dR, dS, r, s, **SCHEDULES[sched])
    assert np.array_equal(got, want)
    assert np.array_equal(cnt, np.bincount(want, minlength=3))
    assert set(np.unique(want)) == {0, 1, 2}
    say(f"[scale] {sched} swapped roles")
    got2, cnt2 = gpu_filter(dS, dR, s, r, **SCHEDULES[sched])
    assert np.array_equal(got2, want)
    assert np.array_equal(cnt2, cnt)


def test_scale_graph_launch_against_oracle(scale, scale_oracle):
    """The benchmark's launch: the batched schedule with library defaults and
    a caller workspace, captured in a hipGraph and replayed; every replay's
    verdicts and counts equal the oracle's."""
    R, S, g, r, s, hR, hS, dR, dS = scale
    want = scale_oracle[2]
    P = len(r)
    ws = torch.empty(april.april_filter_workspace_size(P), dtype=torch.uint8, device="cuda")
    rt, st = cuda(r), cuda(s)
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    say("[scale] graph capture")
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            april.april_filter_pairs(dR, dS, rt, st, verdict, counts, schedule=april.SCHED_BATCHED,
                                     workspace=ws, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        verdict.fill_(99)
        counts.fill_(-1)
        torch.cuda.synchronize()
        say(f"[scale] graph replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(verdict.cpu().numpy(), want), rep
        assert np.array_equal(counts.cpu().numpy(), np.bincount(want, minlength=3)), rep


def test_scale_compressed_against_oracle(scale, scale_oracle):
    """The at-scale lists uploaded delta + VByte: every verdict equals the
    oracle's."""
    R, S, g, r, s, hR, hS, dR, dS = scale
    want = scale_oracle[2]
    cR = april.april_lists_to_device(hR, codec=april.CODEC_VBYTE)
    cS = april.april_lists_to_device(hS, codec=april.CODEC_VBYTE)
    say(f"[scale] compressed over {len(r)} pairs")
    got, cnt = gpu_filter(cR, cS, r, s, schedule=april.SCHED_BATCHED)
    assert np.array_equal(got, want)
    assert np.array_equal(cnt, np.bincount(want, minlength=3))
    cR.free()
    cS.free()


def test_batched_workspace_and_graph(tiny):
    """Batched schedule with a caller workspace, captured in a hipGraph and
    replayed several times with eager work in between; every replay must give
    the oracle's verdicts (the pair buffers are refilled between replays)."""
    R, S, g, LR, LS, r, s, v, b = tiny
    dR, dS = device_lists(g, LR), device_lists(g, LS)
    P = len(r)
    nbytes = april.april_filter_workspace_size(P)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    rt, st = cuda(r), cuda(s)
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    say("[graph] eager with workspace")
    april.april_filter_pairs(dR, dS, rt, st, verdict, counts, schedule=april.SCHED_BATCHED,
                             workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(verdict.cpu().numpy(), v)
    say("[graph] capture")
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            april.april_filter_pairs(dR, dS, rt, st, verdict, counts,
                                     schedule=april.SCHED_BATCHED, workspace=ws,
                                     stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    for rep in range(4):
        perm = rng.permutation(P)
        rt.copy_(cuda(r[perm]))
        st.copy_(cuda(s[perm]))
        verdict.fill_(99)
        counts.fill_(-1)
        torch.cuda.synchronize()
        say(f"[graph] replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(verdict.cpu().numpy(), v[perm]), rep
        assert np.array_equal(counts.cpu().numpy(), np.bincount(v, minlength=3)), rep
