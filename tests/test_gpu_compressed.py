"""Compressed (delta + VByte) lists, decoded while joining (Sec. 5.1).

* round trip: lists uploaded compressed and decoded on the device by the
  decoder the filter uses equal the original lists bit for bit -- lengths 0,
  1, around the 64-interval block and 256-byte window edges, 10^5, large and
  small gaps (1- to 5-byte varints);
* verdicts on compressed lists equal the oracle's (random lists, the tiny
  workload), with the block-index search forced on and off and every tile
  size, with pairs in random order and grouped by R object, and with the
  decode cache in the caller's workspace.
"""

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from synth.intervals import ListSet, random_lists, sub_lists

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2307_01716_amd import april  # noqa: E402

GRID = (0.0, 0.0, float(1 << 16) * 2.0 ** -30 * (1 << 16), 16)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def collection(rng, lengths, spread):
    A, F = [], []
    for L, sp in zip(lengths, spread):
        lo = int(rng.integers(0, 1 << 24))
        a = random_lists(rng, max(L, 1), lo, min(lo + sp * max(L, 1) + 8, 2 ** 32 - 2))
        if L == 0:
            a = (a[0][:0], a[1][:0])
        A.append(a)
        F.append(sub_lists(rng, *a, p=0.6))
    a, f = ListSet.from_lists(A), ListSet.from_lists(F)
    return oracle.Lists(a.off, a.start, a.end, f.off, f.start, f.end)


def upload(grid, L, codec):
    h = april.april_lists_from_arrays(grid, L.offA, L.sA, L.eA, L.offF, L.sF, L.eF, validate=True)
    d = april.april_lists_to_device(h, codec=codec)
    torch.cuda.synchronize()
    return d


LENGTHS = [0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 1000, 4097, 100_000]


@pytest.mark.parametrize("spread", [3, 200, 70_000, 30_000_000])
def test_round_trip(spread):
    rng = np.random.default_rng(spread)
    lens = LENGTHS * 2
    L = collection(rng, lens, [spread] * len(lens))
    say(f"[vbyte] round trip spread={spread} intervals={len(L.sA)}")
    d = upload(GRID, L, april.CODEC_VBYTE)
    back = april.april_lists_download(d)
    got = back.export()
    for a, b in zip(got, (L.offA, L.sA, L.eA, L.offF, L.sF, L.eF)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("tile,search_min,chunk", [(256, 1, 0), (512, 1024, 0), (1024, 64, 0), (512, 64, 1),
                                                    (1024, 1024, 2), (256, 1, 4)])
def test_random_lists_compressed(tile, search_min, chunk):
    rng = np.random.default_rng(tile + search_min)
    n = 160
    lens = rng.choice([1, 5, 60, 64, 65, 130, 300, 1500, 9000], n)
    spread = rng.choice([3, 40, 2000], n)
    LR, LS = collection(rng, lens, spread), collection(rng, lens[::-1].copy(), spread)
    P = 6000
    r = rng.integers(0, n, P).astype(np.uint32)
    s = rng.integers(0, n, P).astype(np.uint32)
    want = oracle.filter_pairs(LR, LS, r, s)
    say(f"[vbyte] filter tile={tile} search_min={search_min} chunk={chunk} P={P}")
    dR, dS = upload(GRID, LR, april.CODEC_VBYTE), upload(GRID, LS, april.CODEC_VBYTE)
    v = torch.empty(P, dtype=torch.uint8, device="cuda")
    c = torch.empty(3, dtype=torch.int64, device="cuda")
    april.april_filter_pairs(dR, dS, cuda(r), cuda(s), v, c, schedule=april.SCHED_BATCHED, tile=tile,
                             search_min=search_min, chunk=chunk)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), want)
    assert np.array_equal(c.cpu().numpy(), np.bincount(want, minlength=3))
    assert len(set(want.tolist())) == 3
    # pairs grouped by R object: runs of pairs share a decoded R list
    # (objects of up to 4,096 intervals) or decode it per pair (longer ones)
    o = np.argsort(r, kind="stable")
    april.april_filter_pairs(dR, dS, cuda(r[o]), cuda(s[o]), v, c, schedule=april.SCHED_BATCHED, tile=tile,
                             search_min=search_min, chunk=chunk)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), want[o])


def test_decode_cache_in_workspace():
    """APRIL_WS_DECODE_CACHE: the decode cache is the tail of the caller's
    workspace, so the call allocates nothing.  Verdicts equal the oracle's on
    two calls in a row through the same workspace, the second on fewer pairs
    (objects above the cache's 4,096 intervals decode per pair); a workspace
    without room for the cache is refused."""
    rng = np.random.default_rng(21)
    n = 120
    lens = rng.choice([1, 5, 60, 300, 1500, 5000], n)
    spread = rng.choice([3, 40, 2000], n)
    LR, LS = collection(rng, lens, spread), collection(rng, lens[::-1].copy(), spread)
    P = 4000
    r = np.sort(rng.integers(0, n, P)).astype(np.uint32)
    s = rng.integers(0, n, P).astype(np.uint32)
    want = oracle.filter_pairs(LR, LS, r, s)
    dR, dS = upload(GRID, LR, april.CODEC_VBYTE), upload(GRID, LS, april.CODEC_VBYTE)
    nb = april.april_filter_workspace_size(P, flags=april.WS_DECODE_CACHE)
    plain_nb = april.april_filter_workspace_size(P)
    assert nb > plain_nb
    say(f"[vbyte] decode cache in a workspace of {nb} bytes")
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for m in (P, P // 3):
        v = torch.empty(m, dtype=torch.uint8, device="cuda")
        c = torch.empty(3, dtype=torch.int64, device="cuda")
        april.april_filter_pairs(dR, dS, cuda(r[:m]), cuda(s[:m]), v, c, schedule=april.SCHED_BATCHED,
                                 flags=april.WS_DECODE_CACHE, workspace=ws)
        torch.cuda.synchronize()
        assert np.array_equal(v.cpu().numpy(), want[:m])
        assert np.array_equal(c.cpu().numpy(), np.bincount(want[:m], minlength=3))
    v = torch.empty(P, dtype=torch.uint8, device="cuda")
    with pytest.raises(april.AprilError) as e:
        april.april_filter_pairs(dR, dS, cuda(r), cuda(s), v, None, schedule=april.SCHED_BATCHED,
                                 flags=april.WS_DECODE_CACHE, workspace=ws[:plain_nb])
    assert e.value.code == april.E_INVALID
    torch.cuda.synchronize()


def test_tiny_workload_compressed():
    R, S, g = synth.configs.tiny()
    LR, LS = oracle.build_lists(g, R), oracle.build_lists(g, S)
    r, s = oracle.mbr_join(R, S)
    want = oracle.filter_pairs(LR, LS, r, s)
    hR = april.april_build_lists(g, R.xy, R.voff, april.STRICT)
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    dR = april.april_lists_to_device(hR, codec=april.CODEC_VBYTE)
    dS = april.april_lists_to_device(hS, codec=april.CODEC_VBYTE)
    v = torch.empty(len(r), dtype=torch.uint8, device="cuda")
    april.april_filter_pairs(dR, dS, cuda(r), cuda(s), v, schedule=april.SCHED_BATCHED)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), want)
    # the plain schedule refuses compressed lists
    with pytest.raises(april.AprilError):
        april.april_filter_pairs(dR, dS, cuda(r), cuda(s), v)


@pytest.mark.parametrize("parts", [4, 16])
def test_partitioned_compressed_against_oracle(parts):
    """Partitioned join on compressed lists: one launch over every partition's
    pairs; verdicts equal the oracle's partition-by-partition filter."""
    from paper_2307_01716_amd import partitioned
    R, S, g = synth.configs.tiny(n=1500)
    lay = synth.partitions.layout(R, S, parts, 10)
    ro, so, vo = oracle.partitioned_filter(lay, R, S)
    say(f"[partitioned] parts={parts} pairs={len(ro)}")
    hR = partitioned.build_instances(lay, R, "r")
    hS = partitioned.build_instances(lay, S, "s")
    dR = april.april_lists_to_device(hR, codec=april.CODEC_VBYTE)
    dS = april.april_lists_to_device(hS, codec=april.CODEC_VBYTE)
    r, s = partitioned.pairs(lay, R, S)
    v = torch.empty(len(r), dtype=torch.uint8, device="cuda")
    c = torch.empty(3, dtype=torch.int64, device="cuda")
    april.april_filter_pairs(dR, dS, cuda(r), cuda(s), v, c, schedule=april.SCHED_BATCHED)
    torch.cuda.synchronize()
    rg, sg = lay.r_obj[r], lay.s_obj[s]
    k = np.lexsort((sg, rg))
    assert np.array_equal(rg[k], ro) and np.array_equal(sg[k], so)
    assert np.array_equal(v.cpu().numpy()[k], vo)
    assert np.array_equal(c.cpu().numpy(), np.bincount(vo, minlength=3))
    # raw lists of the same partitions give the same verdicts
    dRr = april.april_lists_to_device(hR)
    dSr = april.april_lists_to_device(hS)
    v2 = torch.empty(len(r), dtype=torch.uint8, device="cuda")
    april.april_filter_pairs(dRr, dSr, cuda(r), cuda(s), v2, schedule=april.SCHED_BATCHED)
    torch.cuda.synchronize()
    assert torch.equal(v, v2)


def test_partitioned_config_size_against_oracle():
    """The partitioned workload at its layout: 16 x 16 partitions, each with
    its own grid of order 16, 100k polygons per side of the at-scale
    distribution (a fifth of the benchmark's 500k).  The oracle's brute-force
    builder needs about a second per instance at this resolution, so:
      * the library's partition-local pairs equal the oracle's (same instance
        indices, reference-point rule);
      * the library's lists equal the oracle's on 64 sampled instances per
        side, each built on its own partition's grid;
      * Alg. 2 by the oracle on the library's lists, for every pair, equals
        the GPU verdicts on raw and on compressed lists (one launch each)."""
    from paper_2307_01716_amd import partitioned
    R, S, lay = synth.configs.partitioned(n=100_000)
    say(f"[partitioned-16x16] instances {len(lay.r_obj)} + {len(lay.s_obj)}; host lists")
    hR = partitioned.build_instances(lay, R, "r")
    hS = partitioned.build_instances(lay, S, "s")
    r, s = partitioned.pairs(lay, R, S)
    ro, so = oracle.partitioned_pairs(lay, R, S)
    k = np.lexsort((s, r))
    assert np.array_equal(r[k].astype(np.int64), ro) and np.array_equal(s[k].astype(np.int64), so)
    LR, LS = oracle.Lists(*hR.export()), oracle.Lists(*hS.export())
    rng = np.random.default_rng(44)
    for name, L, P, obj, part in (("r", LR, R, lay.r_obj, lay.r_part()),
                                  ("s", LS, S, lay.s_obj, lay.s_part())):
        pick = rng.choice(len(obj), 64, replace=False)
        say(f"[partitioned-16x16] oracle lists of 64 sampled {name} instances")

        def one(i):
            return oracle.build_lists(lay.grids[int(part[i])], P.subset(np.array([obj[i]])), nthreads=1)
        with ThreadPoolExecutor(oracle.default_threads()) as ex:
            built = list(ex.map(one, pick))
        for i, want in zip(pick, built):
            a0, a1 = int(L.offA[i]), int(L.offA[i + 1])
            f0, f1 = int(L.offF[i]), int(L.offF[i + 1])
            assert np.array_equal(L.sA[a0:a1], want.sA) and np.array_equal(L.eA[a0:a1], want.eA), i
            assert np.array_equal(L.sF[f0:f1], want.sF) and np.array_equal(L.eF[f0:f1], want.eF), i
    say(f"[partitioned-16x16] oracle filter over {len(r)} pairs")
    want = oracle.filter_pairs(LR, LS, r, s)
    assert set(np.unique(want)) == {0, 1, 2}
    for codec in (april.CODEC_RAW, april.CODEC_VBYTE):
        dR = april.april_lists_to_device(hR, codec=codec)
        dS = april.april_lists_to_device(hS, codec=codec)
        v = torch.empty(len(r), dtype=torch.uint8, device="cuda")
        c = torch.empty(3, dtype=torch.int64, device="cuda")
        say(f"[partitioned-16x16] batched, codec={codec}")
        april.april_filter_pairs(dR, dS, cuda(r), cuda(s), v, c, schedule=april.SCHED_BATCHED)
        torch.cuda.synchronize()
        assert np.array_equal(v.cpu().numpy(), want), codec
        assert np.array_equal(c.cpu().numpy(), np.bincount(want, minlength=3)), codec
        dR.free()
        dS.free()


def _varint_prefix_bytes(s, e, k):
    """Bytes of the first k intervals of a list in the stream format: the
    values s0 < e0 < s1 < ... as varint(v_t - v_(t-1) - 1), v_(-1) = 2^32 - 1,
    7 bits per byte."""
    if k == 0:
        return 0
    v = np.empty(2 * k, np.int64)
    v[0::2], v[1::2] = s[:k], e[:k]
    d = (v - np.concatenate([[2 ** 32 - 1], v[:-1]]) - 1) % (2 ** 32)
    return int(np.maximum(1, -(-np.floor(np.log2(np.maximum(d, 1)) + 1).astype(np.int64) // 7)).sum())


def test_alg2_bytes_on_compressed_lists():
    """april_alg2_bytes on compressed lists: for every pair of the tiny
    workload, 8 + 16 per list Alg. 2 opens + the stream bytes of each list's
    prefix that Alg. 2 reads (read counts from the oracle's IntervalJoin,
    sizes from the stream format) + 1."""
    R, S, g = synth.configs.tiny()
    LR, LS = oracle.build_lists(g, R), oracle.build_lists(g, S)
    r, s = oracle.mbr_join(R, S)
    want = np.empty(len(r), np.uint64)
    for p in range(len(r)):
        ar, as_, fr, fs = LR.A(int(r[p])), LS.A(int(s[p])), LR.F(int(r[p])), LS.F(int(s[p]))
        hit, k_ar, k_as = oracle.interval_join(ar, as_)
        k_fr = k_fs = 0
        lists = 2
        if hit:
            lists += 1
            af, k, k_fs = oracle.interval_join(ar, fs)
            k_ar = max(k_ar, k)
            if not af:
                lists += 1
                _, k_fr, k = oracle.interval_join(fr, as_)
                k_as = max(k_as, k)
        want[p] = (8 + 16 * lists + 1 + _varint_prefix_bytes(*ar, k_ar) + _varint_prefix_bytes(*as_, k_as)
                   + _varint_prefix_bytes(*fr, k_fr) + _varint_prefix_bytes(*fs, k_fs))
    dR = upload(g, LR, april.CODEC_VBYTE)
    dS = upload(g, LS, april.CODEC_VBYTE)
    by = torch.zeros(len(r), dtype=torch.int64, device="cuda")
    say(f"[compressed] Alg. 2 bytes over {len(r)} pairs")
    april.april_alg2_bytes(dR, dS, cuda(r), cuda(s), by)
    torch.cuda.synchronize()
    assert np.array_equal(by.cpu().numpy().astype(np.uint64), want)
