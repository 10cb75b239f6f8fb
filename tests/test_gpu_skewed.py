"""Parity of the batched filter with the oracle on the skewed workload.

The workload is the at-scale one plus 2000 complex polygons per side
(20k-100k vertices, radius 0.02-0.1), so A-lists span 1 to ~2.4 x 10^5
intervals and ~30M candidate pairs reach one launch.  The oracle's
brute-force builder cannot rasterize the complex polygons in bounded time,
so both sides filter the library's host lists (the host builder equals the
oracle's classification on sampled cells of such polygons, and on every
at-scale polygon); the oracle then runs Alg. 2 on:
  * every pair of two complex polygons (~3 x 10^5 pairs, the longest joins);
  * a seeded sample of 10^6 of all pairs.
The GPU side is the library's default batched launch for this workload, run
eagerly and as replays of a captured hipGraph, and the other schedules.
The host lists of 20 complex polygons are checked on 10^6 sampled cells
each against the oracle's brute-force classification.
"""

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2307_01716_amd import april  # noqa: E402

N_SMALL = 200_000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


@pytest.fixture(scope="module")
def skewed():
    say("[skewed] generating 202k x 202k polygons")
    R, S, g = synth.configs.skewed()
    say("[skewed] host lists")
    hR = april.april_build_lists(g, R.xy, R.voff, april.STRICT)
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    r, s = april.april_mbr_join(R.mbrs(), S.mbrs())
    say(f"[skewed] {len(r)} pairs; upload")
    dR = april.april_lists_to_device(hR)
    dS = april.april_lists_to_device(hS)
    LR, LS = oracle.Lists(*hR.export()), oracle.Lists(*hS.export())
    # 20 of R's complex polygons for the sampled-cell check of the lists
    picks = np.sort(np.random.default_rng(34).choice(np.arange(N_SMALL, len(R)), 20, replace=False))
    big_polys = [(int(k), R.polygon(int(k)).copy()) for k in picks]
    del R, S
    big = np.nonzero((r >= N_SMALL) & (s >= N_SMALL))[0]
    rng = np.random.default_rng(33)
    sample = np.unique(np.concatenate([big, rng.choice(len(r), 1_000_000, replace=False)]))
    say(f"[skewed] oracle over {len(big)} complex x complex pairs + a sample: {len(sample)} pairs")
    want = oracle.filter_pairs(LR, LS, r[sample], s[sample])
    torch.cuda.synchronize()
    return r, s, dR, dS, LR, LS, big, sample, want, g, big_polys


def _check(got, cnt, r, sample, want):
    assert np.array_equal(got[sample], want)
    assert np.array_equal(cnt, np.bincount(got, minlength=3))
    assert cnt.sum() == len(r)


def test_skewed_lists_shape(skewed):
    """The workload reaches what it is for: A-lists from 1 to beyond 10^5
    intervals, and every outcome among the complex pairs."""
    r, s, dR, dS, LR, LS, big, sample, want = skewed[:9]
    n = np.diff(LR.offA.astype(np.int64))
    assert n.min() >= 1 and n.max() > 100_000
    assert len(big) > 100_000
    wb = want[np.searchsorted(sample, big)]
    assert set(np.unique(wb)) == {0, 1, 2}


def test_skewed_default_launch_and_graph(skewed):
    """The library's default batched launch, eager, then replayed from a
    hipGraph with a caller workspace: every sampled verdict (all complex x
    complex pairs among them) equals the oracle's; replays equal the eager
    run on every pair."""
    r, s, dR, dS, LR, LS, big, sample, want = skewed[:9]
    P = len(r)
    rt, st = cuda(r), cuda(s)
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    say("[skewed] default batched launch")
    april.april_filter_pairs(dR, dS, rt, st, verdict, counts, schedule=april.SCHED_BATCHED)
    torch.cuda.synchronize()
    eager = verdict.cpu().numpy()
    _check(eager, counts.cpu().numpy(), r, sample, want)
    ws = torch.empty(april.april_filter_workspace_size(P), dtype=torch.uint8, device="cuda")
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    say("[skewed] graph capture")
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            april.april_filter_pairs(dR, dS, rt, st, verdict, counts, schedule=april.SCHED_BATCHED,
                                     workspace=ws, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(2):
        verdict.fill_(99)
        counts.fill_(-1)
        torch.cuda.synchronize()
        say(f"[skewed] graph replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(verdict.cpu().numpy(), eager), rep
        assert np.array_equal(counts.cpu().numpy(), np.bincount(eager, minlength=3)), rep


SCHEDULES = {
    "batched-tile256": dict(schedule=april.SCHED_BATCHED, tile=256),
    "batched-tile128-narrow": dict(schedule=april.SCHED_BATCHED, tile=128, chunk=1, search_min=64),
    "batched-workgroup-all": dict(schedule=april.SCHED_BATCHED, tile=256, wg_min=1),
    "batched-no-workgroup": dict(schedule=april.SCHED_BATCHED, tile=512, wg_min=0xFFFFFFFF),
}


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_skewed_other_schedules(skewed, sched):
    r, s, dR, dS, LR, LS, big, sample, want = skewed[:9]
    P = len(r)
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    say(f"[skewed] {sched}")
    april.april_filter_pairs(dR, dS, cuda(r), cuda(s), verdict, counts, **SCHEDULES[sched])
    torch.cuda.synchronize()
    _check(verdict.cpu().numpy(), counts.cpu().numpy(), r, sample, want)


def test_skewed_plain_on_sample(skewed):
    """The plain kernel (one wave per pair, merge paths) on the sampled pairs."""
    r, s, dR, dS, LR, LS, big, sample, want = skewed[:9]
    P = len(sample)
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    say(f"[skewed] plain over {P} sampled pairs")
    april.april_filter_pairs(dR, dS, cuda(r[sample]), cuda(s[sample]), verdict, counts)
    torch.cuda.synchronize()
    assert np.array_equal(verdict.cpu().numpy(), want)
    assert np.array_equal(counts.cpu().numpy(), np.bincount(want, minlength=3))


def _member(d, s, e):
    """Is each id in d inside one of the sorted, disjoint intervals [s, e)?"""
    t = np.searchsorted(s, d, side="right").astype(np.int64) - 1
    return (t >= 0) & (d < e[np.maximum(t, 0)])


def test_skewed_lists_on_sampled_cells(skewed):
    """The lists every verdict above rests on, for 20 of the complex
    polygons: 10^6 cells each (half uniform over the polygon's cell window,
    half at and around random points of its edges), each classified by the
    oracle's brute-force closed-cell rule, must be in the A-list iff Partial
    or Full and in the F-list iff Full."""
    r, s, dR, dS, LR, LS, big, sample, want, g, big_polys = skewed
    rng = np.random.default_rng(35)
    w = g.side / (1 << g.order)

    def cells(xy):
        lo = np.floor((xy.min(axis=0) - (g.x0, g.y0)) / w).astype(np.int64) - 1
        hi = np.floor((xy.max(axis=0) - (g.x0, g.y0)) / w).astype(np.int64) + 1
        uni = np.stack([rng.integers(lo[0], hi[0] + 1, 500_000), rng.integers(lo[1], hi[1] + 1, 500_000)], 1)
        e = rng.integers(0, len(xy), 500_000 // 9 + 1)
        f = rng.random(len(e))[:, None]
        pts = xy[e] * (1 - f) + xy[(e + 1) % len(xy)] * f
        c = np.floor((pts - (g.x0, g.y0)) / w).astype(np.int64)
        near = np.concatenate([c + (di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)])
        return np.concatenate([uni, near])

    jobs = [(k, xy, cells(xy)) for k, xy in big_polys]
    say(f"[skewed] oracle classes of {sum(len(j[2]) for j in jobs)} sampled cells of 20 complex polygons")
    with ThreadPoolExecutor(oracle.default_threads()) as ex:
        classes = list(ex.map(lambda j: oracle.classify_cells(g, j[1], j[2]), jobs))
    seen = set()
    for (k, xy, ij), cls in zip(jobs, classes):
        assert len(ij) >= 1_000_000 and len(xy) >= 20_000
        d = oracle.hilbert(g.order, ij[:, 0], ij[:, 1]).astype(np.uint64)
        a0, a1, f0, f1 = int(LR.offA[k]), int(LR.offA[k + 1]), int(LR.offF[k]), int(LR.offF[k + 1])
        in_a = _member(d, LR.sA[a0:a1].astype(np.uint64), LR.eA[a0:a1].astype(np.uint64))
        in_f = _member(d, LR.sF[f0:f1].astype(np.uint64), LR.eF[f0:f1].astype(np.uint64))
        assert np.array_equal(in_a, cls != 0), k
        assert np.array_equal(in_f, cls == 2), k
        seen |= set(np.unique(cls).tolist())
    assert seen == {0, 1, 2}
