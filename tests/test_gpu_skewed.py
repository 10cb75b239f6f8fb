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
"""

import sys

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
    del R, S
    big = np.nonzero((r >= N_SMALL) & (s >= N_SMALL))[0]
    rng = np.random.default_rng(33)
    sample = np.unique(np.concatenate([big, rng.choice(len(r), 1_000_000, replace=False)]))
    say(f"[skewed] oracle over {len(big)} complex x complex pairs + a sample: {len(sample)} pairs")
    want = oracle.filter_pairs(LR, LS, r[sample], s[sample])
    torch.cuda.synchronize()
    return r, s, dR, dS, LR, LS, big, sample, want


def _check(got, cnt, r, sample, want):
    assert np.array_equal(got[sample], want)
    assert np.array_equal(cnt, np.bincount(got, minlength=3))
    assert cnt.sum() == len(r)


def test_skewed_lists_shape(skewed):
    """The workload reaches what it is for: A-lists from 1 to beyond 10^5
    intervals, and every outcome among the complex pairs."""
    r, s, dR, dS, LR, LS, big, sample, want = skewed
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
    r, s, dR, dS, LR, LS, big, sample, want = skewed
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
}


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_skewed_other_schedules(skewed, sched):
    r, s, dR, dS, LR, LS, big, sample, want = skewed
    P = len(r)
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    say(f"[skewed] {sched}")
    april.april_filter_pairs(dR, dS, cuda(r), cuda(s), verdict, counts, **SCHEDULES[sched])
    torch.cuda.synchronize()
    _check(verdict.cpu().numpy(), counts.cpu().numpy(), r, sample, want)


def test_skewed_plain_on_sample(skewed):
    """The plain kernel (one wave per pair, merge paths) on the sampled pairs."""
    r, s, dR, dS, LR, LS, big, sample, want = skewed
    P = len(sample)
    verdict = torch.empty(P, dtype=torch.uint8, device="cuda")
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    say(f"[skewed] plain over {P} sampled pairs")
    april.april_filter_pairs(dR, dS, cuda(r[sample]), cuda(s[sample]), verdict, counts)
    torch.cuda.synchronize()
    assert np.array_equal(verdict.cpu().numpy(), want)
    assert np.array_equal(counts.cpu().numpy(), np.bincount(want, minlength=3))
