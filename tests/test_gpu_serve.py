"""Served selection queries (Sec. 4.3.1): continuous batching on the GPU.

* with S = 200k polygons and 300 queries of 10-10^4 vertices, every
  result equals, bit for bit, the oracle's answer for that query: the S
  objects whose closed MBR meets the query's, with Alg. 2's verdicts on the
  oracle's own lists;
* a request's result is the same alone and in a mix of concurrent requests;
* a request larger than a slot fails with APRIL_E_NOMEM without disturbing
  the others; cancelled requests disappear; unknown tickets are errors;
* query lists built on the GPU (every query, or the large ones by default)
  give the same results as lists built on the host.
"""

import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2307_01716_amd import april  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def served():
    S, Q, g = synth.configs.serving(n_s=200_000, n_queries=300)
    say(f"[serve] S={len(S)} queries={len(Q)}")
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    dS = april.april_lists_to_device(hS)
    torch.cuda.synchronize()
    return S, Q, g, hS, dS


def oracle_answers(S, Q, g):
    """Per query (s ids ascending, verdicts), from the oracle alone: its own
    lists of S and of every query (brute-force classification, one query
    per thread), the closed-MBR pairs, Alg. 2 on each pair."""
    LS = oracle.build_lists(g, S)

    def one(k):
        poly = np.ascontiguousarray(Q.polygon(k))
        return oracle.build_lists(g, synth.PolygonSet(poly, np.array([0, len(poly)], np.int64)), nthreads=1)
    # the largest queries first, so that no thread is left with one at the end
    mb = Q.mbrs()
    order = np.argsort(-(mb[:, 2] - mb[:, 0]) * (mb[:, 3] - mb[:, 1]) * np.diff(Q.voff))
    with ThreadPoolExecutor(oracle.default_threads()) as ex:
        built = dict(zip(order.tolist(), ex.map(one, order.tolist())))
    q, s = oracle.mbr_join(Q, S)
    out = []
    for k in range(len(Q)):
        sk = s[q == k]
        v = oracle.filter_pairs(built[k], LS, np.zeros(len(sk), np.uint32), sk)
        out.append((sk, v))
    return out


def test_alone_equals_mix_and_oracle(served):
    S, Q, g, hS, dS = served
    srv = april.Server(dS, S.mbrs(), slots=3, mem_budget=256 << 20)
    try:
        say("[serve] alone")
        alone = []
        for k in range(40):
            t = srv.submit(Q.polygon(k))
            r = srv.wait(t, 120)
            alone.append(r)
            srv.release(t)
        say("[serve] mix")
        tickets = [srv.submit(Q.polygon(k)) for k in range(len(Q))]
        mix = [srv.wait(t, 300) for t in tickets]
        for t in tickets:
            srv.release(t)
        for k in range(40):
            assert np.array_equal(alone[k].s_ids, mix[k].s_ids), k
            assert np.array_equal(alone[k].verdict, mix[k].verdict), k
        say("[serve] oracle answers for every query")
        want = oracle_answers(S, Q, g)
        for k in range(len(Q)):
            s, v = want[k]
            assert np.array_equal(mix[k].s_ids, s), k
            assert np.array_equal(mix[k].verdict, v), k
            assert mix[k].counts == np.bincount(v, minlength=3).tolist()
        total = sum(len(r.s_ids) for r in mix)
        assert total > 100_000
        allv = np.concatenate([w[1] for w in want])
        assert set(np.unique(allv)) == {0, 1, 2}
        lat = np.array([r.latency for r in mix])
        assert np.all(lat > 0)
        say(f"[serve] {total} pairs; p50 {np.median(lat) * 1e3:.1f} ms")
    finally:
        srv.close()


def test_gpu_built_queries_equal_host_built(served):
    S, Q, g, hS, dS = served
    results = {}
    for name, cells in (("host", 0xFFFFFFFF), ("gpu", 1)):
        srv = april.Server(dS, S.mbrs(), slots=3, mem_budget=256 << 20, gpu_build_cells=cells)
        try:
            say(f"[serve] all queries built on the {name}")
            tickets = [srv.submit(Q.polygon(k)) for k in range(len(Q))]
            results[name] = [srv.wait(t, 300) for t in tickets]
            for r in results[name]:
                assert r.status == april.OK
            results[name] = [(r.s_ids.copy(), r.verdict.copy()) for r in results[name]]
            for t in tickets:
                srv.release(t)
        finally:
            srv.close()
    for k, (a, b) in enumerate(zip(results["host"], results["gpu"])):
        assert np.array_equal(a[0], b[0]), k
        assert np.array_equal(a[1], b[1]), k


def test_admission_limits_and_cancel(served):
    S, Q, g, hS, dS = served
    # a budget so small that the largest queries cannot fit one slot
    srv = april.Server(dS, S.mbrs(), slots=2, mem_budget=2 << 20)
    try:
        st = srv.stats()
        assert st["slots"] == 2 and st["cap_pairs"] >= 1024
        tickets = [srv.submit(Q.polygon(k)) for k in range(60)]
        ok = nomem = 0
        for t in tickets:
            try:
                srv.wait(t, 120)
                ok += 1
            except april.AprilError as e:
                assert e.code == april.E_NOMEM
                nomem += 1
            srv.release(t)
        assert ok > 0 and nomem > 0
        say(f"[serve] admission: {ok} served, {nomem} rejected")
        # cancel: the ticket disappears
        t = srv.submit(Q.polygon(0))
        srv.cancel(t)
        with pytest.raises(april.AprilError):
            srv.poll(t)
        with pytest.raises(april.AprilError):
            srv.poll(10 ** 9)
        # bad polygon: outside the grid
        bad = np.array([[-5.0, -5.0], [-4.0, -5.0], [-4.0, -4.0]])
        t = srv.submit(bad)
        with pytest.raises(april.AprilError) as e:
            srv.wait(t, 60)
        assert e.value.code == april.E_GRID
        srv.release(t)
    finally:
        srv.close()
