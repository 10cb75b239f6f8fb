"""april_filter_pairs_static: the filter entry point that allocates nothing
(its scratch is the library's static device array).  Its verdicts and counts
equal april_filter_pairs' on the same inputs, on two calls in a row, the
second with a smaller input (the array keeps the first call's contents), for
both schedules; it refuses a workspace and compressed lists."""

import sys

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


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


@pytest.fixture(scope="module")
def work():
    R, S, g = synth.configs.tiny(n=1500)
    hR = april.april_build_lists(g, R.xy, R.voff, april.STRICT)
    hS = april.april_build_lists(g, S.xy, S.voff, april.STRICT)
    r, s = april.april_mbr_join(R.mbrs(), S.mbrs())
    return hR, hS, april.april_lists_to_device(hR), april.april_lists_to_device(hS), r, s


def run(fn, dR, dS, r, s, **kw):
    v = torch.full((len(r),), 77, dtype=torch.uint8, device="cuda")
    c = torch.full((3,), -1, dtype=torch.int64, device="cuda")
    fn(dR, dS, cuda(r), cuda(s), v, c, **kw)
    torch.cuda.synchronize()
    return v.cpu().numpy(), c.cpu().numpy()


@pytest.mark.parametrize("schedule", [april.SCHED_PLAIN, april.SCHED_BATCHED])
def test_static_equals_filter_twice(work, schedule):
    hR, hS, dR, dS, r, s = work
    rng = np.random.default_rng(schedule)
    small = np.sort(rng.choice(len(r), len(r) // 3, replace=False))
    want_all = oracle.filter_pairs(oracle.Lists(*hR.export()), oracle.Lists(*hS.export()), r, s)
    for name, (rr, ss) in (("all", (r, s)), ("smaller", (r[small], s[small]))):
        say(f"[static] schedule={schedule} {name}: {len(rr)} pairs")
        a, ca = run(april.april_filter_pairs, dR, dS, rr, ss, schedule=schedule)
        b, cb = run(april.april_filter_pairs_static, dR, dS, rr, ss, schedule=schedule)
        assert np.array_equal(a, b)
        assert np.array_equal(ca, cb)
        want = want_all if name == "all" else want_all[small]
        assert np.array_equal(b, want)
        assert np.array_equal(cb, np.bincount(want, minlength=3))


def test_static_validate_and_refusals(work):
    hR, hS, dR, dS, r, s = work
    say("[static] validation and refusals")
    rr = np.array([0, 1 << 30], np.uint32)
    ss = np.array([0, 0], np.uint32)
    with pytest.raises(april.AprilError) as e:
        run(april.april_filter_pairs_static, dR, dS, rr, ss, flags=april.VALIDATE)
    assert e.value.code == april.E_INVALID
    got, _ = run(april.april_filter_pairs_static, dR, dS, r[:10], s[:10], flags=april.VALIDATE,
                 schedule=april.SCHED_BATCHED)
    want, _ = run(april.april_filter_pairs, dR, dS, r[:10], s[:10])
    assert np.array_equal(got, want)
    ws = torch.empty(april.april_filter_workspace_size(len(r)), dtype=torch.uint8, device="cuda")
    with pytest.raises(april.AprilError) as e:
        run(april.april_filter_pairs_static, dR, dS, r, s, schedule=april.SCHED_BATCHED, workspace=ws)
    assert e.value.code == april.E_INVALID
    cR = april.april_lists_to_device(hR, codec=april.CODEC_VBYTE)
    cS = april.april_lists_to_device(hS, codec=april.CODEC_VBYTE)
    with pytest.raises(april.AprilError) as e:
        run(april.april_filter_pairs_static, cR, cS, r, s, schedule=april.SCHED_BATCHED)
    assert e.value.code == april.E_INVALID
