"""GPU: continuous batching.  Requests admitted while others are resident share launches;
each request's result equals its result alone, bitwise (and the loop reports latency)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1803_00113_amd import serve  # noqa: E402
from synth import gen  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def requests(n, rounds=4):
    rng = np.random.default_rng(5)
    out = []
    for i in range(n):
        prob = gen.crop_patches(gen.config5_request(1000 + i, n_sources=int(rng.integers(1, 9))), 28)
        out.append(serve.Request(i, prob, arrival=0.01 * i, rounds=rounds))
    return out


def test_mixed_equals_alone():
    say("case: serving mix vs alone")
    reqs = requests(7)
    alone = [serve.solo(r.prob, rounds=4) for r in reqs]
    # a budget that holds about three requests: the resident mix changes over the run
    fp = sorted(serve.footprint_bytes(r.prob) for r in reqs)
    srv = serve.Server(0, hbm_budget_bytes=fp[-1] + fp[-2] + fp[-3], rounds=4)
    stats = srv.run(reqs, realtime=False)
    say(f"  {stats}")
    assert stats["completed"] == len(reqs) and stats["deferred_admissions"] > 0 and stats["rebuilds"] > 2
    for r, a in zip(reqs, alone):
        assert np.array_equal(r.result_theta, a.result_theta), r.rid
        assert np.array_equal(r.result_local, a.result_local, equal_nan=True), r.rid
        assert np.array_equal(r.result_status, a.result_status), r.rid
        # sources stepped in the last round report their objective, the others NaN
        stepped = r.result_status != 0
        assert np.isfinite(r.result_local[stepped]).all() and np.isnan(r.result_local[~stepped]).all()


def test_realtime_poisson_arrivals():
    say("case: serving realtime")
    rng = np.random.default_rng(9)
    reqs = requests(12, rounds=3)
    t = np.cumsum(rng.exponential(1 / 40.0, len(reqs)))
    for r, a in zip(reqs, t):
        r.arrival = float(a)
    srv = serve.Server(0, rounds=3)
    stats = srv.run(reqs)
    say(f"  {stats}")
    assert stats["completed"] == 12 and stats["p99_ms"] >= stats["p50_ms"] > 0


def test_cancellation_leaves_others_unchanged():
    say("case: serving cancellation")
    reqs = requests(5)
    alone = {r.rid: serve.solo(r.prob, rounds=4) for r in reqs}
    reqs[1].cancel_after_rounds = 2     # leaves while resident
    reqs[3].cancel_after_rounds = 0     # cancelled before admission
    srv = serve.Server(0, rounds=4)
    stats = srv.run(reqs, realtime=False)
    say(f"  {stats}")
    assert stats["completed"] == 3 and stats["cancelled"] == 2
    for r in reqs:
        if r.rid in (1, 3):
            assert r.cancelled and r.result_theta is None
        else:
            assert not r.cancelled
            assert np.array_equal(r.result_theta, alone[r.rid].result_theta), r.rid
