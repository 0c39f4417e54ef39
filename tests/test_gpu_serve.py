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
    assert stats["completed"] == len(reqs) and stats["deferred_admissions"] > 0 and stats["admissions"] == len(reqs)
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


def test_mixed_equals_alone_full_size_requests():
    """Requests of the serving workload's full size (up to 200 sources, patch sides up to
    96 px, 5 bands, uncropped): each result in the mix equals its result alone, bitwise."""
    say("case: serving mix vs alone, full-size requests")
    sizes = [200, 137, 61, 1, 18]
    reqs = [serve.Request(i, gen.config5_request(2000 + i, n_sources=n), arrival=0.0, rounds=3)
            for i, n in enumerate(sizes)]
    reqs[3].cancel_after_rounds = 1
    alone = [serve.solo(r.prob, rounds=3) for r in reqs]
    srv = serve.Server(0, rounds=3)
    stats = srv.run(reqs, realtime=False)
    say(f"  {stats}")
    assert stats["completed"] == len(reqs) - 1
    for r, a in zip(reqs, alone):
        if r.cancelled:
            continue
        assert np.array_equal(r.result_theta, a.result_theta), r.rid
        assert np.array_equal(r.result_local, a.result_local, equal_nan=True), r.rid
        assert np.array_equal(r.result_status, a.result_status), r.rid


def test_appended_plan_equals_merged_plan():
    """A plan built by appending requests one at a time (cel_plan_append) gives the same
    ELBO, local objectives, gradients and Newton step as one prepared from the merged
    problem, bit for bit (per-source reductions have a fixed order), including after the
    appends outgrow the plan's capacities."""
    say("case: appended plan vs merged plan")
    from paper_1803_00113_amd import api
    probs = [gen.crop_patches(gen.config5_request(3000 + i, n_sources=n), 40) for i, n in enumerate([5, 30, 2, 60])]
    ctx = api.Context(0)
    plan = api.Plan(ctx, probs[0])
    th0 = torch.as_tensor(probs[0].theta0, device="cuda").contiguous()
    api.newton_step(plan, th0.clone(), torch.ones(plan.S, dtype=torch.float64, device="cuda"),
                    plan.colours == 0)          # Newton scratch exists before the appends
    for p in probs[1:]:
        first = plan.append(p)
        assert first + p.n_sources == plan.S
    merged = serve.merge(probs)
    merged.pixels = np.concatenate([p.pixels for p in probs])
    ref = api.Plan(ctx, merged)
    assert np.array_equal(plan.colours, ref.colours) and plan.n_units == ref.n_units
    theta = np.vstack([p.theta0 for p in probs])
    a, b = api.elbo_grad(plan, theta), api.elbo_grad(ref, theta)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    mask = plan.colours == 1
    res = []
    for pl in (plan, ref):
        th = torch.as_tensor(theta, device="cuda").contiguous()
        r = torch.ones(pl.S, dtype=torch.float64, device="cuda")
        st, loc = api.newton_step(pl, th, r, mask)
        res.append((th, r, st, loc))
    for x, y in zip(*res):
        assert torch.equal(x, y) if x.dtype != torch.float64 else torch.equal(torch.nan_to_num(x), torch.nan_to_num(y))
    say(f"  {len(probs)} requests, {plan.S} sources, {plan.n_units} pixels: identical")


@pytest.mark.parametrize("opts,variants,fp64", [({}, 2, False), (dict(hessian_fd=True), 56, False),
                                                (dict(hessian_fp64=True), 2, True)])
def test_footprint_bounds_the_plan_allocation(opts, variants, fp64):
    """footprint_bytes is an upper bound of what a request's plan holds after Newton steps
    (cel_plan_info's device bytes on a fresh context), and not a loose one."""
    from paper_1803_00113_amd import api
    prob = gen.config5_request(4000, n_sources=80)
    ctx = api.Context(0, **opts)
    plan = api.Plan(ctx, prob)
    th = torch.as_tensor(prob.theta0, device="cuda").contiguous()
    api.newton_step(plan, th, torch.ones(plan.S, dtype=torch.float64, device="cuda"), plan.colours == 0)
    torch.cuda.synchronize()
    held = plan.device_bytes()
    est = serve.footprint_bytes(prob, variants, fp64)
    say(f"  opts {opts}: held {held / 1e6:.2f} MB, estimate {est / 1e6:.2f} MB")
    assert held <= est <= 1.25 * held
