"""Host logic of the serving loop (no GPU): merging requests and footprint estimates."""
import numpy as np

from synth import gen


def test_merge_offsets_and_footprint():
    from paper_1803_00113_amd import serve
    a = gen.config5_request(11, n_sources=3)
    b = gen.config5_request(12, n_sources=5)
    m = serve.merge([a, b])
    assert m.n_sources == 8
    assert len(m.img_band) == len(a.img_band) + len(b.img_band)
    assert np.array_equal(m.patch_src[:a.n_patches], a.patch_src)
    assert np.array_equal(m.patch_src[a.n_patches:], b.patch_src + 3)
    assert np.array_equal(m.patch_img[a.n_patches:], b.patch_img + len(a.img_band))
    assert np.array_equal(m.patch_off[a.n_patches:], b.patch_off + len(a.pixels))
    assert np.array_equal(m.img_sky_off[len(a.img_band):], b.img_sky_off + len(a.sky_knots))
    assert np.array_equal(m.theta0, np.vstack([a.theta0, b.theta0]))
    assert serve.footprint_bytes(b) > serve.footprint_bytes(a) > 0


def _as_problem(m, probs):
    import dataclasses
    f = {x.name: getattr(m, x.name) for x in dataclasses.fields(gen.Problem) if hasattr(m, x.name)}
    f["pixels"] = np.concatenate([p.pixels for p in probs])
    return gen.Problem(**f)


def test_merged_requests_keep_their_objectives():
    """Merging is exact: the oracle's per-source objectives of the merged problem equal each
    request's own (requests of one survey share the prior)."""
    from oracle import elbo as E
    from paper_1803_00113_amd import serve
    a = gen.crop_patches(gen.config5_request(21, n_sources=3), 20)
    b = gen.crop_patches(gen.config5_request(22, n_sources=2), 20)
    assert serve.same_model(a, b)
    m = _as_problem(serve.merge([a, b]), [a, b])
    loc_m = E.elbo(E.Model(m), m.theta0, with_total=False)[1].numpy()
    loc_a = E.elbo(E.Model(a), a.theta0, with_total=False)[1].numpy()
    loc_b = E.elbo(E.Model(b), b.theta0, with_total=False)[1].numpy()
    assert np.allclose(loc_m, np.concatenate([loc_a, loc_b]), rtol=1e-13, atol=0)


def test_merge_rejects_different_priors():
    import pytest
    from paper_1803_00113_amd import serve
    a = gen.config5_request(11, n_sources=2)
    b = gen.config2(n_sources=2)
    assert not serve.same_model(a, b)
    with pytest.raises(ValueError):
        serve.merge([a, b])


class _FakeBackend:
    """Stands in for the library in the serving loop's bookkeeping tests: a 'plan' with one
    colour that requests are appended to, and a Newton step that adds 1 to every masked
    source's parameters."""

    def __init__(self):
        self.plans = 0
        self.appends = 0

    def install(self, monkeypatch, serve):
        import torch
        fake = self

        class Ctx:
            def __init__(self, device, **kw):
                self.device = torch.device("cpu")

        class Plan:
            def __init__(self, ctx, prob, pixels_device=None):
                fake.plans += 1
                self.S = prob.n_sources
                self.colours = np.zeros(self.S, np.int32)

            def append(self, prob, pixels_device=None):
                fake.appends += 1
                first = self.S
                self.S += prob.n_sources
                self.colours = np.zeros(self.S, np.int32)
                return first

        def newton_step(plan, theta, radius, mask):
            assert theta.shape[0] == plan.S
            m = torch.as_tensor(mask)
            theta[m] += 1.0
            status = m.to(torch.int32)
            local = torch.where(m, theta[:, 0], torch.full_like(theta[:, 0], float("nan")))
            return status, local

        monkeypatch.setattr(serve.api, "Context", Ctx)
        monkeypatch.setattr(serve.api, "Plan", Plan)
        monkeypatch.setattr(serve.api, "newton_step", newton_step)
        monkeypatch.setattr(serve.torch.cuda, "synchronize", lambda *a, **k: None)


def _reqs(seed0, sizes):
    return [serve_mod().Request(i, gen.crop_patches(gen.config5_request(seed0 + i, n_sources=n), 16), arrival=0.0)
            for i, n in enumerate(sizes)]


def serve_mod():
    from paper_1803_00113_amd import serve
    return serve


def test_server_bookkeeping(monkeypatch):
    """Every finished request carries exactly its own rounds of updates; an admission appends
    to the plan (no new plan), leaving costs nothing; the budget defers admissions."""
    serve = serve_mod()
    fake = _FakeBackend()
    fake.install(monkeypatch, serve)
    reqs = _reqs(300, [2, 3, 4, 5, 6, 7])
    reqs[2].cancel_after_rounds = 1
    fp = sorted(serve.footprint_bytes(r.prob) for r in reqs)
    srv = serve.Server(0, hbm_budget_bytes=2 * (fp[-1] + fp[-2]), rounds=3)
    stats = srv.run(reqs, realtime=False)
    assert stats["completed"] == 5 and stats["cancelled"] == 1
    for r in reqs:
        if r.cancelled:
            assert r.result_theta is None
            continue
        want = np.array(r.prob.theta0, np.float64)
        for _ in range(3):
            want = want + 1.0
        assert np.array_equal(r.result_theta, want), r.rid
        assert np.array_equal(r.result_status, np.ones(r.prob.n_sources, np.int32))
    assert stats["admissions"] == 6 and stats["deferred_admissions"] > 0
    # one plan at the start and one per re-layout; every other admission an append
    assert fake.plans == 1 + stats["rebuilds"]
    # laid out: 6 admissions, plus the requests carried over by each re-layout
    assert fake.plans + fake.appends >= 6


def test_server_relays_out_when_most_of_the_plan_left(monkeypatch):
    """A request that leaves while holding most of the plan's sources triggers one re-layout
    without it; the remaining request's updates are unaffected."""
    serve = serve_mod()
    fake = _FakeBackend()
    fake.install(monkeypatch, serve)
    big, small = _reqs(401, [8, 2])
    big.cancel_after_rounds = 1
    srv = serve.Server(0, rounds=3)
    stats = srv.run([big, small], realtime=False)
    assert stats["completed"] == 1 and stats["cancelled"] == 1
    assert stats["rebuilds"] == 1 and fake.plans == 2 and fake.appends == 1
    want = np.array(small.prob.theta0, np.float64)
    for _ in range(3):
        want = want + 1.0
    assert np.array_equal(small.result_theta, want)
    assert srv.plan.S == small.prob.n_sources


def test_admission_timing_is_recorded(monkeypatch):
    """Each admission records its time, the resident sources before it and its own size."""
    serve = serve_mod()
    fake = _FakeBackend()
    fake.install(monkeypatch, serve)
    reqs = _reqs(500, [2, 3, 4, 2])
    srv = serve.Server(0, rounds=50)
    pending = list(reqs)
    srv.step(0.0, pending)
    assert not pending and srv.stats.admissions == 4 and fake.plans == 1 and fake.appends == 3
    assert srv.stats.admit_resident == [0, 2, 5, 9] and srv.stats.admit_sources == [2, 3, 4, 2]
    summ = srv.stats.summary()
    assert "admission_ms" in summ and summ["admission_ms"]["p99"] >= summ["admission_ms"]["p50"] >= 0
