"""GPU parity: the HIP path (through the C ABI) against the float64 oracle, element by
element on the same seeded inputs.

Tolerances: ELBO (total and every L_s) |d| <= 1e-5 |oracle|; gradient per source and
component |d| <= 1e-4 max(|o|, 0.01 max_k |o_s,k|).  The float64 pixel path is held to
1e-10 / 1e-8."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import elbo as E  # noqa: E402
from paper_1803_00113_amd import api  # noqa: E402
from synth import gen  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check(prob, tot, loc, g, o_tot, o_loc, o_g, rtol_e=1e-5, rtol_g=1e-4, sources=None):
    idx = np.arange(prob.n_sources) if sources is None else np.asarray(sources)
    if tot is not None:
        assert abs(tot - o_tot) <= rtol_e * abs(o_tot), (tot, o_tot)
    dl = np.abs(loc[idx] - o_loc[idx])
    assert np.all(dl <= rtol_e * np.abs(o_loc[idx])), dl.max()
    if g is not None:
        gg, og = g[idx, :27], o_g[idx, :27]
        floor = 0.01 * np.abs(og).max(axis=1, keepdims=True)
        err = np.abs(gg - og) / np.maximum(np.abs(og), floor)
        assert np.all(err <= rtol_g), (err.max(), np.unravel_index(err.argmax(), err.shape))
        assert np.all(g[idx, 27:] == 0)
        return float(err.max())
    return 0.0


def run(prob, **opts):
    ctx = api.Context(0, **opts)
    plan = api.Plan(ctx, prob)
    tot, loc, g = api.elbo_grad(plan, prob.theta0)
    torch.cuda.synchronize()
    return plan, tot.item(), loc.cpu().numpy(), g.cpu().numpy()


@pytest.fixture(scope="module")
def c1():
    prob = gen.config1()
    return prob, E.elbo_total_and_grad(E.Model(prob), prob.theta0)


def test_config1_fp64_pixels(c1):
    say("case: config1 fp64 pixel path")
    prob, (o_tot, o_loc, o_g) = c1
    _, tot, loc, g = run(prob, pixel_fp64=True)
    check(prob, tot, loc, g, o_tot, o_loc, o_g, rtol_e=1e-10, rtol_g=1e-8)


@pytest.mark.parametrize("ppl", [1, 2, 4])
def test_config1_fp32(c1, ppl):
    say(f"case: config1 fp32 ppl={ppl}")
    prob, (o_tot, o_loc, o_g) = c1
    _, tot, loc, g = run(prob, pixels_per_lane=ppl)
    check(prob, tot, loc, g, o_tot, o_loc, o_g)


def test_eval_matches_grad_and_is_deterministic(c1):
    say("case: config1 eval vs grad, repeat")
    prob, _ = c1
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    t1, l1 = api.elbo_eval(plan, prob.theta0)
    t2, l2, g2 = api.elbo_grad(plan, prob.theta0)
    t3, l3, g3 = api.elbo_grad(plan, prob.theta0)
    t4, l4, g4 = api.elbo_grad_plain(plan, prob.theta0)
    torch.cuda.synchronize()
    assert torch.equal(t1, t2) and torch.equal(l1, l2)
    assert torch.equal(g2, g3) and torch.equal(t2, t3)
    assert torch.equal(g2, g4) and torch.equal(t2, t4) and torch.equal(l2, l4)


@pytest.fixture(scope="module")
def small2():
    # several work items per patch and ragged tails: patches cropped to 40 px (1600 px =
    # 3 items of 512 + 64), groups with overlaps, 4 images over 2 epochs
    prob = gen.crop_patches(gen.subset(gen.config2(n_sources=14), images=[0, 2, 5, 7]), 40)
    return prob, E.elbo_total_and_grad(E.Model(prob), prob.theta0)


@pytest.mark.parametrize("chunk", [64, 512, 4096])
def test_small_batched_fp32(small2, chunk):
    say(f"case: small config2 fp32 chunk={chunk}")
    prob, (o_tot, o_loc, o_g) = small2
    _, tot, loc, g = run(prob, chunk_pixels=chunk)
    err = check(prob, tot, loc, g, o_tot, o_loc, o_g)
    say(f"  max grad rel err {err:.2e}")


def test_tuned_plan_matches_a_plan_built_with_its_settings(small2):
    """cel_tune picks a work-item size, pixels per lane and a moment-map variant for the plan;
    the tuned plan's outputs equal, bit for bit, those of a plan prepared with those settings,
    and stay within the oracle's tolerance."""
    say("case: small config2 launch tuning")
    prob, (o_tot, o_loc, o_g) = small2
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    t = plan.tune(prob.theta0)
    say(f"  tuned: {t}")
    assert t["chunk_pixels"] in (256, 512, 1024, 2048) and t["pixels_per_lane"] in (1, 2, 4)
    assert t["map_pixels_per_lane"] in (1, 2, 4, 8, -1) and t["n_timed"] == 2 * (4 * 3 + 5) and t["ms_per_eval"] > 0
    t1, l1, g1 = api.elbo_grad(plan, prob.theta0)
    fresh, t2, l2, g2 = run(prob, chunk_pixels=t["chunk_pixels"], pixels_per_lane=t["pixels_per_lane"],
                            map_pixels_per_lane=t["map_pixels_per_lane"])
    torch.cuda.synchronize()
    assert plan.n_work_items == fresh.n_work_items
    assert t1.item() == t2 and np.array_equal(l1.cpu().numpy(), l2) and np.array_equal(g1.cpu().numpy(), g2)
    check(prob, t2, l2, g2, o_tot, o_loc, o_g)


def _step(plan, theta, mask):
    th = torch.as_tensor(theta, device="cuda").contiguous()
    r = torch.ones(plan.S, dtype=torch.float64, device="cuda")
    st, loc = api.newton_step(plan, th, r, mask)
    torch.cuda.synchronize()
    return th.cpu().numpy(), r.cpu().numpy(), st.cpu().numpy(), np.nan_to_num(loc.cpu().numpy())


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_retiled_plan_equals_fresh_plans_through_newton_and_append():
    """Re-cutting a plan's work items (cel_tune over one candidate) after Newton steps, to
    more items than its capacity and then to fewer, and appending a request after: each
    time its gradient and Newton step equal those of a plan prepared with the settings."""
    say("case: re-cut work items, Newton steps and an append")
    from paper_1803_00113_amd import serve
    prob = gen.crop_patches(gen.config5_request(3000, n_sources=30), 40)
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    mask = plan.colours == 0
    _step(plan, prob.theta0, mask)                       # Newton scratch exists
    n512 = plan.n_work_items
    for chunk, ppl, mp in ((128, 2, 4), (4096, 4, -1)):
        t = plan.tune(prob.theta0, chunk_pixels=[chunk], pixels_per_lane=[ppl], map_pixels_per_lane=[mp])
        assert (t["chunk_pixels"], t["pixels_per_lane"], t["map_pixels_per_lane"]) == (chunk, ppl, mp)
        ref = api.Plan(api.Context(0, chunk_pixels=chunk, pixels_per_lane=ppl, map_pixels_per_lane=mp), prob)
        assert plan.n_work_items == ref.n_work_items and (plan.n_work_items > n512) == (chunk == 128)
        for x, y in zip(api.elbo_grad(plan, prob.theta0), api.elbo_grad(ref, prob.theta0)):
            assert torch.equal(x, y)
        assert _same(_step(plan, prob.theta0, mask), _step(ref, prob.theta0, mask))
        say(f"  chunk {chunk}: {plan.n_work_items} items, identical")
    extra = gen.crop_patches(gen.config5_request(3100, n_sources=9), 40)
    plan.append(extra)
    merged = serve.merge([prob, extra])
    merged.pixels = np.concatenate([prob.pixels, extra.pixels])
    ref = api.Plan(api.Context(0, chunk_pixels=4096, pixels_per_lane=4, map_pixels_per_lane=-1), merged)
    theta = np.vstack([prob.theta0, extra.theta0])
    assert plan.n_work_items == ref.n_work_items
    for x, y in zip(api.elbo_grad(plan, theta), api.elbo_grad(ref, theta)):
        assert torch.equal(x, y)
    m2 = plan.colours == 1
    assert _same(_step(plan, theta, m2), _step(ref, theta, m2))


@pytest.mark.parametrize("mp", [1, 2, 8, -1])
def test_map_variants_against_oracle(small2, mp):
    """Every moment-map variant (1, 2, 8 pixels per lane, the row-run recurrence; 4 is the
    default every other test runs) stays within the oracle's tolerance."""
    say(f"case: small config2 map variant {mp}")
    prob, (o_tot, o_loc, o_g) = small2
    _, tot, loc, g = run(prob, map_pixels_per_lane=mp)
    err = check(prob, tot, loc, g, o_tot, o_loc, o_g)
    say(f"  max grad rel err {err:.2e}")


def test_small_batched_fp64(small2):
    say("case: small config2 fp64")
    prob, (o_tot, o_loc, o_g) = small2
    _, tot, loc, g = run(prob, pixel_fp64=True)
    check(prob, tot, loc, g, o_tot, o_loc, o_g, rtol_e=1e-10, rtol_g=1e-8)


def test_plain_equals_batched(small2):
    say("case: plain vs batched bitwise")
    prob, _ = small2
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    a = api.elbo_grad(plan, prob.theta0)
    b = api.elbo_grad_plain(plan, prob.theta0)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_edge_cases():
    say("case: edge cases (1x1 patch, source without patches, odd sizes)")
    base = gen.subset(gen.config2(n_sources=5), images=[1, 3])
    prob = gen.crop_patches(base, 23)
    # shrink one patch to 1x1 and one to 1x70 -> rows of 1 pixel
    prob.patch_w = prob.patch_w.copy()
    prob.patch_h = prob.patch_h.copy()
    pix = [prob.patch_pixels(p).copy() for p in range(prob.n_patches)]
    prob.patch_w[0], prob.patch_h[0] = 1, 1
    pix[0] = pix[0][:1, :1]
    prob.patch_w[3], prob.patch_h[3] = 23, 1
    pix[3] = pix[3][:1, :]
    sizes = prob.patch_w.astype(np.int64) * prob.patch_h
    prob.patch_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    prob.pixels = np.concatenate([p.ravel() for p in pix]).astype(np.float32)
    # add a source with no patches at all
    prob = gen.subset(prob)
    prob.n_sources += 1
    prob.theta0 = np.vstack([prob.theta0, prob.theta0[:1]])
    o_tot, o_loc, o_g = E.elbo_total_and_grad(E.Model(prob), prob.theta0)
    _, tot, loc, g = run(prob)
    check(prob, tot, loc, g, o_tot, o_loc, o_g)


def test_empty_problem():
    say("case: empty problem")
    prob = gen.subset(gen.config1(), sources=[])
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    tot, loc, g = api.elbo_grad(plan, np.zeros((0, 32)))
    torch.cuda.synchronize()
    assert tot.item() == 0.0 and loc.numel() == 0 and g.numel() == 0


def test_invalid_problems_rejected():
    say("case: invalid inputs")
    from paper_1803_00113_amd import _ffi
    ctx = api.Context(0)
    prob = gen.config1()
    bad = gen.subset(prob)
    bad.patch_x0 = bad.patch_x0.copy()
    bad.patch_x0[0] = 20            # rectangle leaves the 32x32 image
    with pytest.raises(_ffi.CelError) as e:
        api.Plan(ctx, bad)
    assert e.value.status == _ffi.CEL_EINVAL
    bad = gen.subset(prob)
    bad.patch_src = bad.patch_src[::-1].copy()   # unsorted
    with pytest.raises(_ffi.CelError):
        api.Plan(ctx, bad)
    bad = gen.subset(prob)
    bad.sky_knots = bad.sky_knots * 0.0           # non-positive sky
    with pytest.raises(_ffi.CelError):
        api.Plan(ctx, bad)
    bad = gen.subset(prob)
    bad.img_npsf = bad.img_npsf.copy()
    bad.img_npsf[0] = 5                           # above the compiled limit
    bad.img_psf = np.concatenate([bad.img_psf, bad.img_psf[:, :1]], 1)
    with pytest.raises(Exception):
        api.Plan(ctx, bad)
    plan = api.Plan(ctx, prob)
    with pytest.raises(ValueError):
        api.elbo_grad(plan, np.zeros((3, 32)))
