"""GPU: cel_elbo_grad_static, the entry point for callers that cannot allocate device
memory at call time, through the C ABI.  Its outputs equal cel_elbo_grad's bit for bit
(same kernels, same launch order, scratch in the static buffer instead of the plan's),
on two calls in a row on different plans, the second smaller than the first; a plan whose
scratch need exceeds the static buffer is rejected with CEL_ESCRATCH before any launch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1803_00113_amd import _ffi, api  # noqa: E402
from synth import gen  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _same(plan, theta):
    a = api.elbo_grad(plan, theta)
    b = api.elbo_grad_static(plan, theta)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert np.isfinite(b[0].item())
    return b


@pytest.mark.parametrize("fp64", [False, True])
def test_static_scratch_equals_plan_scratch(fp64):
    """A large plan, then a smaller one on the same context (the second call reuses the
    static buffer that still holds the first call's contents)."""
    say(f"case: static-scratch gradient, two plans, fp64={fp64}")
    ctx = api.Context(0, pixel_fp64=fp64)
    big = gen.config2(n_sources=200) if not fp64 else gen.config2(n_sources=60)
    small = gen.crop_patches(gen.subset(gen.config2(n_sources=9), images=[0, 3, 6]), 21)
    for prob in (big, small):
        plan = api.Plan(ctx, prob)
        _same(plan, prob.theta0)
        say(f"  {prob.name}: {plan.n_units} pixels, bitwise equal")
    # and the large one again after the small one
    plan = api.Plan(ctx, big)
    _same(plan, big.theta0)


def test_static_scratch_full_batched_workload_and_limit():
    """The 1000-source batched workload (float32 pixels, 204 MB of scratch) fits the static
    buffer and matches; with float64 pixels (tables and maps twice as large) it does not and
    the call returns CEL_ESCRATCH without writing the outputs."""
    say("case: static-scratch gradient, batched workload, limit")
    prob = gen.config2()
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    _same(plan, prob.theta0)
    ctx64 = api.Context(0, pixel_fp64=True)
    plan64 = api.Plan(ctx64, prob)
    out = (torch.full((1,), 7.0, dtype=torch.float64, device="cuda"),
           torch.full((prob.n_sources,), 7.0, dtype=torch.float64, device="cuda"),
           torch.full((prob.n_sources, 32), 7.0, dtype=torch.float64, device="cuda"))
    with pytest.raises(_ffi.CelError) as e:
        api.elbo_grad_static(plan64, prob.theta0, out=out)
    assert e.value.status == _ffi.CEL_ESCRATCH
    torch.cuda.synchronize()
    assert all(bool((t == 7.0).all()) for t in out)
    # the float32 plan still works after the rejected call
    _same(plan, prob.theta0)
    # and after its work items are re-cut (more items: larger slot rows in the buffer)
    plan.tune(torch.as_tensor(prob.theta0, device="cuda").contiguous(), chunk_pixels=[256],
              pixels_per_lane=[], map_pixels_per_lane=[])
    _same(plan, prob.theta0)
