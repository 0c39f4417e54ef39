"""GPU: failure handling forced from the host -- non-finite parameters give per-source
statuses and context condition bits, never an aborted batch; the other sources' results
are unaffected."""
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


def field():
    # several isolated groups: sources 0.. of different groups do not interact
    return gen.crop_patches(gen.subset(gen.config2(n_sources=12), images=[0, 4]), 24)


def test_nonfinite_theta_flags_and_isolation():
    say("case: non-finite theta")
    prob = field()
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    assert api.last_device_error(ctx) == 0
    th = torch.as_tensor(prob.theta0, device="cuda").contiguous()
    _, loc0, g0 = api.elbo_grad(plan, th)
    assert api.last_device_error(ctx) == 0
    bad = th.clone()
    bad[3, 24] = float("nan")
    _, loc1, g1 = api.elbo_grad(plan, bad)
    torch.cuda.synchronize()
    code = api.last_device_error(ctx)
    say(f"  condition bits after a NaN parameter: {code}")
    assert code & _ffi.DEVERR_NONFINITE_OBJECTIVE
    assert api.last_device_error(ctx) == 0            # read clears
    assert not np.isfinite(loc1[3].item())
    # the NaN reaches only sources sharing pixels with source 3; every other source is
    # bitwise unchanged
    hit = [s for s in range(prob.n_sources) if not np.isfinite(loc1[s].item())]
    say(f"  sources reached by the NaN: {hit}")
    assert 3 in hit and len(hit) < prob.n_sources
    for s in range(prob.n_sources):
        if s not in hit:
            assert loc1[s].item() == loc0[s].item() and torch.equal(g1[s], g0[s])
    # a Newton step on the bad source: status NONFINITE, theta unchanged, flag raised
    mask = np.zeros(prob.n_sources, bool)
    mask[3] = True
    r = torch.ones(prob.n_sources, dtype=torch.float64, device="cuda")
    t2 = bad.clone()
    st, _ = api.newton_step(plan, t2, r, mask)
    torch.cuda.synchronize()
    assert st[3].item() == _ffi.ST_NONFINITE
    assert torch.equal(t2[3, :24], bad[3, :24]) and torch.equal(t2[3, 25:], bad[3, 25:])
    assert api.last_device_error(ctx) & _ffi.DEVERR_NONFINITE_STEP
    # Hessians: the bad source's entries are non-finite and flagged, the others finite
    h, _, _ = api.elbo_hessian(plan, bad)
    torch.cuda.synchronize()
    assert api.last_device_error(ctx) & _ffi.DEVERR_NONFINITE_HESSIAN
    hn = h.cpu().numpy()
    assert not np.all(np.isfinite(hn[3]))
    assert np.all(np.isfinite(hn[[s for s in range(prob.n_sources) if s not in hit]]))


def test_invalid_arguments_rejected_before_launch():
    say("case: invalid arguments")
    prob = field()
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    th = torch.as_tensor(prob.theta0, device="cuda").contiguous()
    with pytest.raises(_ffi.CelError):
        api.sweep(plan, th, n_sweeps=1, start_colour=plan.n_colours + 3, radius=torch.ones(plan.S, dtype=torch.float64,
                  device="cuda"), status=torch.zeros(plan.S, dtype=torch.int32, device="cuda"))
    with pytest.raises(_ffi.CelError):
        api.sweep(plan, th, n_sweeps=1, max_classes=-1)
    assert api.last_device_error(ctx) == 0
