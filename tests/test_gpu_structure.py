"""GPU: the less common structural cases against the oracle -- images whose PSF has one or
four components (the compiled limit) and an eight-component exponential profile (the
kernels' second profile layout), on the float32 and float64 paths, for the objective, the
gradient and the exact Hessian."""
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


def varied():
    prob = gen.crop_patches(gen.subset(gen.config2(n_sources=6), images=[0, 2, 5]), 20)
    psf = prob.img_psf.copy()
    npsf = prob.img_npsf.copy()
    # image 0: one component; image 1: four (a wide, faint fourth)
    psf[0, 1:] = 0.0
    psf[0, 0, 0] = 1.0
    npsf[0] = 1
    psf[1, 3] = [0.0, 0.4, -0.3, 9.0, 0.8, 7.0]
    psf[1, :3, 0] *= 0.9
    psf[1, 3, 0] = 0.1
    npsf[1] = 4
    prob.img_psf, prob.img_npsf = psf, npsf
    # exponential profile with 8 components: two extra wide, faint ones
    a = np.concatenate([prob.exp_alpha * 0.97, [0.02, 0.01]])
    t = np.concatenate([prob.exp_tau, [6.0, 12.0]])
    prob.exp_alpha, prob.exp_tau = a / a.sum(), t
    return prob


def rel_scaled(h, o):
    d = np.sqrt(np.abs(np.diag(o)))
    scale = np.maximum(np.maximum(np.outer(d, d), np.abs(o)), 1e-12 * np.abs(o).max())
    return (np.abs(h - o) / scale).max()


@pytest.mark.parametrize("fp64", [True, False])
def test_psf_counts_and_eight_component_profile(fp64):
    say(f"case: PSF of 1 and 4 components, 8-component exponential profile, fp64={fp64}")
    prob = varied()
    m = E.Model(prob)
    o_tot, o_loc, o_g = E.elbo_total_and_grad(m, prob.theta0)
    ctx = api.Context(0, pixel_fp64=fp64, hessian_fp64=fp64)
    plan = api.Plan(ctx, prob)
    tot, loc, g = api.elbo_grad(plan, prob.theta0)
    torch.cuda.synchronize()
    tot, loc, g = tot.item(), loc.cpu().numpy(), g.cpu().numpy()
    re, rg = (1e-10, 1e-8) if fp64 else (1e-5, 1e-4)
    assert abs(tot - o_tot) <= re * abs(o_tot)
    assert np.all(np.abs(loc - o_loc) <= re * np.abs(o_loc))
    o_g = o_g[:, :27]
    floor = 0.01 * np.abs(o_g).max(axis=1, keepdims=True)
    err = np.abs(g[:, :27] - o_g) / np.maximum(np.abs(o_g), floor)
    say(f"  objective rel {abs(tot - o_tot) / abs(o_tot):.2e}, gradient max rel {err.max():.2e}")
    assert err.max() <= rg
    th = torch.as_tensor(prob.theta0, device="cuda").contiguous()
    h, _, _ = api.elbo_hessian(plan, th)
    torch.cuda.synchronize()
    h = h.cpu().numpy()
    worst = max(rel_scaled(h[s], E.local_hessian(m, prob.theta0, s)) for s in range(prob.n_sources))
    say(f"  Hessian scaled err {worst:.2e}")
    assert worst <= (1e-9 if fp64 else 5e-4)
