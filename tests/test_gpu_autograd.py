"""GPU: the ELBO as a torch.autograd.Function (forward = ELBO kernel, backward = adjoint
kernel with pixel terms recomputed) against central differences and the oracle gradient."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import elbo as E  # noqa: E402
from paper_1803_00113_amd import api, autograd  # noqa: E402
from synth import gen  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_gradcheck_fp64_path():
    """torch.autograd.gradcheck (central differences in float64) on the float64 pixel path."""
    say("case: gradcheck fp64")
    prob = gen.crop_patches(gen.subset(gen.config2(n_sources=3), images=[2, 4]), 12)
    ctx = api.Context(0, pixel_fp64=True)
    plan = api.Plan(ctx, prob)
    th = torch.as_tensor(prob.theta0, device="cuda").clone().requires_grad_(True)
    f = lambda t: autograd.elbo(plan, t)
    assert torch.autograd.gradcheck(f, (th,), eps=1e-6, atol=1e-5, rtol=1e-6, nondet_tol=0.0)


def test_adjoint_config3_against_oracle_and_fd():
    """4096 sources, 5 bands, patches 16-64 px (float32 pixels): autograd gradient of the
    summed ELBO against the oracle gradient on sampled sources, and against the oracle's
    central differences (h = 1e-4) for every parameter of a few sources."""
    say("case: config3 adjoint")
    prob = gen.config3()
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    th = torch.as_tensor(prob.theta0, device="cuda").clone().requires_grad_(True)
    L = autograd.elbo(plan, th)
    L.backward()
    g = th.grad.cpu().numpy()
    tot, _, g2 = api.elbo_grad(plan, prob.theta0)
    assert torch.equal(th.grad, g2) and L.item() == tot.item()
    m = E.Model(prob)
    rng = np.random.default_rng(3)
    for s in rng.choice(prob.n_sources, 48, replace=False):
        _, og = E.local_value_grad(m, prob.theta0, int(s))
        floor = 0.01 * np.abs(og).max()
        assert np.all(np.abs(g[s, :27] - og) <= 1e-4 * np.maximum(np.abs(og), floor)), s
    h = 1e-4
    for s in rng.choice(prob.n_sources, 3, replace=False):
        f = E.local_objective(m, prob.theta0, int(s))
        base = torch.as_tensor(prob.theta0[s, :27])
        for k in range(27):
            e = torch.zeros(27, dtype=torch.float64)
            e[k] = h
            fd = (f(base + e).item() - f(base - e).item()) / (2 * h)
            assert abs(fd - g[s, k]) <= 1e-4 * max(abs(fd), 0.01 * np.abs(g[s, :27]).max()), (s, k, fd, g[s, k])
