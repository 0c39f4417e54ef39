"""GPU: the ELBO as a torch.autograd.Function (forward = ELBO kernel, backward = adjoint
kernel with pixel terms recomputed) against central differences and the oracle gradient."""
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

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
