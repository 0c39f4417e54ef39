"""GPU parity of the point log-likelihood (cel_loglik, the likelihood factor of the MCMC
target, Sections 3 and 3.1) against the float64 oracle, element by element.

Tolerances as for the objective: |d| <= 1e-5 |oracle| with float32 pixels, 1e-10 with the
float64 pixel path; candidates outside the support are -infinity; rows of unselected
sources are not written."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import elbo as E  # noqa: E402
from oracle import likelihood as L  # noqa: E402
from paper_1803_00113_amd import api  # noqa: E402
from synth import gen  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(prob, zf, zc, mask=None, **opts):
    ctx = api.Context(0, **opts)
    plan = api.Plan(ctx, prob)
    ll = api.loglik(plan, torch.as_tensor(zf).cuda().contiguous(), torch.as_tensor(zc).cuda().contiguous(), mask)
    return ll.cpu().numpy()


def oracle(m, zf, zc, pairs):
    return np.array([L.log_likelihood(m, zf, s, zc[c, s]) for c, s in pairs])


@pytest.mark.parametrize("fp64", [False, True])
def test_config1_every_candidate(fp64):
    say(f"case: loglik config1 fp64={fp64}")
    prob = gen.config1()
    m = E.Model(prob)
    zf = gen.truth_point(prob)
    zc = gen.perturbed_points(zf, 9, 11)
    # edges of the support: pure exponential / de Vaucouleurs profile, round galaxy
    zc[0, :, 10] = 0.0
    zc[1, :, 10] = 1.0
    zc[2, :, 11] = 1.0
    # outside the support
    zc[7, 0, 11] = 0.0
    zc[8, 1, 10] = 1.5
    ll = run(prob, zf, zc, pixel_fp64=fp64)
    assert ll[7, 0] == -np.inf and ll[8, 1] == -np.inf
    pairs = [(c, s) for c in range(9) for s in range(prob.n_sources) if (c, s) not in ((7, 0), (8, 1))]
    want = oracle(m, zf, zc, pairs)
    got = np.array([ll[c, s] for c, s in pairs])
    rtol = 1e-10 if fp64 else 1e-5
    err = np.abs(got - want) / np.abs(want)
    assert np.all(err <= rtol), (err.max(), pairs[int(err.argmax())])


def test_masked_selection_two_chunks_and_alone():
    """A selection of overlapping and isolated sources, 58 candidates (two launch chunks):
    every selected entry against the oracle; unselected rows untouched (NaN); each candidate
    evaluated alone gives the same bits as in the batch."""
    say("case: loglik 60-source field, mask, 58 candidates")
    prob = gen.subset(gen.config2(n_sources=60), sources=list(range(60)))
    m = E.Model(prob)
    zf = gen.truth_point(prob)
    zc = gen.perturbed_points(zf, 58, 12)
    sel = np.zeros(prob.n_sources, bool)
    sel[[0, 3, 4, 17, 29, 41, 42, 59]] = True
    ll = run(prob, zf, zc, mask=sel)
    assert np.all(np.isnan(ll[:, ~sel]))
    pairs = [(c, s) for c in (0, 1, 27, 55, 56, 57) for s in np.nonzero(sel)[0]]
    want = oracle(m, zf, zc, pairs)
    got = np.array([ll[c, s] for c, s in pairs])
    err = np.abs(got - want) / np.abs(want)
    assert np.all(err <= 1e-5), (err.max(), pairs[int(err.argmax())])
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    zf_d = torch.as_tensor(zf).cuda().contiguous()
    for c in (0, 56, 57):
        one = api.loglik(plan, zf_d, torch.as_tensor(zc[c:c + 1]).cuda().contiguous(), sel).cpu().numpy()
        assert np.array_equal(one[0, sel], ll[c, sel])


def test_full_batched_workload_sampled():
    """All 1000 sources of the batched workload, 4 candidates: sampled entries against the
    oracle; two calls agree to the last bit."""
    say("case: loglik 1000-source workload, 4 candidates, sampled")
    prob = gen.config2()
    m = E.Model(prob)
    zf = gen.truth_point(prob)
    zc = gen.perturbed_points(zf, 4, 13)
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    zf_d, zc_d = torch.as_tensor(zf).cuda().contiguous(), torch.as_tensor(zc).cuda().contiguous()
    ll = api.loglik(plan, zf_d, zc_d).cpu().numpy()
    again = api.loglik(plan, zf_d, zc_d).cpu().numpy()
    assert np.array_equal(ll, again)
    rng = np.random.default_rng(5)
    pairs = [(int(c), int(s)) for c, s in zip(rng.integers(0, 4, 24), rng.choice(prob.n_sources, 24, replace=False))]
    want = oracle(m, zf, zc, pairs)
    got = np.array([ll[c, s] for c, s in pairs])
    err = np.abs(got - want) / np.abs(want)
    assert np.all(err <= 1e-5), (err.max(), pairs[int(err.argmax())])


def test_log_prior_matches_oracle():
    """cel_log_prior (the annealed sampler's start density, Section 3.1) against the oracle
    for stars, galaxies, the support's edges and points outside it (float64: 1e-12)."""
    say("case: log prior, 2-source field, 40 points")
    prob = gen.config1()
    m = E.Model(prob)
    z = gen.perturbed_points(gen.truth_point(prob), 20, 21).reshape(-1, 16)
    z[0, 10], z[1, 10], z[2, 11] = 0.0, 1.0, 1.0
    z[3, 11], z[4, 10], z[5, 3] = 0.0, -0.1, np.inf
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    got = api.log_prior(plan, torch.as_tensor(z).cuda().contiguous()).cpu().numpy()
    want = np.array([L.log_prior(m, row) for row in z])
    bad = ~np.isfinite(want)
    assert np.array_equal(got[bad], want[bad]) and bad[3:6].all()
    err = np.abs(got[~bad] - want[~bad]) / np.abs(want[~bad])
    assert np.all(err <= 1e-12), err.max()


def test_degenerate_calls():
    """No candidates, an empty selection, and a source whose candidate equals the fixed point
    (the likelihood then equals the variational objective's pixel sum at the point)."""
    say("case: loglik degenerate calls")
    prob = gen.config1()
    m = E.Model(prob)
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    zf = gen.truth_point(prob)
    zf_d = torch.as_tensor(zf).cuda().contiguous()
    empty = api.loglik(plan, zf_d, torch.zeros((0, prob.n_sources, 16), dtype=torch.float64, device="cuda"))
    assert empty.shape == (0, prob.n_sources)
    none = api.loglik(plan, zf_d, zf_d[None].clone(), mask=np.zeros(prob.n_sources, bool))
    assert torch.isnan(none).all()
    same = api.loglik(plan, zf_d, zf_d[None].clone()).cpu().numpy()[0]
    want = np.array([L.log_likelihood(m, zf, s, zf[s]) for s in range(prob.n_sources)])
    assert np.all(np.abs(same - want) <= 1e-5 * np.abs(want))
