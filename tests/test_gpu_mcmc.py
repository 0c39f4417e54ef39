"""GPU: the MCMC source step (Section 3: annealed importance sampling with slice-sampling-
within-Gibbs transitions, further slice-sampling chains, Bayes' rule over the type) through
the C ABI, against the oracle's sampler.

On the float64 pixel path the likelihood agrees with the oracle's to ~1e-13 relative, so
every slice-sampling decision is taken alike: the samples, the log evidences, p(star), the
drawn point and the chains' potential scale reduction equal the oracle's (1e-9 relative).  With float32 pixels decisions near a
slice threshold may go the other way and trajectories then part; the test reports how many
chains kept the float64 trajectory and bounds the log evidence and p(star)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1803_00113_amd import _ffi, api  # noqa: E402
from synth import gen  # noqa: E402
from tests.golden.inputs_hash import load_golden  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tiny():
    """The small problem of the stored oracle step (tests/golden/make_golden.py, mcmc) with
    the options, start points and key it was made with."""
    from tests.golden.make_golden import MCMC_INIT_SEED, mcmc_problem
    prob, z = mcmc_problem()
    ref = load_golden("mcmc_oracle.npz", prob)
    opts = dict(n_temps=int(ref["n_temps"]), n_runs=int(ref["n_runs"]), n_post=int(ref["n_post"]),
                gamma=list(ref["gamma"]), width=list(ref["width"]), box=float(ref["box"]),
                max_step_out=int(ref["max_step_out"]), max_shrink=int(ref["max_shrink"]), seed=int(ref["seed"]))
    assert int(ref["init_seed"]) == MCMC_INIT_SEED
    init = gen.prior_draws(prob, z, opts["n_runs"], seed=MCMC_INIT_SEED, box=opts["box"])
    return prob, z, init, opts, int(ref["key"]), ref


def _run(tiny, fp64, mask=None):
    prob, z, init, opts, key, _ = tiny
    ctx = api.Context(0, pixel_fp64=fp64)
    plan = api.Plan(ctx, prob)
    zf = torch.as_tensor(z, device="cuda").contiguous()
    zi = torch.as_tensor(init, device="cuda").contiguous()
    r = api.mcmc_step(plan, zf, zi, opts, key, mask=mask, want_samples=True)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in r.items()}


def test_mcmc_step_fp64_matches_oracle(tiny):
    say("case: mcmc step, float64 pixels, 2 sources, T=4, N'=3, B'=2")
    prob, z, init, opts, key, ref = tiny
    r = _run(tiny, True)
    say(f"  report {r['report']}")
    for s in range(prob.n_sources):
        assert np.allclose(r["samples"][s], ref["samples"][s], rtol=1e-9, atol=1e-12), \
            np.abs(r["samples"][s] - ref["samples"][s]).max()
        assert np.allclose(r["log_evidence"][s], ref["log_evidence"][s], rtol=1e-9)
        assert abs(r["p_star"][s] - ref["p_star"][s]) <= 1e-9
        assert np.allclose(r["z"][s], ref["z"][s], rtol=1e-9, atol=1e-12) and r["z"][s, 2] == ref["a"][s]
        # the chains' potential scale reduction: the same finite values, NaN and +inf where
        # the oracle has them (coordinates no chain moves; a star's unused galaxy coordinates)
        rh, orh = r["rhat"][s], ref["rhat"][s]
        assert np.array_equal(np.isnan(rh), np.isnan(orh)) and np.array_equal(np.isinf(rh), np.isinf(orh))
        fin = np.isfinite(orh)
        assert np.allclose(rh[fin], orh[fin], rtol=1e-9), np.abs(rh[fin] - orh[fin]).max()
        say(f"  s={s}: log evidence {r['log_evidence'][s]} oracle {ref['log_evidence'][s]}, "
            f"p(star) {r['p_star'][s]:.6f}")
    assert r["report"]["n_chains"] == 2 * 2 * opts["n_runs"] and r["report"]["rounds"] > 0


def test_mcmc_step_mask_and_determinism(tiny):
    """One selected source: its results equal those of the run with both selected (a chain's
    random numbers depend only on its own counters); the other source's rows are untouched;
    a repeated call gives identical results."""
    say("case: mcmc step, mask and repeat")
    prob, z, _, _, _, _ = tiny
    both = _run(tiny, True)
    one = _run(tiny, True, mask=np.array([False, True]))
    assert np.array_equal(one["samples"][1], both["samples"][1]) and np.array_equal(one["z"][1], both["z"][1])
    assert np.array_equal(one["z"][0], z[0]) and np.isnan(one["p_star"][0]) and np.all(one["samples"][0] == 0)
    assert np.isnan(one["rhat"][0]).all() and np.array_equal(one["rhat"][1], both["rhat"][1], equal_nan=True)
    again = _run(tiny, True)
    for k in ("samples", "z", "p_star", "log_evidence", "rhat"):
        assert np.array_equal(again[k], both[k], equal_nan=True)


def test_mcmc_step_fp32_close_to_oracle(tiny):
    say("case: mcmc step, float32 pixels")
    prob, z, _, opts, _, ref = tiny
    r = _run(tiny, False)
    same = 0
    for s in range(prob.n_sources):
        for a in (0, 1):
            for k in range(opts["n_runs"]):
                same += int(np.allclose(r["samples"][s, a, k], ref["samples"][s, a, k], rtol=1e-4, atol=1e-6))
        rel = np.abs(r["log_evidence"][s] - ref["log_evidence"][s]) / np.abs(ref["log_evidence"][s])
        say(f"  s={s}: log evidence {r['log_evidence'][s]} oracle {ref['log_evidence'][s]} (rel {rel.max():.1e}); "
            f"p(star) {r['p_star'][s]:.4f} oracle {float(ref['p_star'][s]):.4f}")
        assert rel.max() <= 1e-3
        smp = r["samples"][s].reshape(-1, 16)
        assert np.all(np.abs(smp[:, 0:2] - z[s, 0:2]) <= opts["box"])
    say(f"  chains on the float64 trajectory: {same} of {2 * 2 * opts['n_runs']}")


def test_mcmc_step_rejects_bad_options(tiny):
    prob, z, init, opts, key, _ = tiny
    ctx = api.Context(0)
    plan = api.Plan(ctx, prob)
    zf = torch.as_tensor(z, device="cuda").contiguous()
    zi = torch.as_tensor(np.repeat(init, 10, axis=1)[:, :29], device="cuda").contiguous()
    with pytest.raises(_ffi.CelError):
        api.mcmc_step(plan, zf, zi, dict(opts, n_runs=29), key)
    zi = torch.as_tensor(init, device="cuda").contiguous()
    with pytest.raises(_ffi.CelError):
        api.mcmc_step(plan, zf, zi, dict(opts, box=0.0), key)
