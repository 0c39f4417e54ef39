"""Pins of the oracle's MCMC source step (oracle/mcmc.py; Section 3: annealed importance
sampling over temperatures with slice-sampling-within-Gibbs transitions, then further
slice-sampling chains and Bayes' rule over the source type).

  * Philox4x64-10 against numpy's implementation of the same published generator;
  * the slice-sampling update leaves known densities invariant (a normal, a truncated
    exponential, a two-mode mixture): sample moments within Monte Carlo error;
  * annealed importance sampling on a conjugate normal model estimates its evidence
    (closed form) and its post-annealing chains sample its posterior (closed form);
  * the source step is deterministic in its key, its type probability is Bayes' rule on its
    own evidence estimates, its draw is one of its samples and it stays in the support."""
import math

import numpy as np
import pytest

from oracle import elbo as E
from oracle import mcmc as M
from synth import gen


def _raw_numpy(ctr, key):
    """numpy's Philox advances the counter before producing a block: block(c) is the first
    output of a generator started at c - 1 (mod 2^256)."""
    c = 0
    for i, v in enumerate(ctr):
        c |= int(v) << (64 * i)
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & M.MASK64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=words, key=np.array(key, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((1, 2, 3, 4), (5, 6)),
                                     ((M.MASK64, M.MASK64, M.MASK64, M.MASK64), (M.MASK64, M.MASK64)),
                                     ((17, 16 * 200 + 10, 123456, 0), (180300110, 3)), ((0, 0, 999, 1), (1, 0))])
def test_philox_matches_numpy(ctr, key):
    assert M.philox4x64(ctr, key) == _raw_numpy(ctr, key)


def test_uniforms_are_inside_the_open_interval():
    assert M.uniform(0) == 2.0 ** -54 and M.uniform(M.MASK64) == 1.0 - 2.0 ** -54


def _chain(logf, x0, width, m, n, key=(11, 0)):
    xs = np.zeros(n)
    x, fx = x0, logf(x0)
    for t in range(n):
        def draws(k, _t=t):
            out = M.philox4x64((k, _t, 0, 0), key)
            return M.uniform(out[0]), M.uniform(out[1]), M.uniform(out[2])
        x, fx = M.slice_update(logf, x, fx, width, m, draws)
        xs[t] = x
    return xs


def _batch_se(xs, nb=50):
    b = xs[: len(xs) // nb * nb].reshape(nb, -1).mean(1)
    return b.std(ddof=1) / math.sqrt(nb)


@pytest.mark.parametrize("width,m", [(1.0, 8), (0.2, 8), (5.0, 1)])
def test_slice_update_leaves_a_normal_invariant(width, m):
    xs = _chain(lambda x: -0.5 * x * x, 0.3, width, m, 20000)
    assert abs(xs.mean()) < 5 * _batch_se(xs)
    assert abs((xs ** 2).mean() - 1.0) < 5 * _batch_se(xs ** 2)
    assert abs((xs < -1).mean() - 0.158655) < 5 * _batch_se((xs < -1).astype(float))


def test_slice_update_on_a_truncated_density():
    """An exponential density on [0, inf): -infinity outside its support."""
    xs = _chain(lambda x: -x if x >= 0 else -math.inf, 0.5, 1.0, 8, 20000)
    assert xs.min() >= 0
    assert abs(xs.mean() - 1.0) < 5 * _batch_se(xs)
    assert abs((xs > 2).mean() - math.exp(-2)) < 5 * _batch_se((xs > 2).astype(float))


def test_slice_update_visits_both_modes_in_proportion():
    """0.3 N(-3, 0.7^2) + 0.7 N(2, 1): the stepping-out interval reaches across the gap."""
    def logf(x):
        return math.log(0.3 * math.exp(-(x + 3) ** 2 / (2 * 0.49)) / 0.7 + 0.7 * math.exp(-(x - 2) ** 2 / 2))
    xs = _chain(logf, 0.0, 2.0, 10, 40000)
    frac = (xs < -0.5).mean()
    assert abs(frac - 0.3) < 5 * _batch_se((xs < -0.5).astype(float))


class _Toy:
    """Prior N(0, 1) on w[0]; n observations y ~ N(w, sigma^2)."""

    def __init__(self, y, sig):
        self.y, self.sig = y, sig

    def parts(self, w):
        x = w[0]
        lp = -0.5 * math.log(2 * math.pi) - 0.5 * x * x
        ll = float(np.sum(-0.5 * math.log(2 * math.pi * self.sig ** 2) - (self.y - x) ** 2 / (2 * self.sig ** 2)))
        return lp, ll


def test_annealed_importance_sampling_on_a_conjugate_model():
    """log p(y) = log N(y; 0, sigma^2 I + 1 1^T) in closed form; the runs' log mean weight
    estimates it, and the B' sweeps after annealing sample the posterior
    N(sum y / (sigma^2 + n), sigma^2 / (sigma^2 + n))."""
    rng = np.random.default_rng(0)
    n, sig = 20, 0.5
    y = rng.normal(0.7, sig, n)
    C = sig ** 2 * np.eye(n) + np.ones((n, n))
    exact = -0.5 * (n * math.log(2 * math.pi) + np.linalg.slogdet(C)[1] + y @ np.linalg.solve(C, y))
    opts = dict(n_temps=60, n_post=20, gamma_power=4.0, width=(1.0,), max_step_out=8, max_shrink=200)
    runs = [M.run_chain(_Toy(y, sig), np.array([rng.normal()]), (0,), r, (7, 0), opts, periodic=())
            for r in range(300)]
    lw = np.array([r[0] for r in runs])
    wts = np.exp(lw - lw.max())
    est = lw.max() + math.log(wts.mean())
    se = wts.std(ddof=1) / wts.mean() / math.sqrt(len(wts))     # delta method for log of a mean
    assert abs(est - exact) < 5 * se + 0.01, (est, exact, se)
    post = np.concatenate([r[1][:, 0] for r in runs])
    pm, pv = y.sum() / (sig ** 2 + n), sig ** 2 / (sig ** 2 + n)
    assert abs(post.mean() - pm) < 5 * math.sqrt(pv / len(runs))
    assert abs(post.var() - pv) < 0.15 * pv


@pytest.fixture(scope="module")
def tiny():
    prob = gen.crop_patches(gen.subset(gen.config1(), images=[1, 2]), 12)
    z = gen.truth_point(prob)
    return prob, E.Model(prob), z


OPTS = dict(M.DEFAULTS, n_temps=2, n_runs=1, n_post=1)


def test_source_step_is_bayes_rule_on_its_estimates_and_deterministic(tiny):
    prob, m, z = tiny
    init = gen.prior_draws(prob, z, OPTS["n_runs"], seed=5, box=OPTS["box"])
    s = 1
    r1 = M.source_step(m, z, s, init[:, :, s], OPTS, key=(9, 0))
    r2 = M.source_step(m, z, s, init[:, :, s], OPTS, key=(9, 0))
    r3 = M.source_step(m, z, s, init[:, :, s], OPTS, key=(9, 1))
    assert np.array_equal(r1["samples"], r2["samples"]) and r1["p_star"] == r2["p_star"]
    assert not np.array_equal(r1["samples"], r3["samples"])
    ev = r1["log_evidence"]
    for a in (0, 1):
        lw = r1["logw"][a]
        assert ev[a] == pytest.approx(math.log(np.mean(np.exp(lw - lw.max()))) + lw.max(), rel=1e-12)
    A = prob.prior_a
    odds = A * math.exp(ev[1] - max(ev)) / ((1 - A) * math.exp(ev[0] - max(ev)))
    assert r1["p_star"] == pytest.approx(odds / (1 + odds), rel=1e-12)
    a, j = r1["a"], r1["index"]
    assert np.array_equal(r1["z"], r1["samples"][a, j // OPTS["n_post"], j % OPTS["n_post"]])
    assert r1["z"][2] == a
    smp = r1["samples"].reshape(-1, 16)
    assert np.all(np.abs(smp[:, 0:2] - z[s, 0:2]) <= OPTS["box"])
    assert np.all((smp[:, 10] >= 0) & (smp[:, 10] <= 1) & (smp[:, 11] > 0) & (smp[:, 11] <= 1))
    assert np.all((smp[:, 8] >= 0) & (smp[:, 8] < math.pi))


def test_rhat_worked_example():
    """Two chains (1, 2, 3) and (2, 3, 4): chain means 2 and 3, grand mean 5/2, between-chain
    B = 3 / 1 x (1/4 + 1/4) = 3/2, within-chain W = (1 + 1) / 2 = 1, V = 2/3 + 1/2 = 7/6,
    R = sqrt(7/6) (worked by hand from the definition in Gelman and Rubin 1992)."""
    x = np.array([[1.0, 2.0, 3.0], [2.0, 3.0, 4.0]])[:, :, None]
    assert M.rhat(x)[0] == pytest.approx(math.sqrt(7.0 / 6.0), rel=1e-15)


def test_rhat_of_chains_with_known_between_and_within_spread():
    """Chain j = c_j + e, one zero-mean pattern e of sample variance s2 shared by every chain:
    W = s2 exactly and B = n var(c) (divisor m - 1), so R^2 = ((n - 1) / n s2 + var(c)) / s2."""
    rng = np.random.default_rng(1)
    n, m = 40, 5
    e = rng.normal(size=n)
    e -= e.mean()
    s2 = e.var(ddof=1)
    c = np.array([0.0, 0.3, -0.2, 1.1, 0.4])
    x = (c[:, None] + e[None, :])[:, :, None]
    want = math.sqrt(((n - 1) / n * s2 + c.var(ddof=1)) / s2)
    assert M.rhat(x)[0] == pytest.approx(want, rel=1e-12)


def test_rhat_invariances_and_limits():
    """Invariant under x -> a x + b (a != 0) coordinatewise; near 1 for independent draws
    from one distribution; large when the chains sit apart; NaN for a coordinate no chain
    moves and for a single draw per chain."""
    rng = np.random.default_rng(2)
    x = rng.normal(size=(4, 50, 3)) + np.array([0.0, 0.5, 2.0])[None, None, :] * np.arange(4)[:, None, None]
    r = M.rhat(x)
    assert np.allclose(M.rhat(-3.0 * x + 7.0), r, rtol=1e-12)
    assert r[0] < r[1] < r[2] and r[2] > 2.0
    iid = M.rhat(rng.normal(size=(4, 100_000, 1)))[0]
    assert abs(iid - 1.0) < 2e-3
    const = np.zeros((3, 5, 1))
    assert np.isnan(M.rhat(const)[0])
    assert np.isnan(M.rhat(rng.normal(size=(3, 1, 2)))).all()
