"""Pins of the oracle's KL divergence (equations eq:kl, kleq; Supplement A, with the
oracle's stated readings) against scipy densities, numerical integration, Monte Carlo
and brute-force minimisation over the free weights of the colour bound."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate, special, stats

from oracle import elbo as E
from synth import gen


def _model_with_prior(J=None, seed=11):
    prob = gen.config1()
    if J is not None:
        rng = np.random.default_rng(seed)
        prob.prior_cw = np.stack([rng.dirichlet(np.ones(J)) for _ in range(2)])
        prob.prior_cmean = rng.normal(0.5, 0.4, (2, J, 4))
        cov = np.zeros((2, J, 4, 4))
        for i in range(2):
            for j in range(J):
                L = rng.normal(0, 0.25, (4, 4))
                cov[i, j] = L @ L.T + 0.05 * np.eye(4)
        prob.prior_ccov = cov
    return prob, E.Model(prob)


def _theta(prob, seed=5):
    rng = np.random.default_rng(seed)
    th = prob.theta0.copy()
    th[:, 2] = rng.normal(0, 1, 2)
    th[:, 5:7] = np.log(rng.uniform(0.02, 0.3, (2, 2)))
    th[:, 7:15] = rng.normal(0.5, 0.3, (2, 8))
    th[:, 15:23] = np.log(rng.uniform(0.02, 0.3, (2, 8)))
    th[:, 24] = np.log(rng.uniform(0.8, 3.0, 2))
    th[:, 25] = rng.normal(0, 1, 2)
    th[:, 26] = rng.normal(0.5, 1, 2)
    return th


def test_type_flux_and_point_mass_terms_against_scipy():
    """KL(Bernoulli || Bernoulli) = scipy entropy; flux KL = integral of q log(q/p) of the two
    log-normals by quadrature; radius, profile and axis point-mass terms = minus scipy's
    log-normal / Beta log densities at the point."""
    prob, m = _model_with_prior()
    th = _theta(prob)
    nat = E.natural(torch.as_tensor(th))
    kl = E.kl_terms(m, nat)
    for s in range(2):
        a = 1 / (1 + math.exp(-th[s, 2]))
        assert abs(kl["a"][s].item() - stats.entropy([a, 1 - a], [prob.prior_a, 1 - prob.prior_a])) < 1e-12
        for i in range(2):
            mq, vq = th[s, 3 + i], math.exp(th[s, 5 + i])
            mp, vp = prob.prior_r[i]
            q = stats.norm(mq, math.sqrt(vq))
            p = stats.norm(mp, math.sqrt(vp))
            val, _ = integrate.quad(lambda x: q.pdf(x) * (q.logpdf(x) - p.logpdf(x)), mq - 12 * math.sqrt(vq),
                                    mq + 12 * math.sqrt(vq), epsabs=1e-13, epsrel=1e-12, limit=200)
            assert abs(kl["r"][s, i].item() - val) < 1e-9
        rad = math.exp(th[s, 24])
        ref = -stats.lognorm(s=math.sqrt(prob.prior_radius[1]), scale=math.exp(prob.prior_radius[0])).logpdf(rad)
        assert abs(kl["radius"][s].item() - ref) < 1e-11
        prof = special.expit(th[s, 25])
        assert abs(kl["profile"][s].item() + stats.beta(*prob.prior_profile).logpdf(prof)) < 1e-11
        ax = special.expit(th[s, 26])
        assert abs(kl["axis"][s].item() + stats.beta(*prob.prior_axis).logpdf(ax)) < 1e-11
    # the total assembles the parts as equation kleq says
    a = torch.sigmoid(torch.as_tensor(th[:, 2]))
    tot = kl["a"] + kl["radius"] + kl["profile"] + kl["axis"] + (1 - a) * (kl["r"][:, 0] + kl["c"][:, 0]) \
        + a * (kl["r"][:, 1] + kl["c"][:, 1])
    assert torch.allclose(tot, kl["total"], rtol=1e-14, atol=1e-12)


def _mc_kl_to_component(mq, vq, mean, cov, rng, N=400000):
    x = mq + np.sqrt(vq) * rng.standard_normal((N, 4))
    lq = stats.multivariate_normal(mq, np.diag(vq)).logpdf(x)
    lp = stats.multivariate_normal(mean, cov).logpdf(x)
    d = lq - lp
    return d.mean(), d.std() / math.sqrt(N), x, lq


@pytest.mark.parametrize("J", [1, 2, 3])
def test_colour_bound(J):
    """Colour KL bound (Section 4.2.3): (i) equals the brute-force minimum over the free
    weights xi on a simplex grid of KL(xi || w) + sum_j xi_j D_j with each D_j estimated by
    Monte Carlo; (ii) is >= a Monte Carlo estimate of the true KL to the mixture; (iii) for
    J = 1 it is the KL to the single component."""
    prob, m = _model_with_prior(J=J)
    th = _theta(prob, seed=9)
    nat = E.natural(torch.as_tensor(th))
    kl_c = E.kl_terms(m, nat)["c"].numpy()
    rng = np.random.default_rng(J)
    s, i = 1, 0
    mq = th[s, 7 + 4 * i:11 + 4 * i]
    vq = np.exp(th[s, 15 + 4 * i:19 + 4 * i])
    D, se = [], []
    for j in range(J):
        d, e, x, lq = _mc_kl_to_component(mq, vq, prob.prior_cmean[i, j], prob.prior_ccov[i, j], rng)
        D.append(d)
        se.append(e)
    D = np.array(D)
    w = prob.prior_cw[i]
    if J == 1:
        best = D[0]
    else:
        grid = np.linspace(1e-6, 1 - 1e-6, 2001 if J == 2 else 301)
        if J == 2:
            xi = np.stack([grid, 1 - grid], 1)
        else:
            a, b = np.meshgrid(grid, grid)
            ok = a + b < 1
            xi = np.stack([a[ok], b[ok], 1 - a[ok] - b[ok]], 1)
        vals = np.sum(xi * (np.log(xi) - np.log(w)[None]), 1) + xi @ D
        best = vals.min()
    tol = 5 * max(se) + 2e-4
    assert abs(kl_c[s, i] - best) < tol
    # true KL to the mixture by Monte Carlo: the bound is an upper bound
    x = mq + np.sqrt(vq) * rng.standard_normal((400000, 4))
    lq = stats.multivariate_normal(mq, np.diag(vq)).logpdf(x)
    lp = special.logsumexp(np.stack([np.log(w[j]) + stats.multivariate_normal(prob.prior_cmean[i, j],
                                     prob.prior_ccov[i, j]).logpdf(x) for j in range(J)]), axis=0)
    true_kl = (lq - lp).mean()
    true_se = (lq - lp).std() / math.sqrt(len(x))
    assert kl_c[s, i] >= true_kl - 5 * true_se
