"""Pins of the point log-likelihood oracle (the likelihood factor of the MCMC target,
Sections 3 and 3.1) against library routines, a special case of the variational objective
and locality (no GPU)."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import elbo as E
from oracle import likelihood as L
from synth import gen


@pytest.fixture(scope="module")
def c1():
    p = gen.config1()
    return p, E.Model(p)


def _plane_sky(prob, p):
    """The generator's planar sky on patch p, rebuilt from its corner knots."""
    n = prob.patch_img[p]
    o = prob.img_sky_off[n]
    k = prob.sky_knots[o:o + 4].reshape(2, 2)
    H, W = prob.img_H[n], prob.img_W[n]
    rows = np.arange(prob.patch_y0[p], prob.patch_y0[p] + prob.patch_h[p])[:, None] / (H - 1)
    cols = np.arange(prob.patch_x0[p], prob.patch_x0[p] + prob.patch_w[p])[None, :] / (W - 1)
    return k[0, 0] + (k[1, 0] - k[0, 0]) * rows + (k[0, 1] - k[0, 0]) * cols


def _brute_force(prob, z, s, kernel):
    """sum over source s's patches of scipy's Poisson log-pmf at lambda = sky + the light of
    every source whose patch covers the pixel; kernel(t, n, pts) is the source's light
    density at the pixel centres pts."""
    total = 0.0
    for p in np.nonzero(prob.patch_src == s)[0]:
        n = prob.patch_img[p]
        x0, y0, w, h = prob.patch_x0[p], prob.patch_y0[p], prob.patch_w[p], prob.patch_h[p]
        yy, xx = np.mgrid[y0:y0 + h, x0:x0 + w]
        lam = _plane_sky(prob, p).copy()
        for q in np.nonzero(prob.patch_img == n)[0]:
            t = prob.patch_src[q]
            qx0, qy0, qw, qh = prob.patch_x0[q], prob.patch_y0[q], prob.patch_w[q], prob.patch_h[q]
            inside = (xx >= qx0) & (xx < qx0 + qw) & (yy >= qy0) & (yy < qy0 + qh)
            if not inside.any():
                continue
            flux = gen.band_fluxes(math.exp(z[t, 3]), z[t, 4:8])[prob.img_band[n]] * prob.img_iota[n]
            pts = np.stack([xx.ravel(), yy.ravel()], 1).astype(float)
            lam = lam + inside * flux * kernel(t, n, pts).reshape(h, w)
        x = prob.patch_pixels(p).astype(int)
        total += stats.poisson.logpmf(x, lam).sum()
    return total


def _psf_density(prob, z, t, n, pts, extra_cov=None):
    mu = prob.img_A[n] @ z[t, 0:2] + prob.img_b[n]
    out = 0.0
    for k in range(prob.img_npsf[n]):
        w_, mx, my, cxx, cxy, cyy = prob.img_psf[n, k]
        cov = np.array([[cxx, cxy], [cxy, cyy]]) + (0 if extra_cov is None else extra_cov)
        out = out + w_ * stats.multivariate_normal(mu + [mx, my], cov).pdf(pts)
    return out


def test_overlapping_stars_exact_poisson_against_scipy(c1):
    """Both sources of the two-source field as stars: the light kernel is the PSF at the
    source's pixel position (Section 2.2.3), the flux in band b comes from the reference
    flux and the colours; the oracle's sum over source s's patches equals scipy's Poisson
    log-pmf summed with scipy's normal densities, the neighbour's light included where its
    patch covers the pixel."""
    prob, m = c1
    z = L.point_of_theta(prob.theta0, [1, 1]).numpy()
    z[0, 0:2] += [0.3, -0.2]
    for s in range(prob.n_sources):
        want = _brute_force(prob, z, s, lambda t, n, pts: _psf_density(prob, z, t, n, pts))
        got = L.log_likelihood(m, z, s, z[s])
        assert abs(got - want) <= 1e-10 * abs(want), (s, got, want)


def test_isotropic_galaxies_exact_poisson_against_scipy(c1):
    """Both sources as round galaxies (axis ratio 1): the galaxy kernel is the profile mixture
    convolved with the PSF, each pair of components a normal density whose covariance is the
    PSF component's plus tau_j radius^2 A A^T (Sections 2.1.2 and 2.2.3), weighted by the
    profile weight (de Vaucouleurs) and its complement (exponential)."""
    prob, m = c1
    z = L.point_of_theta(prob.theta0, [0, 0]).numpy()
    z[:, 11] = 1.0
    z[:, 10] = [0.3, 0.8]
    z[:, 9] = [math.log(1.6), math.log(2.4)]
    ea, et, da, dt = gen.load_profiles()

    def galaxy(t, n, pts):
        A = prob.img_A[n]
        r2 = math.exp(2 * z[t, 9])
        out = 0.0
        for alpha, tau, wt in ((da, dt, z[t, 10]), (ea, et, 1 - z[t, 10])):
            for j in range(len(alpha)):
                out = out + wt * alpha[j] * _psf_density(prob, z, t, n, pts, tau[j] * r2 * A @ A.T)
        return out

    for s in range(prob.n_sources):
        want = _brute_force(prob, z, s, galaxy)
        got = L.log_likelihood(m, z, s, z[s])
        assert abs(got - want) <= 1e-10 * abs(want), (s, got, want)


@pytest.mark.parametrize("types", [(1, 0), (0, 1), (0, 0)])
def test_zero_variance_limit_of_the_variational_pixel_sum(c1, types):
    """With q concentrated on one type (logit +-40) and on single flux and colour values (log
    variances -40), the variational objective's pixel terms (equation eq:log_p_last with the
    delta method) are the exact log-likelihood at the point: L_s + KL_s equals ll_s."""
    prob, m = c1
    z = L.point_of_theta(prob.theta0, list(types))
    z[:, 11] = torch.tensor([0.45, 0.7], dtype=torch.float64)
    th = torch.as_tensor(prob.theta0, dtype=torch.float64).clone()
    for t in range(prob.n_sources):
        th[t, 2] = 40.0 if types[t] else -40.0
        th[t, 3] = th[t, 4] = z[t, 3]
        th[t, 7:11] = th[t, 11:15] = z[t, 4:8]
        th[t, 5:7] = -40.0
        th[t, 15:23] = -40.0
        th[t, 26] = torch.logit(z[t, 11])
        th[t, 25] = torch.logit(z[t, 10])
    kl = E.kl_terms(m, E.natural(th))["total"]
    for s in range(prob.n_sources):
        local = E.elbo(m, th, sources=[s], with_total=False)[1][s]
        got = L.log_likelihood(m, z, s, z[s])
        want = (local + kl[s]).item()
        assert abs(got - want) <= 1e-9 * abs(want), (s, got, want)


def test_depends_on_neighbours_only_through_overlap():
    """ll_s is a function of z_s and of the sources whose patches meet s's patches
    (equation eqzs): moving a source with no overlapping patch leaves it unchanged to the
    last bit, moving an overlapping neighbour changes it."""
    prob = gen.subset(gen.config2(n_sources=40), sources=list(range(40)))
    m = E.Model(prob)
    z = L.point_of_theta(prob.theta0, (prob.theta0[:, 2] > 0).astype(int))
    s = next(s for s in range(prob.n_sources)
             if any(m.psrc[q] != s for p in m.patches_of[s] for q in m.cover[p]))
    nb = {int(m.psrc[q]) for p in m.patches_of[s] for q in m.cover[p]} - {s}
    far = next(t for t in range(prob.n_sources) if t != s and t not in nb)
    base = L.log_likelihood(m, z, s, z[s])
    z2 = z.clone()
    z2[far, 0:2] += 0.7
    z2[far, 3] += 0.5
    assert L.log_likelihood(m, z2, s, z2[s]) == base
    t = min(nb)
    z3 = z.clone()
    z3[t, 3] += 0.5
    assert L.log_likelihood(m, z3, s, z3[s]) != base


@pytest.mark.parametrize("star", [0, 1])
def test_log_prior_against_scipy(c1, star):
    """log p(w_s | a_s) over the point layout's coordinates (Section 2.1 priors): scipy's
    normal density for log flux and log radius, its multivariate normal mixture for the
    colours, its beta density for the profile weight and axis ratio, 1/pi for the angle;
    -inf outside the support."""
    prob, m = c1
    z = gen.perturbed_points(gen.truth_point(prob), 5, 3)[:, 0]
    z[:, 2] = star
    i = star
    for row in z:
        lp = stats.norm(prob.prior_r[i, 0], math.sqrt(prob.prior_r[i, 1])).logpdf(row[3])
        mix = sum(w * stats.multivariate_normal(mu, cov).pdf(row[4:8])
                  for w, mu, cov in zip(prob.prior_cw[i], prob.prior_cmean[i], prob.prior_ccov[i]) if w > 0)
        lp += math.log(mix)
        if not star:
            lp += stats.norm(prob.prior_radius[0], math.sqrt(prob.prior_radius[1])).logpdf(row[9])
            lp += stats.beta(*prob.prior_profile).logpdf(row[10]) + stats.beta(*prob.prior_axis).logpdf(row[11])
            lp -= math.log(math.pi)
        got = L.log_prior(m, row)
        assert abs(got - lp) <= 1e-10 * abs(lp), (got, lp)
    bad = z[0].copy()
    bad[11] = 0.0
    assert L.log_prior(m, bad) == -math.inf
    bad = z[0].copy()
    bad[10] = 1.2
    assert L.log_prior(m, bad) == -math.inf
