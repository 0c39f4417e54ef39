"""Pins of the oracle on the inputs the plain workloads leave at their trivial values: a
WCS with rotation, shear and unequal scales (pixel = A u + b, A != A^T), a calibration
iota != 1 per image, sky knot grids larger than 2 x 2 that sample a field with curvature,
and PSF mixtures with off-centre, tilted components (Section 2.2, Tables 1 and 3; Section
2.2.1 for the sky, Section 2.2.3 for the PSF).  Every reference value here is computed
independently of the oracle: scipy densities and interpolators, closed-form moments and
the generator's photon simulation."""
import math

import numpy as np
import pytest
import torch
from scipy import interpolate, stats

from oracle import elbo as E
from synth import gen


@pytest.fixture(scope="module")
def sk():
    p = gen.config_skew()
    return p, E.Model(p)


def _nat(theta):
    return E.natural(torch.as_tensor(theta, dtype=torch.float64))


def _galaxy_sigma(theta_s):
    """Sigma_s from its eigen-decomposition: major axis (cos t, -sin t) with variance r^2,
    minor axis (sin t, cos t) with variance (axis r)^2 (Section 2.1.2)."""
    t, r, ax = theta_s[23], math.exp(theta_s[24]), 1 / (1 + math.exp(-theta_s[26]))
    v1, v2 = np.array([math.cos(t), -math.sin(t)]), np.array([math.sin(t), math.cos(t)])
    return r * r * np.outer(v1, v1) + (ax * r) ** 2 * np.outer(v2, v2)


def test_skew_inputs_are_not_trivial(sk):
    """The problem really exercises what it is for."""
    prob, _ = sk
    for n in range(prob.n_images):
        A = prob.img_A[n]
        assert np.abs(A - A.T).max() > 0.05 and abs(A[0, 0] - A[1, 1]) > 1e-3
        assert abs(prob.img_iota[n] - 1) > 0.05
        assert prob.img_sky_qh[n] >= 3 and prob.img_sky_qw[n] >= 3
        K = prob.img_npsf[n]
        assert np.abs(prob.img_psf[n, :K, 1:3]).max() > 0.05 and np.abs(prob.img_psf[n, :K, 4]).max() > 0.05
    assert (prob.patch_w != prob.patch_h).any()


def test_sky_knots_have_curvature_and_bilinear_matches_scipy(sk):
    """Sky interpolated linearly between knots spanning the image corners (Section 2.2.1):
    the oracle's sky on every patch equals scipy's RegularGridInterpolator (method
    'linear') on the knot grid, and the grid is far from a plane, so interior knots
    matter."""
    prob, m = sk
    for n in range(prob.n_images):
        qh, qw = prob.img_sky_qh[n], prob.img_sky_qw[n]
        o = prob.img_sky_off[n]
        k = prob.sky_knots[o:o + qh * qw].reshape(qh, qw)
        yy, xx = np.mgrid[0:qh, 0:qw]
        Amat = np.stack([np.ones(qh * qw), yy.ravel(), xx.ravel()], 1)
        coef = np.linalg.lstsq(Amat, k.ravel(), rcond=None)[0]
        assert np.abs(Amat @ coef - k.ravel()).max() > 5.0     # counts per pixel
    for p in range(prob.n_patches):
        n = prob.patch_img[p]
        qh, qw = prob.img_sky_qh[n], prob.img_sky_qw[n]
        o = prob.img_sky_off[n]
        k = prob.sky_knots[o:o + qh * qw].reshape(qh, qw)
        H, W = prob.img_H[n], prob.img_W[n]
        f = interpolate.RegularGridInterpolator((np.linspace(0, H - 1, qh), np.linspace(0, W - 1, qw)), k,
                                                method="linear")
        yy, xx = np.mgrid[prob.patch_y0[p]:prob.patch_y0[p] + prob.patch_h[p],
                          prob.patch_x0[p]:prob.patch_x0[p] + prob.patch_w[p]]
        want = f(np.stack([yy.ravel(), xx.ravel()], 1).astype(float)).reshape(yy.shape)
        assert np.allclose(m.sky(p).numpy(), want, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("s", [0, 3])
def test_mixture_moments_under_general_wcs(sk, s):
    """Light kernels through a general WCS (Sections 2.1.2, 2.2.3): on a fine pixel grid the
    star's and the galaxy's densities sum to 1, their mean is A u + b + sum_k w_k m_k, and
    the galaxy's covariance is the PSF mixture's covariance plus (sum_j weight_j tau_j)
    A Sigma_s A^T (Sigma_s from its eigenvectors).  A transposed A, a dropped PSF offset or
    cross term fails here."""
    prob, m = sk
    theta = prob.theta0.copy()
    nat = _nat(theta)
    for n in range(prob.n_images):
        A, b = prob.img_A[n], prob.img_b[n]
        mu = A @ theta[s, 0:2] + b
        half = 110
        x0, y0 = int(mu[0]) - half, int(mu[1]) - half
        f0, f1 = E.source_profiles(m, nat, s, n, x0, y0, 2 * half, 2 * half)
        f0, f1 = f0.numpy(), f1.numpy()
        cols = np.arange(x0, x0 + 2 * half)[None, :].astype(float)
        rows = np.arange(y0, y0 + 2 * half)[:, None].astype(float)
        K = prob.img_npsf[n]
        psf = prob.img_psf[n, :K]
        wk = psf[:, 0]
        mbar = (wk[:, None] * psf[:, 1:3]).sum(0)
        cov_k = [np.array([[c[3], c[4]], [c[4], c[5]]]) for c in psf]
        psf_cov = sum(wk[k] * (cov_k[k] + np.outer(psf[k, 1:3], psf[k, 1:3])) for k in range(K)) - np.outer(mbar, mbar)
        ea, et, da, dt = gen.load_profiles()
        prof = 1 / (1 + math.exp(-theta[s, 25]))
        ctau = prof * np.sum(da * dt) + (1 - prof) * np.sum(ea * et)
        want_gal = psf_cov + ctau * A @ _galaxy_sigma(theta[s]) @ A.T
        for f, want in ((f1, psf_cov), (f0, want_gal)):
            assert abs(f.sum() - 1) < 1e-7
            mx, my = (f * cols).sum(), (f * rows).sum()
            assert abs(mx - (mu[0] + mbar[0])) < 1e-6 and abs(my - (mu[1] + mbar[1])) < 1e-6
            dx, dy = cols - mx, rows - my
            mom = np.array([[(f * dx * dx).sum(), (f * dx * dy).sum()], [(f * dx * dy).sum(), (f * dy * dy).sum()]])
            assert np.allclose(mom, want, rtol=1e-6, atol=1e-6)


def test_galaxy_covariance_matches_photon_simulation(sk):
    """The pixel-frame covariance of a galaxy's light against the generator's photon
    simulation, which draws sky-frame offsets from the profile mixture and maps them by
    pixel = A u + b: the empirical covariance of a million mapped offsets equals the
    oracle density's covariance minus the PSF's, within 5 standard errors."""
    prob, m = sk
    s, n = 3, 2
    theta = prob.theta0.copy()
    nat = _nat(theta)
    t = theta[s]
    src = dict(radius=math.exp(t[24]), axis=1 / (1 + math.exp(-t[26])), angle=t[23],
               profile=1 / (1 + math.exp(-t[25])))
    rng = np.random.default_rng(11)
    N = 1_000_000
    off = gen._galaxy_offsets(rng, N, src, gen.load_profiles()) @ prob.img_A[n].T
    emp = np.cov(off.T)
    # oracle density covariance minus the PSF mixture's (a zero-width PSF is not allowed, so
    # take the difference of the galaxy and star densities' covariances)
    mu = prob.img_A[n] @ t[0:2] + prob.img_b[n]
    half = 110
    x0, y0 = int(mu[0]) - half, int(mu[1]) - half
    f0, f1 = [f.numpy() for f in E.source_profiles(m, nat, s, n, x0, y0, 2 * half, 2 * half)]
    cols = np.arange(x0, x0 + 2 * half)[None, :].astype(float)
    rows = np.arange(y0, y0 + 2 * half)[:, None].astype(float)

    def cov(f):
        mx, my = (f * cols).sum(), (f * rows).sum()
        dx, dy = cols - mx, rows - my
        return np.array([[(f * dx * dx).sum(), (f * dx * dy).sum()], [(f * dx * dy).sum(), (f * dy * dy).sum()]])

    got = cov(f0) - cov(f1)
    # standard error of a covariance entry: sqrt((E[x^2 y^2] - c^2) / N)
    se = np.sqrt(np.array([[np.mean(off[:, i] ** 2 * off[:, j] ** 2) - emp[i, j] ** 2 for j in range(2)]
                           for i in range(2)]) / N)
    assert np.all(np.abs(got - emp) < 5 * se), (got, emp, se)


@pytest.mark.parametrize("s,star", [(0, True), (3, True), (1, False), (4, False)])
def test_degenerate_q_is_exact_poisson_under_general_wcs(sk, s, star):
    """With q concentrated on one type and one flux/colour value, the objective's pixel terms
    are the exact Poisson log-likelihood (Section 4.2.2; V = 0).  Reference: scipy's Poisson
    log-pmf with rate sky + iota l_b f, f from scipy's bivariate normal densities with mean
    A u + b + m_k and covariance Sigma_k (+ tau_j A Sigma_s A^T for a galaxy, Sigma_s from
    its eigenvectors), sky from scipy's linear grid interpolator, l_b from the generator's
    colour -> band-flux map.  Only source s's light is included."""
    prob, m = sk
    theta = prob.theta0.copy()
    theta[s, 2] = 40.0 if star else -40.0
    theta[s, 5:7] = -40.0
    theta[s, 15:23] = -40.0
    nat = _nat(theta)
    i = 1 if star else 0
    ea, et, da, dt = gen.load_profiles()
    prof = 1 / (1 + math.exp(-theta[s, 25]))
    for p in [q for q in range(prob.n_patches) if prob.patch_src[q] == s]:
        n = prob.patch_img[p]
        x0, y0, w, h = prob.patch_x0[p], prob.patch_y0[p], prob.patch_w[p], prob.patch_h[p]
        Es, Vs = E.source_rate_moments(m, nat, s, n, x0, y0, w, h)
        got = E.pixel_terms(m.pixels(p), m.sky(p) + Es, Vs).sum().item()
        flux = gen.band_fluxes(math.exp(theta[s, 3 + i]), theta[s, 7 + 4 * i:11 + 4 * i])[prob.img_band[n]]
        A = prob.img_A[n]
        mu = A @ theta[s, 0:2] + prob.img_b[n]
        yy, xx = np.mgrid[y0:y0 + h, x0:x0 + w]
        pts = np.stack([xx.ravel(), yy.ravel()], 1).astype(float)
        P = A @ _galaxy_sigma(theta[s]) @ A.T
        f = 0.0
        for k in range(prob.img_npsf[n]):
            wk, mx, my, cxx, cxy, cyy = prob.img_psf[n, k]
            C = np.array([[cxx, cxy], [cxy, cyy]])
            if star:
                f = f + wk * stats.multivariate_normal(mu + [mx, my], C).pdf(pts)
            else:
                for al, ta, pw in [(a_, t_, prof) for a_, t_ in zip(da, dt)] + \
                        [(a_, t_, 1 - prof) for a_, t_ in zip(ea, et)]:
                    f = f + pw * al * wk * stats.multivariate_normal(mu + [mx, my], C + ta * P).pdf(pts)
        qh, qw = prob.img_sky_qh[n], prob.img_sky_qw[n]
        o = prob.img_sky_off[n]
        grid = interpolate.RegularGridInterpolator(
            (np.linspace(0, prob.img_H[n] - 1, qh), np.linspace(0, prob.img_W[n] - 1, qw)),
            prob.sky_knots[o:o + qh * qw].reshape(qh, qw), method="linear")
        sky = grid(np.stack([yy.ravel(), xx.ravel()], 1).astype(float))
        lam = sky + prob.img_iota[n] * flux * f
        want = stats.poisson.logpmf(prob.patch_pixels(p).ravel().astype(int), lam).sum()
        assert abs(got - want) <= 1e-10 * abs(want), (p, got, want)


def test_rate_moments_with_calibration_match_monte_carlo(sk):
    """E_q[lambda] and V_q[lambda] with iota != 1 against brute force: the expected count is
    iota times the flux, so its variance carries iota^2 (equations conditional, vareq).
    Sample type, log flux and colours from q for the overlapping sources 0-2 on a 5 x 5
    window, form sky + sum_s iota l_s f_s and compare mean and variance per pixel within 5
    standard errors."""
    prob, m = sk
    theta = prob.theta0.copy()
    S = 3
    theta[:S, 2] = [0.4, -0.7, 0.1]
    theta[:S, 5:7] = np.log([[0.08, 0.03], [0.05, 0.12], [0.1, 0.06]])
    theta[:S, 15:23] = np.log(np.linspace(0.02, 0.2, 8))[None, :]
    nat = _nat(theta)
    n = 1
    assert abs(prob.img_iota[n] - 1) > 0.5
    p0 = [q for q in range(prob.n_patches) if prob.patch_src[q] == 0 and prob.patch_img[q] == n][0]
    mu = prob.img_A[n] @ theta[0, 0:2] + prob.img_b[n]
    x0, y0 = int(mu[0]) - 2, int(mu[1]) - 2
    px0, py0 = prob.patch_x0[p0], prob.patch_y0[p0]
    sky = m.sky(p0)[y0 - py0:y0 - py0 + 5, x0 - px0:x0 - px0 + 5].numpy()
    Emap, Vmap = sky.copy(), np.zeros_like(sky)
    fs = []
    for s in range(S):
        Es, Vs = E.source_rate_moments(m, nat, s, n, x0, y0, 5, 5)
        Emap += Es.numpy()
        Vmap += Vs.numpy()
        fs.append([f.numpy() for f in E.source_profiles(m, nat, s, n, x0, y0, 5, 5)])
    rng = np.random.default_rng(5)
    N = 400000
    lam = np.tile(sky[None], (N, 1, 1))
    band = prob.img_band[n]
    refb = gen.REF_BAND
    for s in range(S):
        a = 1 / (1 + np.exp(-theta[s, 2]))
        star = rng.random(N) < a
        i = star.astype(int)
        logr = theta[s, 3 + i] + np.sqrt(np.exp(theta[s, 5 + i])) * rng.standard_normal(N)
        cm = np.where(star[:, None], theta[s, 11:15], theta[s, 7:11])
        cv = np.where(star[:, None], np.exp(theta[s, 19:23]), np.exp(theta[s, 15:19]))
        c = cm + np.sqrt(cv) * rng.standard_normal((N, 4))
        logl = logr + (c[:, refb:band].sum(1) if band > refb else -c[:, band:refb].sum(1))
        ell = np.array([gen.band_fluxes(math.exp(lr), cc)[band] for lr, cc in zip(logr[:2000], c[:2000])])
        assert np.allclose(np.exp(logl[:2000]), ell, rtol=1e-12)
        f = np.where(star[:, None, None], fs[s][1][None], fs[s][0][None])
        lam += prob.img_iota[n] * np.exp(logl)[:, None, None] * f
    mean, var = lam.mean(0), lam.var(0)
    se_mean = np.sqrt(var / N)
    se_var = np.sqrt((((lam - mean) ** 4).mean(0) - var ** 2) / N)
    assert np.all(np.abs(mean - Emap) < 5 * se_mean + 1e-9)
    assert np.all(np.abs(var - Vmap) < 5 * se_var + 1e-9)
    # V scales as iota^2: with iota in V instead, the variance would be off by this factor
    assert abs(prob.img_iota[n] - 1) * Vmap.max() > 20 * se_var.max()


@pytest.mark.parametrize("s", [1, 4])
def test_gradient_matches_central_differences_under_general_wcs(sk, s):
    """The oracle's reverse-mode gradient of L_s against central differences (h = 1e-5) in
    every coordinate on the skewed field: the chain rule through A (position and shape) and
    iota holds."""
    prob, m = sk
    theta = prob.theta0.copy()
    v, g = E.local_value_grad(m, theta, s)
    f = E.local_objective(m, theta, s)
    h = 1e-5
    base = torch.as_tensor(theta[s, :27], dtype=torch.float64)
    fd = np.zeros(27)
    for k in range(27):
        e = torch.zeros(27, dtype=torch.float64)
        e[k] = h
        fd[k] = (f(base + e).item() - f(base - e).item()) / (2 * h)
    scale = np.maximum(np.abs(g), 0.01 * np.abs(g).max())
    assert np.all(np.abs(fd - g) <= 1e-5 * scale + 1e-6), np.abs(fd - g) / scale
