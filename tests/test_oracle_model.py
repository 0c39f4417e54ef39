"""Pins of the oracle's model arithmetic against closed forms, library routines and brute
force (no GPU).  Each test names the passage it pins."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import elbo as E
from synth import gen


@pytest.fixture(scope="module")
def c1():
    p = gen.config1()
    return p, E.Model(p)


def _nat_row(theta):
    return E.natural(torch.as_tensor(theta, dtype=torch.float64))


def test_profiles_normalised_and_half_light_radius_one():
    """Galaxy profile constants (Section 2.1.2, equation hsi): weights sum to 1 and an
    isotropic mixture with Sigma = I holds half its light inside radius 1:
    sum_j alpha_j exp(-1/(2 tau_j)) = 1/2 (closed form for the enclosed fraction)."""
    ea, et, da, dt = gen.load_profiles()
    for a, t in ((ea, et), (da, dt)):
        assert abs(a.sum() - 1) < 1e-12
        assert abs(np.sum(a * np.exp(-1 / (2 * t))) - 0.5) < 1e-10
        # and by brute-force radial integration of the density
        r = np.linspace(0, 1, 200001)
        dens = np.sum(a[:, None] * np.exp(-r[None] ** 2 / (2 * t[:, None])) / (2 * math.pi * t[:, None]), 0)
        inside = np.trapezoid(2 * math.pi * r * dens, r)
        assert abs(inside - 0.5) < 2e-4


@pytest.mark.parametrize("s", [0, 1])
def test_mixtures_integrate_to_one_and_moments(c1, s):
    """f_nms of a star (PSF at u) and of a galaxy (Gaussian-Gaussian convolution) are
    densities over the pixel grid (Section 2.2.3): their sum over pixel centres is 1 to
    within the aliasing error 2 exp(-2 pi^2 sigma^2) < 1e-7 (sigma >= 1 px).  Their first
    moment is A u + b (+ PSF offsets) and the galaxy's second moment is the PSF covariance
    plus (sum_j weight_j tau_j) A Sigma_s A^T with Sigma_s built from its eigenvectors
    (cos t, -sin t) [radius^2] and (sin t, cos t) [(axis radius)^2] (Section 2.1.2)."""
    prob, m = c1
    theta = prob.theta0.copy()
    theta[s, 0:2] = [16.3, 15.7]
    theta[s, 24] = math.log(1.7)
    theta[s, 23] = 0.6
    theta[s, 26] = E.torch.logit(torch.tensor(0.45, dtype=torch.float64)).item()
    nat = _nat_row(theta)
    n = 3
    half = 120
    x0, y0 = 16 - half, 16 - half
    f0, f1 = E.source_profiles(m, nat, s, n, x0, y0, 2 * half, 2 * half)
    f0, f1 = f0.numpy(), f1.numpy()
    assert abs(f1.sum() - 1) < 1e-7
    assert abs(f0.sum() - 1) < 1e-7
    cols = np.arange(x0, x0 + 2 * half)[None, :].astype(float)
    rows = np.arange(y0, y0 + 2 * half)[:, None].astype(float)
    A, b = prob.img_A[n], prob.img_b[n]
    mu = A @ theta[s, 0:2] + b
    K = prob.img_npsf[n]
    psf = prob.img_psf[n, :K]
    off = (psf[:, 0:1] * psf[:, 1:3]).sum(0)
    for f in (f0, f1):
        assert abs((f * cols).sum() - (mu[0] + off[0])) < 1e-6
        assert abs((f * rows).sum() - (mu[1] + off[1])) < 1e-6
    # second central moment of the galaxy profile
    dx, dy = cols - (f0 * cols).sum(), rows - (f0 * rows).sum()
    mom = np.array([[(f0 * dx * dx).sum(), (f0 * dx * dy).sum()], [(f0 * dx * dy).sum(), (f0 * dy * dy).sum()]])
    psf_cov = sum(psf[k, 0] * np.array([[psf[k, 3], psf[k, 4]], [psf[k, 4], psf[k, 5]]]) for k in range(K))
    ea, et, da, dt = gen.load_profiles()
    prof = 1 / (1 + math.exp(-theta[s, 25]))
    ctau = prof * np.sum(da * dt) + (1 - prof) * np.sum(ea * et)
    t, r, ax = theta[s, 23], math.exp(theta[s, 24]), 1 / (1 + math.exp(-theta[s, 26]))
    v1, v2 = np.array([math.cos(t), -math.sin(t)]), np.array([math.sin(t), math.cos(t)])
    sig = r * r * np.outer(v1, v1) + (ax * r) ** 2 * np.outer(v2, v2)
    want = psf_cov + ctau * A @ sig @ A.T
    assert np.allclose(mom, want, rtol=1e-6, atol=1e-6)


def test_sky_bilinear_reproduces_planar_field():
    """Sky interpolated linearly from the knot grid (Section 2.2.1): the generator's sky is
    a plane, which bilinear interpolation reproduces exactly at every pixel."""
    prob = gen.config2(n_sources=6)
    m = E.Model(prob)
    rng = np.random.default_rng(0)
    for p in rng.choice(prob.n_patches, 8, replace=False):
        n = prob.patch_img[p]
        # reconstruct the generator's plane from its corner knots (independent of the oracle)
        o = prob.img_sky_off[n]
        k = prob.sky_knots[o:o + 4].reshape(2, 2)
        H, W = prob.img_H[n], prob.img_W[n]
        rows = np.arange(prob.patch_y0[p], prob.patch_y0[p] + prob.patch_h[p])[:, None] / (H - 1)
        cols = np.arange(prob.patch_x0[p], prob.patch_x0[p] + prob.patch_w[p])[None, :] / (W - 1)
        plane = k[0, 0] + (k[1, 0] - k[0, 0]) * rows + (k[0, 1] - k[0, 0]) * cols
        assert np.allclose(m.sky(p).numpy(), plane, rtol=1e-13, atol=1e-10)


def test_isolated_star_degenerate_q_is_exact_poisson(c1):
    """With q concentrated on 'star' and on a single flux/colour value, the delta-method
    expected log likelihood (equation eq:log_p_last, Section 4.2.2) reduces to the exact
    Poisson log-likelihood sum_m log Poisson(x_m; sky + l f_m).  The reference value uses
    scipy's Poisson pmf, scipy's normal pdf for the PSF and the generator's own colour ->
    band-flux map."""
    prob, m = c1
    theta = prob.theta0.copy()
    s = 0
    theta[s, 2] = 40.0                       # a -> 1 (star)
    theta[s, 5:7] = -40.0                    # log-flux variances -> 0
    theta[s, 15:23] = -40.0                  # colour variances -> 0
    nat = _nat_row(theta)
    for n in range(prob.n_images):
        p = [q for q in range(prob.n_patches) if prob.patch_src[q] == s and prob.patch_img[q] == n][0]
        x0, y0, w, h = prob.patch_x0[p], prob.patch_y0[p], prob.patch_w[p], prob.patch_h[p]
        # oracle: only this source (the galaxy is dropped to isolate the star)
        Es, Vs = E.source_rate_moments(m, nat, s, n, x0, y0, w, h)
        Ex = m.sky(p) + Es
        got = E.pixel_terms(m.pixels(p), Ex, Vs).sum().item()
        # independent: exact Poisson likelihood
        flux = gen.band_fluxes(math.exp(theta[s, 4]), theta[s, 11:15])[prob.img_band[n]] * prob.img_iota[n]
        mu = prob.img_A[n] @ theta[s, 0:2] + prob.img_b[n]
        yy, xx = np.mgrid[y0:y0 + h, x0:x0 + w]
        pts = np.stack([xx.ravel(), yy.ravel()], 1).astype(float)
        psf = 0
        for k in range(prob.img_npsf[n]):
            w_, mx, my, cxx, cxy, cyy = prob.img_psf[n, k]
            psf = psf + w_ * stats.multivariate_normal(mu + [mx, my], [[cxx, cxy], [cxy, cyy]]).pdf(pts)
        lam = m.sky(p).numpy().ravel() + flux * psf
        want = stats.poisson.logpmf(prob.patch_pixels(p).ravel().astype(int), lam).sum()
        assert abs(got - want) <= 1e-10 * abs(want)


def test_rate_moments_match_monte_carlo():
    """E_q[lambda] (equation conditional) and V_q[lambda] (equation vareq) against brute
    force: sample the type, log flux and colours from q, form lambda = sky + sum_s l_s f_s
    with the generator's colour -> band-flux map, and compare mean and variance per pixel
    within 5 standard errors.  Two overlapping sources on a 5x5 patch."""
    prob = gen.config1()
    m = E.Model(prob)
    theta = prob.theta0.copy()
    theta[:, 2] = [0.4, -0.7]
    theta[:, 5:7] = np.log([[0.08, 0.03], [0.05, 0.12]])
    theta[:, 15:23] = np.log(np.linspace(0.02, 0.2, 8))[None, :]
    nat = _nat_row(theta)
    n = 1
    p0 = [q for q in range(prob.n_patches) if prob.patch_src[q] == 0 and prob.patch_img[q] == n][0]
    x0, y0 = 14, 13
    Emap = m.sky(p0)[y0:y0 + 5, x0:x0 + 5].clone()
    Vmap = torch.zeros_like(Emap)
    fs = []
    for s in range(2):
        Es, Vs = E.source_rate_moments(m, nat, s, n, x0, y0, 5, 5)
        Emap += Es
        Vmap += Vs
        fs.append([f.numpy() for f in E.source_profiles(m, nat, s, n, x0, y0, 5, 5)])
    rng = np.random.default_rng(7)
    N = 400000
    lam = np.tile(m.sky(p0)[y0:y0 + 5, x0:x0 + 5].numpy()[None], (N, 1, 1))
    band = prob.img_band[n]
    for s in range(2):
        a = 1 / (1 + np.exp(-theta[s, 2]))
        star = rng.random(N) < a
        i = star.astype(int)
        logr = theta[s, 3 + i] + np.sqrt(np.exp(theta[s, 5 + i])) * rng.standard_normal(N)
        cm = np.where(star[:, None], theta[s, 11:15], theta[s, 7:11])
        cv = np.where(star[:, None], np.exp(theta[s, 19:23]), np.exp(theta[s, 15:19]))
        c = cm + np.sqrt(cv) * rng.standard_normal((N, 4))
        ell = np.array([gen.band_fluxes(math.exp(lr), cc)[band] for lr, cc in zip(logr[:20000], c[:20000])])
        # vectorised version of the same generator map, checked on the first 20000 draws
        refb = gen.REF_BAND
        logl = logr.copy()
        if band > refb:
            logl = logl + c[:, refb:band].sum(1)
        elif band < refb:
            logl = logl - c[:, band:refb].sum(1)
        assert np.allclose(np.exp(logl[:20000]), ell, rtol=1e-12)
        f = np.where(star[:, None, None], fs[s][1][None], fs[s][0][None])
        lam += prob.img_iota[n] * np.exp(logl)[:, None, None] * f
    mean, var = lam.mean(0), lam.var(0)
    se_mean = np.sqrt(var / N)
    fourth = ((lam - mean) ** 4).mean(0)
    se_var = np.sqrt((fourth - var ** 2) / N)
    assert np.all(np.abs(mean - Emap.numpy()) < 5 * se_mean + 1e-9)
    assert np.all(np.abs(var - Vmap.numpy()) < 5 * se_var + 1e-9)
    assert Vmap.numpy().max() > 1.0   # the check is not vacuous


def test_delta_method_close_to_monte_carlo_log_rate():
    """The delta-method E_q[log lambda] (Section 4.2.2) is an approximation, not exact:
    sanity check only, against Monte Carlo, within the size of the third-order Taylor term.
    Parity of the oracle with the true expectation is unpinned by design."""
    rng = np.random.default_rng(3)
    sky, L, v = 100.0, 400.0, 0.05
    logl = math.log(L) + math.sqrt(v) * rng.standard_normal(2_000_000)
    lam = sky + np.exp(logl)
    Ev = sky + L * math.exp(v / 2)
    Vv = L * L * math.exp(v) * (math.exp(v) - 1)
    approx = math.log(Ev) - Vv / (2 * Ev * Ev)
    third = np.mean((lam - Ev) ** 3) / Ev ** 3 / 3
    assert abs(np.log(lam).mean() - approx) < abs(third) + 1e-3


def test_zero_counts_pixel_term():
    """x = 0 gives -E[lambda] exactly (0 log 0 := 0, log 0! = 0)."""
    x = torch.zeros(3, dtype=torch.float64)
    Ev = torch.tensor([1.0, 50.0, 200.0], dtype=torch.float64)
    Vv = torch.tensor([0.5, 3.0, 10.0], dtype=torch.float64)
    assert torch.equal(E.pixel_terms(x, Ev, Vv), -Ev)


def test_union_counted_once_matches_dense_canvas():
    """The global objective counts each pixel of the union of patches once (the sum over
    pixels in equation eq:log_p_last): compare the owner-rule total with a dense canvas per
    image on which every source's light is splatted over its patch and the union is
    masked."""
    prob = gen.config2(n_sources=7)
    m = E.Model(prob)
    theta = torch.as_tensor(prob.theta0)
    total, _ = E.elbo(m, theta)
    nat = E.natural(theta)
    kl = E.kl_terms(m, nat)["total"].sum().item()
    acc = 0.0
    for n in range(prob.n_images):
        ps = [p for p in range(prob.n_patches) if prob.patch_img[p] == n]
        X0 = min(prob.patch_x0[p] for p in ps); Y0 = min(prob.patch_y0[p] for p in ps)
        X1 = max(prob.patch_x0[p] + prob.patch_w[p] for p in ps)
        Y1 = max(prob.patch_y0[p] + prob.patch_h[p] for p in ps)
        Ec = torch.zeros((Y1 - Y0, X1 - X0), dtype=torch.float64)
        Vc = torch.zeros_like(Ec)
        Xc = torch.zeros_like(Ec)
        Sc = torch.zeros_like(Ec)
        mask = torch.zeros_like(Ec, dtype=torch.bool)
        for p in ps:
            x0, y0, w, h = prob.patch_x0[p], prob.patch_y0[p], prob.patch_w[p], prob.patch_h[p]
            sl = (slice(y0 - Y0, y0 - Y0 + h), slice(x0 - X0, x0 - X0 + w))
            Es, Vs = E.source_rate_moments(m, nat, prob.patch_src[p], n, x0, y0, w, h)
            Ec[sl] += Es
            Vc[sl] += Vs
            Xc[sl] = m.pixels(p)
            Sc[sl] = m.sky(p)
            mask[sl] = True
        T = E.pixel_terms(Xc, Ec + Sc, Vc)
        acc += T[mask].sum().item()
    assert abs((acc - kl) - total.item()) <= 1e-11 * abs(total.item())
