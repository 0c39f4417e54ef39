"""Pins of the oracle's spatially varying PSF (oracle/psf.py; Section 2.2.2 and Table 1:
eigen-images with smoothly varying loadings; Section 2.2.3: a Gaussian-mixture PSF)
against closed forms, numpy's weighted moments, scipy densities and invariants of
expectation-maximisation."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import psf as OP
from synth import gen


def _knots(side):
    """Offsets of the knots from the centre: row i, column j at (j - c, i - c)."""
    c = (side - 1) / 2
    i, j = np.mgrid[0:side, 0:side]
    return j - c, i - c


def _render(mix, side):
    """Density of a mixture at the knots, by scipy (independent of the oracle)."""
    dx, dy = _knots(side)
    pts = np.stack([dx.ravel(), dy.ravel()], 1)
    out = np.zeros(side * side)
    for w, mx, my, cxx, cxy, cyy in mix:
        out += w * stats.multivariate_normal([mx, my], [[cxx, cxy], [cxy, cyy]]).pdf(pts)
    return out.reshape(side, side)


@pytest.fixture(scope="module")
def small():
    return gen.config_eigen_small()


def test_loading_convention_and_reconstruction():
    """The PSF at (x, y) is sum_e loading_e eigen_e with loading_e quadratic in (x/W, y/H):
    with one-hot eigen-images each knot shows one loading, which must equal the polynomial
    evaluated by hand; negative values are clipped."""
    side, W, H = 5, 200.0, 120.0
    eig = np.zeros((4, side, side))
    for e in range(4):
        eig[e, e, e] = 1.0
    coef = np.array([[1, 2, 3, 4, 5, 6], [-1, 0, 0, 0, 0, 0], [0.5, -1, 0.25, 0, 2, 0], [0, 0, 0, 1, 1, 1]],
                    dtype=float)
    x, y = 37.0, 91.0
    u, v = x / W, y / H
    img = OP.psf_image(eig, coef, W, H, x, y)
    want = [1 + 2 * u + 3 * v + 4 * u * u + 5 * u * v + 6 * v * v, -1.0, 0.5 - u + 0.25 * v + 2 * u * v,
            u * u + u * v + v * v]
    for e in range(4):
        assert img[e, e] == pytest.approx(max(want[e], 0.0), rel=1e-14, abs=1e-15)
    assert np.count_nonzero(img) == 3


def test_knot_layout():
    """Knot (row i, column j) lies at the offset (x, y) = (j - c, i - c) from the source: a
    PSF with all its weight on row 2, column 7 of an 11 x 11 grid has its one-component fit
    centred at (2, -3)."""
    img = np.zeros((11, 11))
    img[2, 7] = 1.0
    img[2, 8] = 1.0
    mix = OP.fit_mixture(img, 1, 0)
    assert np.allclose(mix[0, 1:3], [2.5, -3.0], atol=1e-15)
    assert mix[0, 3] == pytest.approx(0.25) and mix[0, 4] == 0.0 and mix[0, 5] == 0.0


@pytest.mark.parametrize("n_iter", [0, 1, 7])
def test_single_component_is_the_weighted_moments(small, n_iter):
    """K = 1: the start and every EM step give the image's weighted mean and covariance
    (closed form of the maximum-likelihood normal), computed here by numpy's weighted
    average and covariance."""
    n = 1
    img = OP.psf_image(small.psf_eigen[n], small.psf_coef[n], small.img_W[n], small.img_H[n], 70.0, 211.0)
    mix = OP.fit_mixture(img, 1, n_iter)
    dx, dy = _knots(img.shape[0])
    w = img.ravel()
    m = [np.average(dx.ravel(), weights=w), np.average(dy.ravel(), weights=w)]
    C = np.cov(np.stack([dx.ravel(), dy.ravel()]), aweights=w, bias=True)
    assert mix[0, 0] == 1.0
    assert np.allclose(mix[0, 1:3], m, rtol=0, atol=1e-12)
    assert np.allclose(mix[0, [3, 4, 5]], [C[0, 0], C[0, 1], C[1, 1]], rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_em_increases_its_objective_and_keeps_unit_mass(small, K):
    """EM never decreases sum_p w_p log(mixture density at p); weights sum to one."""
    n = 2
    img = OP.psf_image(small.psf_eigen[n], small.psf_coef[n], small.img_W[n], small.img_H[n], 200.0, 30.0)
    hist = []
    mix = OP.fit_mixture(img, K, 40, history=hist)
    assert np.all(np.diff(hist) >= -1e-12 * abs(hist[-1]))
    assert hist[-1] > hist[0]
    assert abs(mix[:, 0].sum() - 1.0) < 1e-15
    assert np.all(mix[:, 3] > 0) and np.all(mix[:, 3] * mix[:, 5] - mix[:, 4] ** 2 > 0)


def test_recovers_a_separated_two_component_mixture():
    """Knot values rendered from a known two-component mixture (scipy), sigma >= 1.4 px so
    the unit grid holds its moments to ~1e-15: the two-component fit recovers it."""
    truth = np.array([[0.35, -6.0, 1.0, 2.0, 0.4, 1.5], [0.65, 5.0, 3.0, 3.0, -0.6, 2.2]])
    img = _render(truth, 41)
    mix = OP.fit_mixture(img, 2, 400)
    mix = mix[np.argsort(mix[:, 1])]
    assert np.allclose(mix, truth, rtol=0, atol=2e-6), mix - truth


def test_fit_is_close_to_the_psf_and_normalised(small):
    """The three-component fit (30 iterations) at positions across each image stays within
    2% in L2 of the eigen-PSF there, and sums to one over a wide grid (it is a density
    sampled on unit knots)."""
    rng = np.random.default_rng(4)
    for n in range(small.n_images):
        for _ in range(3):
            x, y = rng.uniform(0, small.img_W[n]), rng.uniform(0, small.img_H[n])
            img = OP.psf_image(small.psf_eigen[n], small.psf_coef[n], small.img_W[n], small.img_H[n], x, y)
            mix = OP.fit_mixture(img, 3, 30)
            dens = _render(mix, img.shape[0])
            rel = np.linalg.norm(dens - img / img.sum()) / np.linalg.norm(img / img.sum())
            assert rel < 0.02, rel
            # a density: its sum over unit knots is one up to the aliasing error
            # 2 exp(-2 pi^2 sigma^2) of its narrowest direction
            smin = min(np.linalg.eigvalsh([[m[3], m[4]], [m[4], m[5]]]).min() for m in mix)
            assert abs(_render(mix, 121).sum() - 1.0) < 2 * math.exp(-2 * math.pi ** 2 * smin) + 1e-12


def test_fit_keeps_the_psf_covariance_and_follows_its_drift(small):
    """The fitted mixture's overall covariance equals the eigen-PSF's weighted covariance at
    that position within 3% (the fit is a likelihood fit, not a moment match, for K > 1),
    and it changes between opposite corners of the frame as the PSF drifts."""
    n = 0
    W, H = small.img_W[n], small.img_H[n]
    covs = []
    for x, y in [(20.0, 20.0), (240.0, 280.0)]:
        img = OP.psf_image(small.psf_eigen[n], small.psf_coef[n], W, H, x, y)
        dx, dy = _knots(img.shape[0])
        cm = np.cov(np.stack([dx.ravel(), dy.ravel()]), aweights=img.ravel(), bias=True)
        mix = OP.fit_mixture(img, 3, 30)
        mbar = (mix[:, 0:1] * mix[:, 1:3]).sum(0)
        cfit = sum(m[0] * (np.array([[m[3], m[4]], [m[4], m[5]]]) + np.outer(m[1:3], m[1:3])) for m in mix) \
            - np.outer(mbar, mbar)
        assert np.allclose(cfit, cm, rtol=0.03, atol=0.03)
        covs.append(cfit)
    assert np.abs(covs[0] - covs[1]).max() > 0.05
