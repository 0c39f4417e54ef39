"""Reference spatially varying PSF: reconstruction from eigen-images and a Gaussian-mixture
fit, float64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): the product path never imports this.

Follows Section 2.2.2 and Table 1 of the paper: an image's PSF is given by E principal
images ("eigen-images") on a grid of side x side knots centred on a light source, and by
loadings that vary smoothly over the image; Section 2.2.3 approximates the PSF by a mixture
of bivariate normals so that the light of a galaxy convolved with it stays analytic.

Readings of what the paper leaves open:
  * the loading of eigen-image e at pixel position (x, y) of an image of W columns and H
    rows is a quadratic in u = x / W, v = y / H: sum_t coef[e, t] m_t with
    m = (1, u, v, u^2, u v, v^2);
  * knot (i, j) of the grid lies at the offset (dx, dy) = (j - c, i - c) pixels from the
    source, c = (side - 1) / 2; the PSF at a position is sum_e loading_e * eigen_e, its
    negative values (principal-component ringing) clipped to zero;
  * the mixture is fitted by expectation-maximisation with the clipped image as weights at
    the knots, from a start made of the image's moments (every component at the centroid,
    component k's covariance the image's second central moment times 2^(k - (K-1)/2),
    equal weights), for a fixed number of iterations; a component whose weight drops to
    1e-12 or below is left as it was;
  * the fitted weights sum to one (a star's photons all fall somewhere), and the means are
    offsets from the source's position;
  * the PSF of a source in an image is the fit at the centre of the source's patch there,
    fixed during inference.
"""
from __future__ import annotations

import numpy as np

MAX_PSF = 4


def loadings(coef, W, H, x, y):
    """Loadings [E] at pixel position (x, y): quadratic in (x / W, y / H)."""
    u, v = x / W, y / H
    m = np.array([1.0, u, v, u * u, u * v, v * v])
    return np.asarray(coef, dtype=np.float64) @ m


def psf_image(eigen, coef, W, H, x, y):
    """The PSF at (x, y) as weights on the knot grid: sum_e loading_e eigen_e, clipped at 0."""
    img = np.tensordot(loadings(coef, W, H, x, y), np.asarray(eigen, dtype=np.float64), axes=1)
    return np.maximum(img, 0.0)


def knot_offsets(side):
    c = (side - 1) / 2.0
    i, j = np.mgrid[0:side, 0:side]
    return (j - c).astype(np.float64), (i - c).astype(np.float64)


def _density(dx, dy, mx, my, cxx, cxy, cyy):
    det = cxx * cyy - cxy * cxy
    ex, ey = dx - mx, dy - my
    q = (cyy * ex * ex - 2.0 * cxy * ex * ey + cxx * ey * ey) / det
    return np.exp(-0.5 * q) / (2.0 * np.pi * np.sqrt(det))


def em_start(wts, dx, dy, K):
    """Moment start: all K components at the centroid, covariances the image's second
    central moment scaled by 2^(k - (K-1)/2), weights 1/K.  Returns [K, 6]."""
    M = wts.sum()
    mx, my = (wts * dx).sum() / M, (wts * dy).sum() / M
    cxx = (wts * (dx - mx) ** 2).sum() / M
    cxy = (wts * (dx - mx) * (dy - my)).sum() / M
    cyy = (wts * (dy - my) ** 2).sum() / M
    out = np.zeros((K, 6))
    for k in range(K):
        f = 2.0 ** (k - (K - 1) / 2.0)
        out[k] = [1.0 / K, mx, my, f * cxx, f * cxy, f * cyy]
    return out


def em_objective(wts, dx, dy, mix):
    """sum_p w_p log sum_k weight_k N(p; mean_k, cov_k): the quantity EM increases."""
    dens = sum(m[0] * _density(dx, dy, *m[1:]) for m in mix)
    return float((wts * np.log(np.maximum(dens, 1e-300))).sum())


def em_step(wts, dx, dy, mix):
    """One expectation-maximisation step of a Gaussian mixture on weighted points."""
    K = len(mix)
    comp = np.array([m[0] * _density(dx, dy, *m[1:]) for m in mix])       # [K, side, side]
    tot = comp.sum(0)
    resp = np.where(tot > 0, comp / np.where(tot > 0, tot, 1.0), 0.0)
    M = wts.sum()
    out = np.array(mix, dtype=np.float64).copy()
    for k in range(K):
        r = wts * resp[k]
        nk = r.sum()
        if nk <= 1e-12 * M:
            continue
        mx, my = (r * dx).sum() / nk, (r * dy).sum() / nk
        out[k] = [nk / M, mx, my, (r * (dx - mx) ** 2).sum() / nk, (r * (dx - mx) * (dy - my)).sum() / nk,
                  (r * (dy - my) ** 2).sum() / nk]
    return out


def fit_mixture(img, K, n_iter, history=None):
    """K-component Gaussian mixture fitted to the knot weights `img` [side, side]: rows of
    (weight, mean_x, mean_y, cov_xx, cov_xy, cov_yy), weights summing to one.  `history`
    (a list) receives the EM objective before each step and at the end."""
    side = img.shape[0]
    dx, dy = knot_offsets(side)
    wts = np.asarray(img, dtype=np.float64)
    mix = em_start(wts, dx, dy, K)
    for _ in range(n_iter):
        if history is not None:
            history.append(em_objective(wts, dx, dy, mix))
        mix = em_step(wts, dx, dy, mix)
    if history is not None:
        history.append(em_objective(wts, dx, dy, mix))
    mix[:, 0] /= mix[:, 0].sum()
    return mix


def patch_psfs(prob, K, n_iter):
    """The PSF mixture of every patch of a problem with eigen-PSFs: the fit at the centre of
    the patch, [P, 4, 6] (rows beyond K zero)."""
    out = np.zeros((prob.n_patches, MAX_PSF, 6))
    for p in range(prob.n_patches):
        n = int(prob.patch_img[p])
        x = prob.patch_x0[p] + (prob.patch_w[p] - 1) / 2.0
        y = prob.patch_y0[p] + (prob.patch_h[p] - 1) / 2.0
        img = psf_image(prob.psf_eigen[n], prob.psf_coef[n], float(prob.img_W[n]), float(prob.img_H[n]), x, y)
        out[p, :K] = fit_mixture(img, K, n_iter)
    return out
