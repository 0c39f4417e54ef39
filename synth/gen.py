"""Seeded synthetic problems shaped like the paper's workloads.

This module is the ONLY code shared by the reference oracle and the HIP path, and it
holds none of the method's arithmetic: no light-kernel densities, no rates, no ELBO.
Pixels are produced by simulating the generative process of Section 2 photon by photon:
each source emits Poisson(iota * band flux) photons, each photon's sky offset is drawn
from the galaxy light kernel (a component of the profile mixture, then a scaled and
rotated normal vector), mapped to the pixel frame by the image's affine WCS, blurred by
a draw from the image's PSF mixture and binned to the nearest pixel centre; skyglow adds
Poisson counts from a smooth rate field per image (a plane, optionally with an
undulation, sampled on the image's sky knot grid).  The problem arrays follow
the layout documented in include/celmi.h.

Workloads (seed = 180300110 + k for workload k):
  1 "plain":   1 star + 1 galaxy, 5 bands, one 32x32 image per band, sky 100.
  2 "batched": 1000 sources in overlapping groups of 1-5, square patches of side 20-60,
               5 bands x 2 epochs, power-law fluxes, sky 50-200.
  3 "adjoint": 4096 sources, same grouping, side 16-64, 5 bands, 1 epoch.
  4 "field":   one 2048x1489 field, 5 bands x 3 epochs (offsets up to 20 px, small
               rotations), ~600 uniformly placed sources, 70% galaxies.
  5 "serving": region requests of 1-200 sources, side 16-96, 5 bands.
  6 "skew":    a small blended field with general WCS, calibration, sky grid and PSF
               (config_skew).
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
N_BANDS = 5
REF_BAND = 2          # r band, 0-based (u, g, r, i, z)
N_COLOURS = 4
N_THETA = 32
N_COLOUR_COMPONENTS = 8
MAX_PSF = 4
SEED_BASE = 180300110
SURVEY_PRIOR_SEED = SEED_BASE + 55   # the prior every region request of one survey shares


def load_profiles():
    with open(os.path.join(HERE, "profiles.json")) as f:
        p = json.load(f)
    return (np.array(p["exp"]["alpha"]), np.array(p["exp"]["tau"]),
            np.array(p["dev"]["alpha"]), np.array(p["dev"]["tau"]))


@dataclass
class Problem:
    """A cataloging problem: images, per-source patches of observed pixels, priors and an
    initial variational parameter vector per source.  Plain numpy; no method arithmetic."""
    n_sources: int
    # images [N]
    img_band: np.ndarray      # int32 band index 0..4
    img_H: np.ndarray         # int32 rows
    img_W: np.ndarray         # int32 cols
    img_npsf: np.ndarray      # int32 number of PSF components (<= 4)
    img_psf: np.ndarray       # f64 [N,4,6]: weight, mean_x, mean_y, cov_xx, cov_xy, cov_yy (pixels)
    img_A: np.ndarray         # f64 [N,2,2]: pixel = A @ u + b
    img_b: np.ndarray         # f64 [N,2]
    img_iota: np.ndarray      # f64 [N] expected counts per flux unit
    img_sky_qh: np.ndarray    # int32 sky knot rows
    img_sky_qw: np.ndarray    # int32 sky knot cols
    img_sky_off: np.ndarray   # int64 offset into sky_knots
    sky_knots: np.ndarray     # f64 concatenated row-major knot grids
    # patches [P], sorted by (source, image)
    patch_src: np.ndarray     # int32
    patch_img: np.ndarray     # int32
    patch_x0: np.ndarray      # int32 first column
    patch_y0: np.ndarray      # int32 first row
    patch_w: np.ndarray       # int32
    patch_h: np.ndarray       # int32
    patch_off: np.ndarray     # int64 offset of the patch's first pixel in `pixels`
    pixels: np.ndarray        # f32 counts, row-major within each patch
    # prior hyperparameters
    prior_a: float            # prior probability of a star
    prior_r: np.ndarray       # f64 [2,2]: per type (0 galaxy, 1 star) mean, variance of log r
    prior_cw: np.ndarray      # f64 [2,J] colour GMM weights
    prior_cmean: np.ndarray   # f64 [2,J,4]
    prior_ccov: np.ndarray    # f64 [2,J,4,4]
    prior_radius: np.ndarray  # f64 [2]: mean, variance of log radius
    prior_profile: np.ndarray  # f64 [2]: Beta parameters
    prior_axis: np.ndarray    # f64 [2]: Beta parameters
    # galaxy profile mixtures
    exp_alpha: np.ndarray
    exp_tau: np.ndarray
    dev_alpha: np.ndarray
    dev_tau: np.ndarray
    # initial variational parameters [S,32] (unconstrained coordinates)
    theta0: np.ndarray
    truth: dict = field(default_factory=dict)
    name: str = ""
    # spatially varying PSF (None: each image's PSF is img_psf everywhere): eigen-images
    # [N, E, 51, 51] and quadratic loading coefficients [N, E, 6] per image
    psf_eigen: np.ndarray = None
    psf_coef: np.ndarray = None

    @property
    def n_images(self):
        return int(self.img_band.shape[0])

    @property
    def n_patches(self):
        return int(self.patch_src.shape[0])

    @property
    def n_units(self):
        return int(np.sum(self.patch_w.astype(np.int64) * self.patch_h))

    def patch_pixels(self, p):
        o = int(self.patch_off[p])
        h, w = int(self.patch_h[p]), int(self.patch_w[p])
        return self.pixels[o:o + h * w].reshape(h, w)


# ----------------------------------------------------------------------------------------
# hyperparameters

def make_prior(rng, star_prob=0.3, log_r_gal=(math.log(3e3), 1.0), log_r_star=(math.log(5e3), 1.2)):
    J = N_COLOUR_COMPONENTS
    cw = np.stack([rng.dirichlet(np.full(J, 3.0)) for _ in range(2)])
    cmean = np.zeros((2, J, N_COLOURS))
    ccov = np.zeros((2, J, N_COLOURS, N_COLOURS))
    for i in range(2):
        for j in range(J):
            if i == 1:   # stars: near a one-dimensional temperature sequence
                t = rng.uniform(-0.5, 1.5)
                cmean[i, j] = np.array([1.0, 0.5, 0.2, 0.1]) * t + np.array([0.8, 0.2, 0.05, 0.0])
                scale = 0.05
            else:        # galaxies: broader
                cmean[i, j] = rng.normal([1.2, 0.6, 0.3, 0.2], 0.3)
                scale = 0.15
            L = rng.normal(0, scale, (N_COLOURS, N_COLOURS))
            ccov[i, j] = L @ L.T + np.eye(N_COLOURS) * scale ** 2
    return dict(
        prior_a=float(star_prob),
        prior_r=np.array([log_r_gal, log_r_star], dtype=np.float64),
        prior_cw=cw, prior_cmean=cmean, prior_ccov=ccov,
        prior_radius=np.array([math.log(2.0), 0.4 ** 2]),
        prior_profile=np.array([1.5, 1.5]),
        prior_axis=np.array([4.0, 2.0]),
    )


def draw_gmm(rng, w, mean, cov):
    j = rng.choice(len(w), p=w)
    return rng.multivariate_normal(mean[j], cov[j])


def band_fluxes(r, colours):
    """Fluxes in the five bands from the reference-band flux and the four colours, each
    colour being the natural log of the ratio of the flux in band b+1 to the flux in b."""
    out = np.zeros(N_BANDS)
    out[REF_BAND] = r
    for b in range(REF_BAND, N_BANDS - 1):
        out[b + 1] = out[b] * math.exp(colours[b])
    for b in range(REF_BAND - 1, -1, -1):
        out[b] = out[b + 1] * math.exp(-colours[b])
    return out


def make_psf(rng, npsf=3):
    sig = np.sort(rng.uniform(1.0, 3.0, npsf))
    w = rng.dirichlet(np.full(npsf, 2.0))
    psf = np.zeros((MAX_PSF, 6))
    for k in range(npsf):
        psf[k] = [w[k], 0.0, 0.0, sig[k] ** 2, 0.0, sig[k] ** 2]
    return psf


# ----------------------------------------------------------------------------------------
# photon simulation

def _galaxy_offsets(rng, n, src, profiles):
    exp_a, exp_t, dev_a, dev_t = profiles
    is_dev = rng.random(n) < src["profile"]
    comp_dev = rng.choice(len(dev_a), size=n, p=dev_a)
    comp_exp = rng.choice(len(exp_a), size=n, p=exp_a)
    tau = np.where(is_dev, dev_t[comp_dev], exp_t[comp_exp])
    z = rng.standard_normal((n, 2)) * np.sqrt(tau)[:, None]
    # scale to the axes (radius, axis*radius) and rotate by R^T, R = [[c,-s],[s,c]]
    z[:, 0] *= src["radius"]
    z[:, 1] *= src["radius"] * src["axis"]
    c, s = math.cos(src["angle"]), math.sin(src["angle"])
    return np.stack([c * z[:, 0] + s * z[:, 1], -s * z[:, 0] + c * z[:, 1]], axis=1)


def _psf_offsets(rng, n, psf, npsf):
    w = psf[:npsf, 0] / psf[:npsf, 0].sum()
    k = rng.choice(npsf, size=n, p=w)
    out = psf[k, 1:3].copy()
    for kk in range(npsf):
        sel = k == kk
        m = int(sel.sum())
        if m:
            cov = np.array([[psf[kk, 3], psf[kk, 4]], [psf[kk, 4], psf[kk, 5]]])
            out[sel] += rng.multivariate_normal(np.zeros(2), cov, size=m)
    return out


def psf_true_at(img, x, y):
    """The image's true PSF mixture at pixel position (x, y) when it varies over the frame
    (Section 2.2.2: the PSF has smooth spatial variation): each component's covariance is
    scaled by (1 + a u + b v + c u v)^2 and sheared, its mean shifted, u = x/W - 1/2,
    v = y/H - 1/2, with per-component drift coefficients drawn by the generator."""
    K = img["npsf"]
    out = np.array(img["psf"], dtype=np.float64).copy()
    u, v = x / img["W"] - 0.5, y / img["H"] - 0.5
    for k in range(K):
        d = img["psf_drift"][k]
        sc = (1.0 + d[0] * u + d[1] * v + d[2] * u * v) ** 2
        cxx, cxy, cyy = out[k, 3] * sc, out[k, 4] * sc, out[k, 5] * sc
        cxy += d[3] * u * math.sqrt(cxx * cyy)
        out[k, 3], out[k, 4], out[k, 5] = cxx, cxy, cyy
        out[k, 1] += d[4] * v
        out[k, 2] += d[5] * u
    return out


PSF_SIDE = 51         # knots per side of a PSF eigen-image (Table 1: F = 51 x 51)
N_EIGEN = 4           # eigen-images per image (Table 1: E = 4)
PSF_LOADING_TERMS = 6  # loadings are quadratic in position: 1, u, v, u^2, u v, v^2


def loading_monomials(img, x, y):
    """Monomials of the loading polynomial at pixel position (x, y), u = x/W, v = y/H."""
    u, v = x / img["W"], y / img["H"]
    return np.array([1.0, u, v, u * u, u * v, v * v])


def eigen_psf(rng, img, grid=5, photons=400_000, side=PSF_SIDE, n_eigen=N_EIGEN):
    """Stand-in for the survey's PSF preprocessing (Section 2.2.2: the PSF is fitted by
    pre-existing software and represented by the top principal components of the PSF
    rendered on a grid centred on a source, with loadings that vary smoothly over the
    image).  The PSF is rendered at a grid x grid set of positions by histogramming photon
    offsets drawn from the true PSF there (binned to the nearest pixel, the centre at the
    middle knot), the images' top principal components (uncentred, by SVD) are the
    eigen-images, and each loading is fitted by least squares as a quadratic in position.
    Returns (eigen [E, side, side], coefficients [E, 6])."""
    H, W = img["H"], img["W"]
    xs = np.linspace(0.05 * W, 0.95 * W, grid)
    ys = np.linspace(0.05 * H, 0.95 * H, grid)
    half = side // 2
    rows, mons = [], []
    for y in ys:
        for x in xs:
            off = _psf_offsets(rng, photons, psf_true_at(img, x, y), img["npsf"])
            c = np.rint(off[:, 0]).astype(np.int64) + half
            r = np.rint(off[:, 1]).astype(np.int64) + half
            ok = (c >= 0) & (c < side) & (r >= 0) & (r < side)
            im = np.zeros((side, side))
            np.add.at(im, (r[ok], c[ok]), 1.0)
            rows.append(im.ravel() / photons)
            mons.append(loading_monomials(img, x, y))
    X, Mo = np.array(rows), np.array(mons)
    U, S, Vt = np.linalg.svd(X, full_matrices=False)
    eig = Vt[:n_eigen]
    load = U[:, :n_eigen] * S[:n_eigen]
    coef = np.linalg.lstsq(Mo, load, rcond=None)[0].T        # [E, 6]
    return eig.reshape(n_eigen, side, side), coef


def render(rng, img, canvas, sources, profiles):
    """Counts on a canvas (y0, x0, h, w) of image `img` from skyglow and the given sources."""
    y0, x0, h, w = canvas
    rows = np.arange(y0, y0 + h, dtype=np.float64)[:, None]
    cols = np.arange(x0, x0 + w, dtype=np.float64)[None, :]
    sky = sky_field(img, rows, cols)
    counts = rng.poisson(np.maximum(sky, 0.0)).astype(np.int64)
    A, b = img["A"], img["b"]
    for src in sources:
        lam = img["iota"] * src["fluxes"][img["band"]]
        n = rng.poisson(lam)
        if n == 0:
            continue
        if src["star"]:
            off = np.zeros((n, 2))
        else:
            off = _galaxy_offsets(rng, n, src, profiles)
        pos = src["u"][None, :] + off
        pix = pos @ A.T + b[None, :]
        psf = psf_true_at(img, *(A @ src["u"] + b)) if "psf_drift" in img else img["psf"]
        pix = pix + _psf_offsets(rng, n, psf, img["npsf"])
        c = np.rint(pix[:, 0]).astype(np.int64) - x0
        r = np.rint(pix[:, 1]).astype(np.int64) - y0
        ok = (c >= 0) & (c < w) & (r >= 0) & (r < h)
        np.add.at(counts, (r[ok], c[ok]), 1)
    return counts


def sky_field(img, rows, cols):
    """The image's true skyglow rate at pixel centres (rows, cols broadcast): a plane, plus,
    when the image has one, a smooth undulation of relative amplitude sky_wave (a product of
    sines over the frame), so that a knot grid samples a field with curvature."""
    H, W = img["H"], img["W"]
    sky = img["sky0"] + img["sky_gy"] * (rows - H / 2) + img["sky_gx"] * (cols - W / 2)
    amp = img.get("sky_wave", 0.0)
    if amp:
        ph = img["sky_phase"]
        sky = sky * (1.0 + amp * np.sin(2 * math.pi * (rows / H * img["sky_ky"] + ph[0]))
                     * np.sin(2 * math.pi * (cols / W * img["sky_kx"] + ph[1])))
    return sky


def sky_knots_for(img, qh, qw):
    """Knot values of the image's sky field on a qh x qw grid spanning the corners."""
    H, W = img["H"], img["W"]
    ky = np.linspace(0, H - 1, qh) if qh > 1 else np.array([(H - 1) / 2.0])
    kx = np.linspace(0, W - 1, qw) if qw > 1 else np.array([(W - 1) / 2.0])
    return sky_field(img, ky[:, None], kx[None, :]) * np.ones((len(ky), len(kx)))


# ----------------------------------------------------------------------------------------
# truth and initialisation

def _logit(p):
    return math.log(p / (1 - p))


def draw_source(rng, prior, star, u, flux=None, radius=None, axis=None, profile=None, angle=None):
    i = 1 if star else 0
    if flux is None:
        flux = math.exp(rng.normal(prior["prior_r"][i, 0], math.sqrt(prior["prior_r"][i, 1])))
    colours = draw_gmm(rng, prior["prior_cw"][i], prior["prior_cmean"][i], prior["prior_ccov"][i])
    colours = np.clip(colours, -3.0, 3.0)
    if radius is None:
        radius = float(np.clip(math.exp(rng.normal(prior["prior_radius"][0],
                                                   math.sqrt(prior["prior_radius"][1]))), 0.5, 8.0))
    if axis is None:
        axis = float(np.clip(rng.beta(*prior["prior_axis"]), 0.15, 0.98))
    if profile is None:
        profile = float(np.clip(rng.beta(*prior["prior_profile"]), 0.02, 0.98))
    if angle is None:
        angle = float(rng.uniform(0, math.pi))
    return dict(star=bool(star), u=np.asarray(u, dtype=np.float64), flux=float(flux),
                colours=colours, fluxes=band_fluxes(flux, colours), radius=radius,
                axis=axis, profile=profile, angle=angle)


def init_theta(rng, src, pos_sigma=0.5):
    """Perturbed truth in the unconstrained parameter layout of include/celmi.h."""
    t = np.zeros(N_THETA)
    t[0:2] = src["u"] + rng.normal(0, pos_sigma, 2)
    t[2] = 0.0
    lr = math.log(src["flux"])
    t[3] = lr + rng.normal(0, 0.1)
    t[4] = lr + rng.normal(0, 0.1)
    t[5] = t[6] = math.log(0.05)
    t[7:11] = src["colours"] + rng.normal(0, 0.1, 4)
    t[11:15] = src["colours"] + rng.normal(0, 0.1, 4)
    t[15:23] = math.log(0.05)
    t[23] = src["angle"] + rng.normal(0, 0.1)
    t[24] = math.log(src["radius"]) + rng.normal(0, 0.05)
    t[25] = _logit(float(np.clip(src["profile"], 0.05, 0.95))) + rng.normal(0, 0.2)
    t[26] = _logit(float(np.clip(src["axis"], 0.05, 0.95))) + rng.normal(0, 0.2)
    return t


# ----------------------------------------------------------------------------------------
# assembly

def _assemble(name, images, sources, patch_rects, pixel_lists, prior, profiles, theta0, extra=None):
    """patch_rects: list of (src, img, x0, y0, w, h) sorted by (src, img); pixel_lists aligned."""
    N = len(images)
    sky_off, knots = [], []
    off = 0
    for img in images:
        k = sky_knots_for(img, img["qh"], img["qw"])
        sky_off.append(off)
        knots.append(k.ravel())
        off += k.size
    P = len(patch_rects)
    pr = np.array(patch_rects, dtype=np.int64).reshape(P, 6)
    sizes = pr[:, 4] * pr[:, 5]
    poff = np.zeros(P, dtype=np.int64)
    if P:
        poff[1:] = np.cumsum(sizes)[:-1]
    pixels = np.concatenate([p.ravel() for p in pixel_lists]).astype(np.float32) if P else np.zeros(0, np.float32)
    exp_a, exp_t, dev_a, dev_t = profiles
    truth = dict(star=np.array([s["star"] for s in sources]),
                 u=np.array([s["u"] for s in sources]).reshape(-1, 2),
                 flux=np.array([s["flux"] for s in sources]),
                 colours=np.array([s["colours"] for s in sources]).reshape(-1, 4),
                 radius=np.array([s["radius"] for s in sources]),
                 axis=np.array([s["axis"] for s in sources]),
                 profile=np.array([s["profile"] for s in sources]),
                 angle=np.array([s["angle"] for s in sources]))
    if extra:
        truth.update(extra)
    eig = coef = None
    if images and "eigen" in images[0]:
        eig = np.array([im["eigen"] for im in images], np.float64)
        coef = np.array([im["eigen_coef"] for im in images], np.float64)
    return Problem(
        n_sources=len(sources),
        img_band=np.array([im["band"] for im in images], np.int32),
        img_H=np.array([im["H"] for im in images], np.int32),
        img_W=np.array([im["W"] for im in images], np.int32),
        img_npsf=np.array([im["npsf"] for im in images], np.int32),
        img_psf=np.array([im["psf"] for im in images], np.float64).reshape(N, MAX_PSF, 6),
        img_A=np.array([im["A"] for im in images], np.float64).reshape(N, 2, 2),
        img_b=np.array([im["b"] for im in images], np.float64).reshape(N, 2),
        img_iota=np.array([im["iota"] for im in images], np.float64),
        img_sky_qh=np.array([im["qh"] for im in images], np.int32),
        img_sky_qw=np.array([im["qw"] for im in images], np.int32),
        img_sky_off=np.array(sky_off, np.int64),
        sky_knots=np.concatenate(knots).astype(np.float64),
        patch_src=pr[:, 0].astype(np.int32), patch_img=pr[:, 1].astype(np.int32),
        patch_x0=pr[:, 2].astype(np.int32), patch_y0=pr[:, 3].astype(np.int32),
        patch_w=pr[:, 4].astype(np.int32), patch_h=pr[:, 5].astype(np.int32),
        patch_off=poff, pixels=pixels,
        prior_a=prior["prior_a"], prior_r=prior["prior_r"], prior_cw=prior["prior_cw"],
        prior_cmean=prior["prior_cmean"], prior_ccov=prior["prior_ccov"],
        prior_radius=prior["prior_radius"], prior_profile=prior["prior_profile"],
        prior_axis=prior["prior_axis"],
        exp_alpha=exp_a, exp_tau=exp_t, dev_alpha=dev_a, dev_tau=dev_t,
        theta0=np.array(theta0, np.float64).reshape(len(sources), N_THETA),
        truth=truth, name=name, psf_eigen=eig, psf_coef=coef)


def _image(rng, band, H, W, sky0, A=None, b=None, sky_grad=0.0, qh=2, qw=2, npsf=3, iota=1.0, psf=None,
           sky_wave=0.0):
    im = dict(band=int(band), H=int(H), W=int(W), npsf=npsf, psf=make_psf(rng, npsf) if psf is None else psf,
              A=np.eye(2) if A is None else np.asarray(A, np.float64),
              b=np.zeros(2) if b is None else np.asarray(b, np.float64),
              iota=float(iota), sky0=float(sky0),
              sky_gy=float(rng.uniform(-sky_grad, sky_grad)),
              sky_gx=float(rng.uniform(-sky_grad, sky_grad)), qh=qh, qw=qw)
    if sky_wave:
        im.update(sky_wave=float(sky_wave), sky_ky=float(rng.uniform(0.7, 1.6)), sky_kx=float(rng.uniform(0.7, 1.6)),
                  sky_phase=rng.uniform(0, 1, 2))
    return im


def make_psf_skewed(rng, npsf):
    """A PSF mixture with off-centre components and correlated (tilted, elongated)
    covariances: sigma 1-2.5 px along each principal axis, means within 0.6 px."""
    w = rng.dirichlet(np.full(npsf, 2.0))
    psf = np.zeros((MAX_PSF, 6))
    for k in range(npsf):
        s1, s2 = rng.uniform(1.0, 2.5, 2)
        t = rng.uniform(0, math.pi)
        c, sn = math.cos(t), math.sin(t)
        cxx = s1 * s1 * c * c + s2 * s2 * sn * sn
        cyy = s1 * s1 * sn * sn + s2 * s2 * c * c
        cxy = (s1 * s1 - s2 * s2) * c * sn
        mx, my = rng.uniform(-0.6, 0.6, 2)
        psf[k] = [w[k], mx, my, cxx, cxy, cyy]
    return psf


def random_wcs(rng, scale=(0.85, 1.2), shear=0.15, angle=0.6):
    """An affine map sky -> pixels with rotation, shear and unequal axis scales (A != A^T,
    det > 0): A = R(phi) [[1, sh], [0, 1]] diag(sx, sy)."""
    phi = rng.uniform(-angle, angle)
    sh = rng.uniform(-shear, shear)
    sx, sy = rng.uniform(*scale, 2)
    R = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
    return R @ np.array([[1.0, sh], [0.0, 1.0]]) @ np.diag([sx, sy])


def _grouped(name, seed, n_sources, side_lo, side_hi, n_epochs, flux_mode, max_group=5,
             spacing=None, epoch_shift=0.5, prior_seed=None):
    """Sources in isolated groups of 1..max_group whose patches overlap pairwise.  The prior
    is drawn from `prior_seed` when given (one prior shared by every region of a survey),
    else from the problem's own stream."""
    rng = np.random.default_rng(seed)
    profiles = load_profiles()
    prior = make_prior(rng) if prior_seed is None else make_prior(np.random.default_rng(prior_seed))
    groups = []
    left = n_sources
    while left > 0:
        g = min(int(rng.integers(1, max_group + 1)), left)
        groups.append(g)
        left -= g
    spacing = spacing or (side_hi * 2 + 80)
    ncol = int(math.ceil(math.sqrt(len(groups))))
    nrow = int(math.ceil(len(groups) / ncol))
    H = nrow * spacing + 2 * spacing
    W = ncol * spacing + 2 * spacing
    images = []
    for e in range(n_epochs):
        shift = rng.uniform(-epoch_shift, epoch_shift, 2) if e > 0 else np.zeros(2)
        for band in range(N_BANDS):
            images.append(_image(rng, band, H, W, rng.uniform(50, 200), b=shift, sky_grad=0.01))
    sources, sides, gid = [], [], []
    for gi, g in enumerate(groups):
        cy = (gi // ncol + 1.5) * spacing
        cx = (gi % ncol + 1.5) * spacing
        for _ in range(g):
            u = np.array([cx, cy]) + rng.uniform(-0.25 * side_lo, 0.25 * side_lo, 2)
            star = rng.random() < prior["prior_a"]
            if flux_mode == "powerlaw":
                fmin, fmax = 1e3, 1e5
                q = rng.random()
                flux = fmin * (1 - q * (1 - (fmin / fmax) ** 1.5)) ** (-1 / 1.5)
            else:
                flux = None
            sources.append(draw_source(rng, prior, star, u, flux=flux))
            sides.append(int(rng.integers(side_lo, side_hi + 1)))
            gid.append(gi)
    theta0 = [init_theta(rng, s) for s in sources]
    rects = []
    for s, src in enumerate(sources):
        for n, img in enumerate(images):
            pos = img["A"] @ src["u"] + img["b"]
            side = sides[s]
            x0 = int(round(pos[0])) - side // 2
            y0 = int(round(pos[1])) - side // 2
            rects.append((s, n, x0, y0, side, side))
    # render each group's canvas per image and cut patches
    pix = [None] * len(rects)
    by_group = {}
    for k, (s, n, x0, y0, w, h) in enumerate(rects):
        by_group.setdefault((gid[s], n), []).append(k)
    for (g, n), ks in by_group.items():
        xs0 = min(rects[k][2] for k in ks)
        ys0 = min(rects[k][3] for k in ks)
        xs1 = max(rects[k][2] + rects[k][4] for k in ks)
        ys1 = max(rects[k][3] + rects[k][5] for k in ks)
        members = [sources[rects[k][0]] for k in ks]
        canvas = render(rng, images[n], (ys0, xs0, ys1 - ys0, xs1 - xs0), members, profiles)
        for k in ks:
            _, _, x0, y0, w, h = rects[k]
            pix[k] = canvas[y0 - ys0:y0 - ys0 + h, x0 - xs0:x0 - xs0 + w]
    return _assemble(name, images, sources, rects, pix, prior, profiles, theta0,
                     extra=dict(group=np.array(gid)))


def config1(seed=SEED_BASE + 1):
    rng = np.random.default_rng(seed)
    profiles = load_profiles()
    prior = make_prior(rng)
    images = [_image(rng, b, 32, 32, 100.0, qh=2, qw=2) for b in range(N_BANDS)]
    sources = []
    for star in (True, False):
        u = rng.uniform(10, 22, 2)
        flux = math.exp(rng.uniform(math.log(1e3), math.log(1e4)))
        sources.append(draw_source(rng, prior, star, u, flux=flux, radius=rng.uniform(1, 4),
                                   axis=rng.uniform(0.3, 1.0), angle=rng.uniform(0, math.pi),
                                   profile=rng.uniform(0, 1)))
    theta0 = [init_theta(rng, s) for s in sources]
    rects, pix = [], []
    canv = [render(rng, images[n], (0, 0, 32, 32), sources, profiles) for n in range(N_BANDS)]
    for s in range(2):
        for n in range(N_BANDS):
            rects.append((s, n, 0, 0, 32, 32))
            pix.append(canv[n])
    return _assemble("plain_1star_1gal_5x32x32", images, sources, rects, pix, prior, profiles, theta0)


def config2(seed=SEED_BASE + 2, n_sources=1000):
    return _grouped(f"batched_{n_sources}src_5bx2e_side20-60", seed, n_sources, 20, 60, 2, "powerlaw")


def config3(seed=SEED_BASE + 3, n_sources=4096):
    return _grouped(f"adjoint_{n_sources}src_5b_side16-64", seed, n_sources, 16, 64, 1, "prior")


def config5_request(seed, n_sources=None):
    rng = np.random.default_rng(seed)
    n = int(n_sources if n_sources is not None else rng.integers(1, 201))
    return _grouped(f"request_{n}src_5b_side16-96", seed + 7, n, 16, 96, 1, "prior", prior_seed=SURVEY_PRIOR_SEED)


def config_skew(seed=SEED_BASE + 6, n_groups=2, H=83, W=97, qh=4, qw=5):
    """A small blended field on which every image differs from the plain workloads in the
    ways they leave out: a WCS with rotation, shear and unequal scales and a sub-pixel
    offset, a calibration iota in [0.4, 3] per image, a sky knot grid of qh x qw (>= 3 x 3)
    sampling a field with curvature, PSF mixtures of 2-4 off-centre, tilted components;
    rectangular patches of unequal sides, some cut by the image edge.  Sources sit in
    overlapping groups of 2-3 (4 images: bands g and i, two epochs)."""
    rng = np.random.default_rng(seed)
    profiles = load_profiles()
    prior = make_prior(rng)
    images = []
    for e in range(2):
        for band in (1, 3):
            npsf = int(rng.integers(2, 5))
            images.append(_image(rng, band, H, W, rng.uniform(60, 150), A=random_wcs(rng),
                                 b=rng.uniform(-3, 3, 2), sky_grad=0.05, qh=qh, qw=qw, npsf=npsf,
                                 iota=rng.uniform(0.4, 3.0), psf=make_psf_skewed(rng, npsf), sky_wave=0.25))
    # sky positions whose pixel positions stay inside every frame
    sources = []
    centres = [np.array([W * 0.3, H * 0.35]), np.array([W * 0.68, H * 0.62])][:n_groups]
    for c in centres:
        for _ in range(int(rng.integers(2, 4))):
            u = c + rng.uniform(-5, 5, 2)
            sources.append(draw_source(rng, prior, rng.random() < 0.4, u, flux=rng.uniform(2e3, 2e4)))
    theta0 = [init_theta(rng, s_) for s_ in sources]
    rects = []
    for s_, src in enumerate(sources):
        for n, img in enumerate(images):
            pos = img["A"] @ src["u"] + img["b"]
            w = int(rng.integers(14, 31))
            h = int(rng.integers(14, 31))
            x0 = int(round(pos[0])) - w // 2 + int(rng.integers(-2, 3))
            y0 = int(round(pos[1])) - h // 2 + int(rng.integers(-2, 3))
            x1, y1 = min(W, x0 + w), min(H, y0 + h)
            x0, y0 = max(0, x0), max(0, y0)
            rects.append((s_, n, x0, y0, x1 - x0, y1 - y0))
    frames = [render(rng, images[n], (0, 0, H, W), sources, profiles) for n in range(len(images))]
    pix = [frames[n][y0:y0 + h, x0:x0 + w] for (s_, n, x0, y0, w, h) in rects]
    return _assemble(f"skew_{len(sources)}src_{H}x{W}_4img_sky{qh}x{qw}", images, sources, rects, pix,
                     prior, profiles, theta0)


def serving_field(seed=SEED_BASE + 5, n_sources=1500):
    """A survey field from which region requests are cut: sources in overlapping groups of
    1-5, patch sides 16-96, 5 bands, the survey's shared prior (the serving workload's
    shapes)."""
    return _grouped(f"serving_field_{n_sources}src_5b_side16-96", seed, n_sources, 16, 96, 1, "prior",
                    prior_seed=SURVEY_PRIOR_SEED)


def region_requests(field_prob, n, seed, max_sources=200):
    """n region requests cut from a field: each a run of whole groups starting at a random
    group, of U{1..max_sources} sources (shorter at the field's end); distinct requests are
    distinct regions, and each holds its sources' patches and pixels only."""
    rng = np.random.default_rng(seed)
    gid = field_prob.truth["group"]
    starts = np.concatenate([[0], np.nonzero(np.diff(gid))[0] + 1])
    out = []
    for _ in range(n):
        g0 = int(rng.integers(0, len(starts)))
        s0 = int(starts[g0])
        want = int(rng.integers(1, max_sources + 1))
        s1 = min(s0 + want, field_prob.n_sources)
        # end on a group boundary (at least one whole group)
        ends = starts[starts > s0]
        cut = ends[ends <= s1]
        s1 = int(cut[-1]) if len(cut) else (int(ends[0]) if len(ends) else field_prob.n_sources)
        out.append(subset(field_prob, sources=range(s0, s1), name=f"region_{s0}-{s1}"))
    return out


def _extent_halfwidth(src, psf_sigma_max):
    """A conservative source extent in pixels (stand-in for a detector's extent estimate):
    a few times the PSF width plus the galaxy half-light radius, growing slowly with flux."""
    size = psf_sigma_max * 2.0 + (0.0 if src["star"] else 2.5 * src["radius"])
    grow = 1.0 + 0.35 * max(0.0, math.log10(src["flux"] / 1e3))
    return int(np.clip(math.ceil(size * grow), 8, 48))


def _drifting_psf(rng, img):
    """Give an image a PSF that drifts over the frame and its eigen-PSF representation."""
    K = img["npsf"]
    img["psf_drift"] = np.column_stack([rng.uniform(-0.25, 0.25, K), rng.uniform(-0.25, 0.25, K),
                                        rng.uniform(-0.2, 0.2, K), rng.uniform(-0.3, 0.3, K),
                                        rng.uniform(-0.4, 0.4, K), rng.uniform(-0.4, 0.4, K)])
    img["eigen"], img["eigen_coef"] = eigen_psf(rng, img)


def config4(seed=SEED_BASE + 4, n_sources=600, H=2048, W=1489, n_epochs=3, bands=None, eigen=False, sky_q=None,
            name=None):
    """The field workload.  eigen: each image's PSF drifts over the frame and is given as
    E = 4 eigen-images with quadratic loadings (Section 2.2.2); sky_q = (qh, qw): a knot
    grid of that size sampling a sky field with curvature (Section 2.2.1; Table 1 gives
    Q = 192 x 256)."""
    rng = np.random.default_rng(seed)
    profiles = load_profiles()
    prior = make_prior(rng, star_prob=0.3)
    images = []
    for e in range(n_epochs):
        if e == 0:
            A, b = np.eye(2), np.zeros(2)
        else:
            ang = math.radians(rng.uniform(-0.3, 0.3))
            A = np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
            b = rng.uniform(-20, 20, 2)
        for band in (range(N_BANDS) if bands is None else bands):
            kw = {} if sky_q is None else dict(qh=sky_q[0], qw=sky_q[1], sky_wave=0.2)
            images.append(_image(rng, band, H, W, rng.uniform(50, 200), A=A, b=b, sky_grad=0.005, **kw))
            if eigen:
                _drifting_psf(rng, images[-1])
    margin = min(70, H // 4, W // 4)
    sources = []
    for _ in range(n_sources):
        u = np.array([rng.uniform(margin, W - margin), rng.uniform(margin, H - margin)])
        sources.append(draw_source(rng, prior, rng.random() < prior["prior_a"], u))
    theta0 = [init_theta(rng, s) for s in sources]
    psf_sig = [math.sqrt(max(im["psf"][k, 3] for k in range(im["npsf"]))) for im in images]
    rects = []
    for s, src in enumerate(sources):
        for n, img in enumerate(images):
            hw = _extent_halfwidth(src, psf_sig[n])
            pos = img["A"] @ src["u"] + img["b"]
            cx, cy = int(round(pos[0])), int(round(pos[1]))
            x0, x1 = max(0, cx - hw), min(W, cx + hw)
            y0, y1 = max(0, cy - hw), min(H, cy + hw)
            if x1 - x0 >= 4 and y1 - y0 >= 4:
                rects.append((s, n, x0, y0, x1 - x0, y1 - y0))
    frames = [render(rng, images[n], (0, 0, H, W), sources, profiles) for n in range(len(images))]
    pix = [frames[n][y0:y0 + h, x0:x0 + w] for (s, n, x0, y0, w, h) in rects]
    name = name or f"field_{n_sources}src_{H}x{W}_{len(images) // n_epochs}bx{n_epochs}e"
    return _assemble(name, images, sources, rects, pix, prior, profiles, theta0)


def config_eigen(seed=SEED_BASE + 7, n_sources=600, H=2048, W=1489):
    """The field workload with a spatially varying PSF given by eigen-images (E = 4 on
    51 x 51 knots, quadratic loadings) and a 192 x 256 sky knot grid (Table 1)."""
    return config4(seed=seed, n_sources=n_sources, H=H, W=W, eigen=True, sky_q=(192, 256),
                   name=f"field_eigenpsf_{n_sources}src_{H}x{W}_5bx3e_sky192x256")


def config_eigen_small(seed=SEED_BASE + 8):
    """A small field with a drifting PSF: 14 sources on 300 x 260 pixels, bands g and r over
    two epochs, a 24 x 32 sky knot grid."""
    return config4(seed=seed, n_sources=14, H=300, W=260, n_epochs=2, bands=(1, 2), eigen=True, sky_q=(24, 32),
                   name="field_eigenpsf_14src_300x260_2bx2e_sky24x32")


def truth_point(prob):
    """The true latent values of every source as a [S,16] float64 array of point values
    (position, type 1 = star, log reference-band flux, four colours, angle, log half-light
    radius, profile weight, axis ratio, then zeros): the layout of cel_loglik's z."""
    t = prob.truth
    z = np.zeros((prob.n_sources, 16))
    z[:, 0:2] = t["u"]
    z[:, 2] = t["star"].astype(np.float64)
    z[:, 3] = np.log(t["flux"])
    z[:, 4:8] = t["colours"]
    z[:, 8] = t["angle"]
    z[:, 9] = np.log(t["radius"])
    z[:, 10] = t["profile"]
    z[:, 11] = t["axis"]
    return z


def perturbed_points(z, n, seed):
    """n seeded perturbations [n,S,16] of point values z [S,16] (candidate states of a
    sampler): position +-0.4 px, log flux 0.2, colours 0.1, angle 0.3, log radius 0.2 (normal
    sd), profile weight uniform on [0, 1], axis ratio uniform on [0.2, 1], the type
    alternating over candidates and sources."""
    rng = np.random.default_rng(seed)
    S = z.shape[0]
    out = np.repeat(np.asarray(z, dtype=np.float64)[None], n, 0).copy()
    out[:, :, 0:2] += rng.normal(0, 0.4, (n, S, 2))
    out[:, :, 2] = (np.arange(n)[:, None] + np.arange(S)[None, :]) % 2
    out[:, :, 3] += rng.normal(0, 0.2, (n, S))
    out[:, :, 4:8] += rng.normal(0, 0.1, (n, S, 4))
    out[:, :, 8] += rng.normal(0, 0.3, (n, S))
    out[:, :, 9] += rng.normal(0, 0.2, (n, S))
    out[:, :, 10] = rng.uniform(0, 1, (n, S))
    out[:, :, 11] = rng.uniform(0.2, 1, (n, S))
    return out


def prior_draws(prob, z_fixed, n_runs, seed, box):
    """Start points of annealed importance sampling runs drawn from the prior of each source
    type (the generative model of Section 2.1, the runs' pi_0): [2, n_runs, S, 16] point
    values, index 0 galaxy, 1 star.  Position uniform on the square of half-width `box`
    around z_fixed's position, log flux normal, colours from the type's mixture, angle
    uniform on [0, pi), log radius normal, profile weight and axis ratio beta (drawn for
    stars too, where they are unused)."""
    rng = np.random.default_rng(seed)
    S = prob.n_sources
    out = np.zeros((2, n_runs, S, 16))
    for a in (0, 1):
        for r in range(n_runs):
            for s in range(S):
                z = out[a, r, s]
                z[0:2] = np.asarray(z_fixed[s, 0:2]) + rng.uniform(-box, box, 2)
                z[2] = float(a)
                z[3] = rng.normal(prob.prior_r[a, 0], math.sqrt(prob.prior_r[a, 1]))
                z[4:8] = draw_gmm(rng, prob.prior_cw[a], prob.prior_cmean[a], prob.prior_ccov[a])
                z[8] = rng.uniform(0, math.pi)
                z[9] = rng.normal(prob.prior_radius[0], math.sqrt(prob.prior_radius[1]))
                z[10] = rng.beta(*prob.prior_profile)
                z[11] = rng.beta(*prob.prior_axis)
    return out


def make_config(k, **kw):
    return {1: config1, 2: config2, 3: config3, 4: config4}[k](**kw)


def subset(prob, sources=None, images=None, name=None):
    """The problem restricted to some sources and images (ids renumbered in order).  Pure
    bookkeeping on the arrays; used to make small test problems and serving requests."""
    S, N = prob.n_sources, prob.n_images
    src = np.arange(S) if sources is None else np.asarray(sorted(sources), dtype=np.int64)
    img = np.arange(N) if images is None else np.asarray(sorted(images), dtype=np.int64)
    smap = np.full(S, -1)
    smap[src] = np.arange(len(src))
    imap = np.full(N, -1)
    imap[img] = np.arange(len(img))
    keep = (smap[prob.patch_src] >= 0) & (imap[prob.patch_img] >= 0)
    ps = np.nonzero(keep)[0]
    order = np.lexsort((imap[prob.patch_img[ps]], smap[prob.patch_src[ps]]))
    ps = ps[order]
    sizes = prob.patch_w[ps].astype(np.int64) * prob.patch_h[ps]
    poff = np.zeros(len(ps), np.int64)
    if len(ps):
        poff[1:] = np.cumsum(sizes)[:-1]
    pixels = np.concatenate([prob.pixels[prob.patch_off[p]:prob.patch_off[p] + sizes[k]]
                             for k, p in enumerate(ps)]) if len(ps) else np.zeros(0, np.float32)
    knots, koff, o = [], [], 0
    for n in img:
        q = int(prob.img_sky_qh[n] * prob.img_sky_qw[n])
        knots.append(prob.sky_knots[prob.img_sky_off[n]:prob.img_sky_off[n] + q])
        koff.append(o)
        o += q
    truth = {k: (v[src] if isinstance(v, np.ndarray) and v.shape[:1] == (S,) else v)
             for k, v in prob.truth.items()}
    return Problem(
        n_sources=len(src), img_band=prob.img_band[img], img_H=prob.img_H[img], img_W=prob.img_W[img],
        img_npsf=prob.img_npsf[img], img_psf=prob.img_psf[img], img_A=prob.img_A[img],
        img_b=prob.img_b[img], img_iota=prob.img_iota[img], img_sky_qh=prob.img_sky_qh[img],
        img_sky_qw=prob.img_sky_qw[img], img_sky_off=np.array(koff, np.int64),
        sky_knots=np.concatenate(knots) if knots else np.zeros(0),
        patch_src=smap[prob.patch_src[ps]].astype(np.int32), patch_img=imap[prob.patch_img[ps]].astype(np.int32),
        patch_x0=prob.patch_x0[ps], patch_y0=prob.patch_y0[ps], patch_w=prob.patch_w[ps],
        patch_h=prob.patch_h[ps], patch_off=poff, pixels=pixels.astype(np.float32),
        prior_a=prob.prior_a, prior_r=prob.prior_r, prior_cw=prob.prior_cw, prior_cmean=prob.prior_cmean,
        prior_ccov=prob.prior_ccov, prior_radius=prob.prior_radius, prior_profile=prob.prior_profile,
        prior_axis=prob.prior_axis, exp_alpha=prob.exp_alpha, exp_tau=prob.exp_tau,
        dev_alpha=prob.dev_alpha, dev_tau=prob.dev_tau, theta0=prob.theta0[src].copy(), truth=truth,
        name=name or (prob.name + "_subset"),
        psf_eigen=None if prob.psf_eigen is None else prob.psf_eigen[img],
        psf_coef=None if prob.psf_coef is None else prob.psf_coef[img])


def crop_patches(prob, max_side, name=None):
    """Shrink every patch to at most max_side x max_side around its centre (re-cut from the
    stored pixels), to make small test problems."""
    import copy
    out = copy.copy(prob)
    P = prob.n_patches
    x0, y0 = prob.patch_x0.copy(), prob.patch_y0.copy()
    w, h = prob.patch_w.copy(), prob.patch_h.copy()
    pix = []
    for p in range(P):
        img = prob.patch_pixels(p)
        nw, nh = min(int(w[p]), max_side), min(int(h[p]), max_side)
        dx, dy = (int(w[p]) - nw) // 2, (int(h[p]) - nh) // 2
        pix.append(img[dy:dy + nh, dx:dx + nw].ravel())
        x0[p] += dx
        y0[p] += dy
        w[p], h[p] = nw, nh
    sizes = w.astype(np.int64) * h
    poff = np.zeros(P, np.int64)
    if P:
        poff[1:] = np.cumsum(sizes)[:-1]
    out.patch_x0, out.patch_y0, out.patch_w, out.patch_h = x0, y0, w, h
    out.patch_off = poff
    out.pixels = np.concatenate(pix).astype(np.float32) if P else np.zeros(0, np.float32)
    out.name = name or (prob.name + f"_crop{max_side}")
    return out
