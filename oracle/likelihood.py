"""Reference Poisson log-likelihood at point values of the latent variables, float64, plain
PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): the product path never imports this.

The MCMC procedure (Section 3) samples one light source at a time with its overlapping
neighbours' latent variables held fixed (equation eqzs).  Its annealed importance sampler
(Section 3.1) and its slice-sampling transitions (Sections 3.1-3.2) evaluate the target
pi(w_s) = p(x | w_s, a_s, z_{-s}) p(w_s | a_s), whose likelihood factor is the Poisson
likelihood of the pixels given the latent variables (Section 2.2.3): x ~ Poisson(lambda),
lambda = sky + sum over sources of l f, with l the source's flux in the image's band and f
its light kernel there.  Only the pixels of source s's patches depend on z_s (each source's
light is truncated to its patches, as in the variational objective), so the conditional
log-likelihood is the sum over those pixels; the rest is a constant of z_s.

Point values per source z[s] (16 float64):
  0-1 u (reference pixel frame) | 2 type (1 star, 0 galaxy) | 3 log r (reference band) |
  4-7 colours c_k = ln(l_{k+1}/l_k) | 8 angle | 9 log half-light radius | 10 profile weight
  (de Vaucouleurs) | 11 axis ratio | 12-15 unused

The light kernels are the variational oracle's (oracle.elbo.source_profiles, pinned there);
pinned here by tests/test_oracle_likelihood.py: exact Poisson sums with scipy's pmf and
normal densities for stars and for isotropic galaxies (with the overlapping neighbour), the
zero-variance limit of the variational objective's pixel terms, and locality in z_{-s}; the
prior density by scipy's normal, multivariate normal and beta densities.
"""
from __future__ import annotations

import math

import torch

from oracle import elbo as E

DT = torch.float64
N_Z = 16


def _shape(z):
    """The light-kernel inputs of every source at its point value."""
    return dict(u=z[:, 0:2], angle=z[:, 8], radius=torch.exp(z[:, 9]), axis=z[:, 11], profile=z[:, 10])


def point_light(model, z, t, n, x0, y0, w, h):
    """l_t f_t of source t at its point value z[t] on a rectangle of image n: the flux in the
    image's band, log l_b = log r + W_b . c (colours as log flux ratios of adjacent bands),
    times the image's calibration, times the star or galaxy kernel (Section 2.2.3)."""
    f0, f1 = E.source_profiles(model, _shape(z), t, n, x0, y0, w, h)
    band = int(model.band[n])
    l = model.iota[n] * torch.exp(z[t, 3] + E.W_COLOUR[band] @ z[t, 4:8])
    return l * (f1 if float(z[t, 2]) != 0.0 else f0)


def patch_log_likelihood(model, z, p):
    """sum over the pixels of patch p of x log lambda - lambda - log x!, lambda = sky plus the
    light of every source whose patch in the same image covers the pixel, at z."""
    n = model.pimg[p]
    x0, y0, w, h = model.px0[p], model.py0[p], model.pw[p], model.ph[p]
    lam = model.sky(p).clone()
    for q in model.cover[p]:
        t = model.psrc[q]
        ix0 = max(x0, model.px0[q]); ix1 = min(x0 + w, model.px0[q] + model.pw[q])
        iy0 = max(y0, model.py0[q]); iy1 = min(y0 + h, model.py0[q] + model.ph[q])
        lt = point_light(model, z, t, n, ix0, iy0, ix1 - ix0, iy1 - iy0)
        lam[iy0 - y0:iy1 - y0, ix0 - x0:ix1 - x0] += lt
    x = model.pixels(p)
    return (x * torch.log(lam) - lam - torch.lgamma(x + 1.0)).sum()


def log_likelihood(model, z_fixed, s, z_s):
    """ll_s(z_s) = sum over source s's patches of their pixels' Poisson log-likelihood, with
    source s at z_s and every other source at z_fixed (Section 3, equation eqzs)."""
    z = torch.as_tensor(z_fixed, dtype=DT).clone()
    z[s] = torch.as_tensor(z_s, dtype=DT)
    return sum(patch_log_likelihood(model, z, p) for p in model.patches_of[s]).item()


def point_of_theta(theta, star):
    """Point values z [S,16] at the variational means of theta [S,32] (layout of
    oracle.elbo): position, the given type per source, the type's mean log flux and
    colours, and the shape."""
    th = torch.as_tensor(theta, dtype=DT)
    S = th.shape[0]
    z = torch.zeros((S, N_Z), dtype=DT)
    st = torch.as_tensor(star, dtype=torch.bool).reshape(S)
    z[:, 0:2] = th[:, 0:2]
    z[:, 2] = st.to(DT)
    # type index 0 = galaxy, 1 = star in theta's flux and colour blocks
    z[:, 3] = torch.where(st, th[:, 4], th[:, 3])
    z[:, 4:8] = torch.where(st[:, None], th[:, 11:15], th[:, 7:11])
    z[:, 8] = th[:, 23]
    z[:, 9] = th[:, 24]
    z[:, 10] = torch.sigmoid(th[:, 25])
    z[:, 11] = torch.sigmoid(th[:, 26])
    return z


def log_prior(model, z_s):
    """log p(w_s | a_s) at a point (the AIS start distribution pi_0 of Section 3.1), over the
    coordinates of the point layout: the model's priors (Section 2.1) -- log r normal given
    the type (the flux is log-normal), colours from the type's Gaussian mixture, and for a
    galaxy log radius normal (log-normal radius), profile weight and axis ratio beta, angle
    uniform on [0, pi) radians; the position's uniform prior is a constant and left out.
    -inf outside the support (profile weight not in [0, 1], axis ratio not in (0, 1])."""
    z = torch.as_tensor(z_s, dtype=DT)
    prof, axis = float(z[10]), float(z[11])
    if not (0.0 <= prof <= 1.0 and 0.0 < axis <= 1.0 and bool(torch.isfinite(z[:12]).all())):
        return -math.inf
    i = 1 if float(z[2]) != 0.0 else 0

    def normal(x, mean, var):
        return -0.5 * math.log(2 * math.pi * var) - (x - mean) ** 2 / (2 * var)

    lp = normal(z[3], model.prior_r[i, 0], model.prior_r[i, 1])
    c = z[4:8]
    terms = []
    for j in range(model.prior_cw.shape[1]):
        w = model.prior_cw[i, j]
        if w <= 0:
            continue
        cov = model.prior_ccov[i, j]
        d = c - model.prior_cmean[i, j]
        maha = d @ torch.linalg.solve(cov, d)
        terms.append(torch.log(w) - 2.0 * math.log(2 * math.pi) - 0.5 * torch.logdet(cov) - 0.5 * maha)
    lp = lp + torch.logsumexp(torch.stack(terms), 0)
    if i == 0:
        def beta(x, ab):
            a, b = ab[0], ab[1]
            lb = torch.lgamma(a) + torch.lgamma(b) - torch.lgamma(a + b)
            return (a - 1) * torch.log(x) + (b - 1) * torch.log1p(-x) - lb

        lp = lp + normal(z[9], model.prior_radius[0], model.prior_radius[1])
        lp = lp + beta(z[10], model.prior_profile) + beta(z[11], model.prior_axis) - math.log(math.pi)
    return float(lp)
