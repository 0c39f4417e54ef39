"""Reference variational objective, float64, plain PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): the product path never imports this.

Follows the paper's model and objective step by step:
  * variational family, Section 4.1 (equations eq:q_factorization, eq0-eq1)
  * ELBO = E_q log p(x|z) - KL(q||p), Section 4.2 (equation elbo)
  * E_q log p(x|z) as a sum of per-pixel Poisson terms (equation eq:log_p_last)
  * E_q[lambda] factorised on the source type (equation conditional)
  * E_q[log lambda] by the second-order delta method, and V_q[lambda] (equation vareq)
  * KL separated per source (equations eq:kl, kleq) with the GMM colour bound whose free
    weights take their closed-form optimum, and the Supplement A divergences
  * light kernels: stars are points, galaxies are rotated/scaled Gaussian scale mixtures
    (Section 2.1.2, equation hsi), convolved analytically with a Gaussian-mixture PSF
    (Section 2.2.3)

Readings of garbled or silent passages:
  colours c_b = ln(l_{b+1}/l_b) with r the reference band; log-normal and normal second
  parameters are variances; e_profile weights the de Vaucouleurs profile; Sigma_s taken
  literally as R^T diag(r^2, axis^2 r^2) R with R = [[cos,-sin],[sin,cos]]; angle in
  radians and radius in pixels; pixel response = mixture density at the pixel centre;
  sky = bilinear interpolation on a knot grid spanning the image corners; calibration is
  a scalar per image; point-mass KLs for direction and angle are constants (dropped);
  point-mass KLs for radius/profile/axis are minus the log prior density; the flux KL is
  the textbook normal KL on log r; each source's light is truncated to its patches.

Parameter layout per source (32 float64, unconstrained coordinates):
  0-1 u (reference pixel frame) | 2 logit(a) | 3,4 mean log r (galaxy, star) |
  5,6 log var log r | 7-10 colour means (galaxy) | 11-14 colour means (star) |
  15-18 log colour variances (galaxy) | 19-22 log colour variances (star) |
  23 angle | 24 log radius | 25 logit(profile) | 26 logit(axis) | 27-31 unused (zero)
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

DT = torch.float64
N_PARAM = 27
REF_BAND = 2
# log l_b = log r + W[b] . c   (c_k = ln(l_{k+1}/l_k), reference band r = index 2)
W_COLOUR = torch.tensor([[-1.0, -1.0, 0.0, 0.0],
                         [0.0, -1.0, 0.0, 0.0],
                         [0.0, 0.0, 0.0, 0.0],
                         [0.0, 0.0, 1.0, 0.0],
                         [0.0, 0.0, 1.0, 1.0]], dtype=DT)


class Model:
    """The problem's fixed inputs as float64 tensors plus patch-overlap bookkeeping.
    patch_psf: optional [P, 4, 6] PSF mixture of each patch (a spatially varying PSF, e.g.
    oracle.psf.patch_psfs); a source's light in an image then uses its patch's mixture."""

    def __init__(self, prob, patch_psf=None):
        self.prob = prob
        self.patch_psf = None if patch_psf is None else torch.as_tensor(np.asarray(patch_psf), dtype=DT)
        self.S = prob.n_sources
        t = lambda a: torch.as_tensor(np.asarray(a), dtype=DT)
        self.band = prob.img_band.astype(np.int64)
        self.H = prob.img_H.astype(np.int64)
        self.W = prob.img_W.astype(np.int64)
        self.npsf = prob.img_npsf.astype(np.int64)
        self.psf = t(prob.img_psf)
        self.A = t(prob.img_A)
        self.b = t(prob.img_b)
        self.iota = t(prob.img_iota)
        self.prior_a = float(prob.prior_a)
        self.prior_r = t(prob.prior_r)
        self.prior_cw = t(prob.prior_cw)
        self.prior_cmean = t(prob.prior_cmean)
        self.prior_ccov = t(prob.prior_ccov)
        self.prior_radius = t(prob.prior_radius)
        self.prior_profile = t(prob.prior_profile)
        self.prior_axis = t(prob.prior_axis)
        self.exp_alpha, self.exp_tau = t(prob.exp_alpha), t(prob.exp_tau)
        self.dev_alpha, self.dev_tau = t(prob.dev_alpha), t(prob.dev_tau)
        self.psrc = prob.patch_src.astype(np.int64)
        self.pimg = prob.patch_img.astype(np.int64)
        self.px0 = prob.patch_x0.astype(np.int64)
        self.py0 = prob.patch_y0.astype(np.int64)
        self.pw = prob.patch_w.astype(np.int64)
        self.ph = prob.patch_h.astype(np.int64)
        self.patches_of = [[] for _ in range(self.S)]
        self.patch_at = {}
        for p, s in enumerate(self.psrc):
            self.patches_of[s].append(p)
            self.patch_at[(int(s), int(self.pimg[p]))] = p
        # patches whose rectangles intersect, per patch (same image; includes itself)
        self.cover = [None] * len(self.psrc)
        for n in range(len(self.band)):
            ps = np.nonzero(self.pimg == n)[0]
            if len(ps) == 0:
                continue
            x0, y0 = self.px0[ps], self.py0[ps]
            x1, y1 = x0 + self.pw[ps], y0 + self.ph[ps]
            inter = ((x0[:, None] < x1[None, :]) & (x0[None, :] < x1[:, None]) &
                     (y0[:, None] < y1[None, :]) & (y0[None, :] < y1[:, None]))
            for a, p in enumerate(ps):
                self.cover[p] = ps[np.nonzero(inter[a])[0]]
        self._sky = {}
        self._x = {}

    def psf_for(self, s, n):
        """PSF mixture [K, 6] of source s in image n: its patch's where given, else the image's."""
        K = int(self.npsf[n])
        if self.patch_psf is not None and (int(s), int(n)) in self.patch_at:
            return self.patch_psf[self.patch_at[(int(s), int(n))], :K]
        return self.psf[n, :K]

    def pixels(self, p):
        if p not in self._x:
            self._x[p] = torch.as_tensor(self.prob.patch_pixels(p).astype(np.float64))
        return self._x[p]

    def sky(self, p):
        """Sky intensity on patch p: bilinear interpolation of the image's knot grid, the
        knots spanning the image corners (Section 2.2.1, 'interpolated linearly')."""
        if p in self._sky:
            return self._sky[p]
        n = self.pimg[p]
        qh, qw = int(self.prob.img_sky_qh[n]), int(self.prob.img_sky_qw[n])
        o = int(self.prob.img_sky_off[n])
        knots = np.asarray(self.prob.sky_knots[o:o + qh * qw], dtype=np.float64).reshape(qh, qw)
        rows = np.arange(self.py0[p], self.py0[p] + self.ph[p], dtype=np.float64)
        cols = np.arange(self.px0[p], self.px0[p] + self.pw[p], dtype=np.float64)

        def axis(coord, q, size):
            if q == 1:
                return np.zeros_like(coord, dtype=np.int64), np.zeros_like(coord)
            f = coord * (q - 1) / (size - 1)
            i = np.clip(np.floor(f).astype(np.int64), 0, q - 2)
            return i, f - i

        iy, ty = axis(rows, qh, self.H[n])
        ix, tx = axis(cols, qw, self.W[n])
        k = lambda di, dj: knots[np.minimum(iy + di, qh - 1)[:, None], np.minimum(ix + dj, qw - 1)[None, :]]
        val = ((1 - ty)[:, None] * (1 - tx)[None, :] * k(0, 0) + (1 - ty)[:, None] * tx[None, :] * k(0, 1)
               + ty[:, None] * (1 - tx)[None, :] * k(1, 0) + ty[:, None] * tx[None, :] * k(1, 1))
        self._sky[p] = torch.as_tensor(val)
        return self._sky[p]


# ----------------------------------------------------------------------------------------
# variational parameters

def natural(theta):
    """Map the unconstrained layout to the variational family's parameters (Section 4.1).
    theta: [S,32].  Returns a dict of tensors."""
    return dict(
        u=theta[:, 0:2],
        a=torch.sigmoid(theta[:, 2]),
        log_a=F.logsigmoid(theta[:, 2]),
        log_1ma=F.logsigmoid(-theta[:, 2]),
        r_mean=theta[:, 3:5],                    # [S,2] type 0 galaxy, 1 star
        r_var=torch.exp(theta[:, 5:7]),
        c_mean=theta[:, 7:15].reshape(-1, 2, 4),
        c_var=torch.exp(theta[:, 15:23]).reshape(-1, 2, 4),
        log_c_var=theta[:, 15:23].reshape(-1, 2, 4),
        log_r_var=theta[:, 5:7],
        angle=theta[:, 23],
        log_radius=theta[:, 24],
        radius=torch.exp(theta[:, 24]),
        profile=torch.sigmoid(theta[:, 25]),
        log_profile=F.logsigmoid(theta[:, 25]),
        log_1mprofile=F.logsigmoid(-theta[:, 25]),
        axis=torch.sigmoid(theta[:, 26]),
        log_axis=F.logsigmoid(theta[:, 26]),
        log_1maxis=F.logsigmoid(-theta[:, 26]),
    )


def band_flux_moments(nat, s, band, iota):
    """E[l_b | a=i] and E[l_b^2 | a=i] for i = 0 (galaxy), 1 (star), times the image's
    calibration.  Given a, log r and the colours are independent normals under q
    (Section 4.1), so log l_b = log r + W_b . c is normal with mean m and variance v, and
    E[l] = exp(m + v/2), E[l^2] = exp(2m + 2v) (Section 4.2.1, equation conditional)."""
    w = W_COLOUR[band]
    m = nat["r_mean"][s] + nat["c_mean"][s] @ w                 # [2]
    v = nat["r_var"][s] + nat["c_var"][s] @ (w * w)             # [2]
    L = iota * torch.exp(m + 0.5 * v)
    M = iota * iota * torch.exp(2.0 * m + 2.0 * v)
    return L, M


def galaxy_covariance(angle, radius, axis):
    """Sigma_s = R^T diag(radius^2, axis^2 radius^2) R, R = [[cos,-sin],[sin,cos]]
    (Section 2.1.2).  Returns (xx, xy, yy)."""
    R = torch.stack([torch.stack([torch.cos(angle), -torch.sin(angle)]),
                     torch.stack([torch.sin(angle), torch.cos(angle)])])
    D = torch.diag(torch.stack([radius * radius, axis * axis * radius * radius]))
    Sig = R.T @ D @ R
    return Sig[0, 0], Sig[0, 1], Sig[1, 1]


def normal_density(dx, dy, cxx, cxy, cyy):
    """Bivariate normal density with covariance [[cxx,cxy],[cxy,cyy]] at offsets (dx,dy).
    Broadcasts over leading component dimensions."""
    det = cxx * cyy - cxy * cxy
    q = (cyy * dx * dx - 2.0 * cxy * dx * dy + cxx * dy * dy) / det
    return torch.exp(-0.5 * q) / (2.0 * math.pi * torch.sqrt(det))


def source_profiles(model, nat, s, n, x0, y0, w, h):
    """f_{nms} for a star (f1) and for a galaxy (f0) on the rectangle of pixel centres
    cols x0..x0+w-1, rows y0..y0+h-1 of image n (Section 2.2.3: the PSF is a Gaussian
    mixture, so the galaxy integral is a Gaussian-Gaussian convolution, and the star's
    light is the PSF at the source's position)."""
    A, b = model.A[n], model.b[n]
    mu = A @ nat["u"][s] + b
    sxx, sxy, syy = galaxy_covariance(nat["angle"][s], nat["radius"][s], nat["axis"][s])
    Sig = torch.stack([torch.stack([sxx, sxy]), torch.stack([sxy, syy])])
    P = A @ Sig @ A.T                                          # galaxy covariance in pixels
    cols = torch.arange(x0, x0 + w, dtype=DT)
    rows = torch.arange(y0, y0 + h, dtype=DT)
    psf = model.psf_for(s, n)                                  # [K,6]
    pw, pmx, pmy = psf[:, 0], psf[:, 1], psf[:, 2]
    pcxx, pcxy, pcyy = psf[:, 3], psf[:, 4], psf[:, 5]
    dx = cols[None, None, :] - (mu[0] + pmx)[:, None, None]     # [K,1,w]
    dy = rows[None, :, None] - (mu[1] + pmy)[:, None, None]     # [K,h,1]
    f1 = (pw[:, None, None] * normal_density(dx, dy, pcxx[:, None, None], pcxy[:, None, None],
                                             pcyy[:, None, None])).sum(0)

    def profile(alpha, tau):
        # components indexed [J,K]: PSF covariance plus tau_j times the galaxy covariance
        cxx = pcxx[None, :] + tau[:, None] * P[0, 0]
        cxy = pcxy[None, :] + tau[:, None] * P[0, 1]
        cyy = pcyy[None, :] + tau[:, None] * P[1, 1]
        wt = alpha[:, None] * pw[None, :]
        dens = normal_density(dx[None], dy[None], cxx[..., None, None], cxy[..., None, None],
                              cyy[..., None, None])
        return (wt[..., None, None] * dens).sum((0, 1))

    prof = nat["profile"][s]
    f0 = prof * profile(model.dev_alpha, model.dev_tau) + (1.0 - prof) * profile(model.exp_alpha, model.exp_tau)
    return f0, f1


def source_rate_moments(model, nat, s, n, x0, y0, w, h):
    """E_q[l f] and V_q[l f] of source s on a rectangle of image n (equations conditional
    and vareq; u and e are point masses, so E[f^2 | a] = f^2)."""
    f0, f1 = source_profiles(model, nat, s, n, x0, y0, w, h)
    L, M = band_flux_moments(nat, s, int(model.band[n]), model.iota[n])
    a = nat["a"][s]
    E = (1.0 - a) * L[0] * f0 + a * L[1] * f1
    E2 = (1.0 - a) * M[0] * f0 * f0 + a * M[1] * f1 * f1
    return E, E2 - E * E


def pixel_terms(x, E, V):
    """-E[lambda] + x E[log lambda] - log x!, with E[log lambda] by the second-order delta
    method: log E[lambda] - V[lambda] / (2 E[lambda]^2) (equation eq:log_p_last, Section
    4.2.2)."""
    return -E + x * (torch.log(E) - V / (2.0 * E * E)) - torch.lgamma(x + 1.0)


def patch_rate(model, nat, p):
    """E_q[lambda] and V_q[lambda] on patch p: skyglow plus every source whose patch in the
    same image covers the pixel (Section 2.2.3, the rate as a sum over sources)."""
    n = model.pimg[p]
    x0, y0, w, h = model.px0[p], model.py0[p], model.pw[p], model.ph[p]
    E = model.sky(p).clone()
    V = torch.zeros_like(E)
    for q in model.cover[p]:
        t = model.psrc[q]
        ix0 = max(x0, model.px0[q]); ix1 = min(x0 + w, model.px0[q] + model.pw[q])
        iy0 = max(y0, model.py0[q]); iy1 = min(y0 + h, model.py0[q] + model.ph[q])
        Et, Vt = source_rate_moments(model, nat, t, n, ix0, iy0, ix1 - ix0, iy1 - iy0)
        pad = (int(ix0 - x0), int(x0 + w - ix1), int(iy0 - y0), int(y0 + h - iy1))
        E = E + F.pad(Et, pad)
        V = V + F.pad(Vt, pad)
    return E, V


def owned_mask(model, p):
    """Pixels of patch p not covered by a patch of a lower-numbered source in the same
    image, so that the union of patches counts every pixel once."""
    s = model.psrc[p]
    x0, y0, w, h = model.px0[p], model.py0[p], model.pw[p], model.ph[p]
    m = np.ones((h, w), dtype=bool)
    for q in model.cover[p]:
        if model.psrc[q] < s:
            ix0 = max(x0, model.px0[q]); ix1 = min(x0 + w, model.px0[q] + model.pw[q])
            iy0 = max(y0, model.py0[q]); iy1 = min(y0 + h, model.py0[q] + model.ph[q])
            m[iy0 - y0:iy1 - y0, ix0 - x0:ix1 - x0] = False
    return torch.as_tensor(m)


# ----------------------------------------------------------------------------------------
# KL divergence (equations eq:kl, kleq; Supplement A)

def kl_terms(model, nat):
    """Per-source KL(q(z_s) || p(z_s)) and its parts.  Returns dict of [S] tensors."""
    A = model.prior_a
    a = nat["a"]
    kl_a = a * (nat["log_a"] - math.log(A)) + (1 - a) * (nat["log_1ma"] - math.log(1 - A))
    # flux: normal KL on log r, both second parameters variances
    R1, R2 = model.prior_r[:, 0], model.prior_r[:, 1]                   # [2]
    kl_r = 0.5 * torch.log(R2[None, :] / nat["r_var"]) + \
        (nat["r_var"] + (nat["r_mean"] - R1[None, :]) ** 2) / (2 * R2[None, :]) - 0.5   # [S,2]
    # colours: GMM prior; KL to each component is a normal-normal KL; the free weights xi
    # of the bound take their optimum xi_j ~ w_j exp(-D_j), giving -log sum_j w_j exp(-D_j)
    prec = torch.linalg.inv(model.prior_ccov)                          # [2,J,4,4]
    logdet = torch.logdet(model.prior_ccov)                            # [2,J]
    cm, cv = nat["c_mean"], nat["c_var"]                               # [S,2,4]
    diff = model.prior_cmean[None] - cm[:, :, None, :]                 # [S,2,J,4]
    tr = torch.einsum("ijkk,sik->sij", prec, cv)
    maha = torch.einsum("sijk,ijkl,sijl->sij", diff, prec, diff)
    D = 0.5 * (tr + maha - 4.0 + logdet[None] - nat["log_c_var"].sum(-1)[:, :, None])
    kl_c = -torch.logsumexp(torch.log(model.prior_cw)[None] - D, dim=-1)   # [S,2]
    # point masses: minus the log prior density at the point
    E1, E2 = model.prior_radius[0], model.prior_radius[1]
    kl_radius = nat["log_radius"] + 0.5 * torch.log(2 * math.pi * E2) + (nat["log_radius"] - E1) ** 2 / (2 * E2)

    def neg_log_beta(logx, log1mx, ab):
        a_, b_ = ab[0], ab[1]
        lbeta = torch.lgamma(a_) + torch.lgamma(b_) - torch.lgamma(a_ + b_)
        return -(a_ - 1) * logx - (b_ - 1) * log1mx + lbeta

    kl_profile = neg_log_beta(nat["log_profile"], nat["log_1mprofile"], model.prior_profile)
    kl_axis = neg_log_beta(nat["log_axis"], nat["log_1maxis"], model.prior_axis)
    q = torch.stack([1 - a, a], dim=1)
    total = kl_a + kl_radius + kl_profile + kl_axis + (q * (kl_r + kl_c)).sum(1)
    return dict(total=total, a=kl_a, r=kl_r, c=kl_c, radius=kl_radius, profile=kl_profile, axis=kl_axis)


# ----------------------------------------------------------------------------------------
# objective

def elbo(model, theta, sources=None, with_total=True):
    """Returns (total, local): the global ELBO (every pixel of the union of patches once,
    minus every source's KL) and the per-source local objectives
    L_s = sum over the pixels of s's patches of the pixel term - KL_s (float64 [S]; sources
    not requested are left at 0).  Pinned by the tests in tests/test_oracle_*.py."""
    theta = torch.as_tensor(theta, dtype=DT)
    nat = natural(theta)
    kl = kl_terms(model, nat)["total"]
    S = model.S
    want = range(S) if sources is None else sources
    local = [torch.zeros((), dtype=DT)] * S
    total = torch.zeros((), dtype=DT)
    done = set()
    for s in want:
        acc = torch.zeros((), dtype=DT)
        for p in model.patches_of[s]:
            E, V = patch_rate(model, nat, p)
            T = pixel_terms(model.pixels(p), E, V)
            acc = acc + T.sum()
            if with_total:
                total = total + T[owned_mask(model, p)].sum()
        local[s] = acc - kl[s]
        done.add(s)
    if with_total:
        if sources is not None and len(done) != S:
            raise ValueError("the global ELBO needs every source")
        total = total - kl.sum()
    return total, torch.stack(local)


def elbo_total_and_grad(model, theta):
    """Global ELBO and its gradient [S,32] (reverse mode; padding entries are 0)."""
    th = torch.as_tensor(np.asarray(theta), dtype=DT).clone().requires_grad_(True)
    total, local = elbo(model, th)
    g, = torch.autograd.grad(total, th)
    return total.item(), local.detach().numpy(), g.numpy()


def local_objective(model, theta, s):
    """Function of theta_s[0:27] giving L_s with every other source fixed."""
    base = torch.as_tensor(np.asarray(theta), dtype=DT)

    def f(ts):
        th = torch.cat([base[:s], torch.cat([ts, base[s, N_PARAM:]])[None], base[s + 1:]], 0)
        return elbo(model, th, sources=[s], with_total=False)[1][s]
    return f


def local_value_grad(model, theta, s):
    """L_s and dL_s/dtheta_s (27 entries)."""
    f = local_objective(model, theta, s)
    ts = torch.as_tensor(np.asarray(theta)[s, :N_PARAM], dtype=DT).clone().requires_grad_(True)
    v = f(ts)
    g, = torch.autograd.grad(v, ts)
    return v.item(), g.numpy()


def local_hessian(model, theta, s):
    """d^2 L_s / dtheta_s^2 (27 x 27) by forward-over-reverse autodiff."""
    f = local_objective(model, theta, s)
    ts = torch.as_tensor(np.asarray(theta)[s, :N_PARAM], dtype=DT)
    return torch.autograd.functional.hessian(f, ts, vectorize=True).numpy()


def n_active_pixels(model, s):
    return int(sum(model.pw[p] * model.ph[p] for p in model.patches_of[s]))
