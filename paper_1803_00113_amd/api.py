"""Python binding of the celmi library: argument marshalling around the C ABI.

Every computation runs in the HIP kernels of libcelmi.so; this module only builds the
host tables of a problem, moves arrays to the device with torch and passes pointers.

A problem is any object with the array attributes of include/celmi.h's cel_problem in
numpy form (img_band, img_H, img_W, img_npsf, img_psf, img_A, img_b, img_iota, img_sky_qh,
img_sky_qw, img_sky_off, sky_knots, patch_src, patch_img, patch_x0, patch_y0, patch_w,
patch_h, patch_off, pixels, prior_a, prior_r, prior_cw, prior_cmean, prior_ccov,
prior_radius, prior_profile, prior_axis, exp_alpha, exp_tau, dev_alpha, dev_tau,
n_sources).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _ffi as F


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Context:
    """A library context on one HIP device (cel_create)."""

    def __init__(self, device=0, pixels_per_lane=0, chunk_pixels=0, pixel_fp64=False, hessian_fp64=False,
                 hessian_fd=False, fd_step=0.0, timing=False, map_pixels_per_lane=0, **tr):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the celmi library needs an MI355X (gfx950)")
        o = F.CelOptions()
        o.pixels_per_lane = int(pixels_per_lane)
        o.chunk_pixels = int(chunk_pixels)
        o.pixel_fp64 = int(bool(pixel_fp64))
        o.hessian_fp64 = int(bool(hessian_fp64))
        o.hessian_fd = int(bool(hessian_fd))
        o.fd_step = float(fd_step)
        o.timing = int(bool(timing))
        o.map_pixels_per_lane = int(map_pixels_per_lane)
        for k in ("radius0", "radius_max", "eta", "gtol", "ftol", "radius_min"):
            setattr(o, k, float(tr.get(k, 0.0)))
        h = C.c_void_p()
        F.check("cel_create", F.lib.cel_create(C.byref(h), int(device), C.byref(o)))
        self.h = h
        self._lib = F.lib          # kept for close() during interpreter shutdown
        self.device = torch.device("cuda", int(device))
        self.options = o

    def close(self):
        lib = getattr(self, "_lib", None)
        if getattr(self, "h", None) and lib is not None:
            lib.cel_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()


def host_tables(prob):
    """cel_image / cel_patch arrays and prior / profile structs of a problem."""
    N = int(len(prob.img_band))
    P = int(len(prob.patch_src))
    # cel_image records filled column by column (numpy mirrors the C struct's layout)
    images = np.zeros(max(N, 1), dtype=np.dtype(F.CelImage))
    if N:
        im = images[:N]
        im["band"], im["H"], im["W"] = prob.img_band, prob.img_H, prob.img_W
        im["n_psf"] = prob.img_npsf
        psf = np.asarray(prob.img_psf, dtype=np.float64)
        im["psf"][:, :psf.shape[1], :] = psf[:, :F.MAX_PSF, :]
        im["A"], im["b"], im["iota"] = prob.img_A, prob.img_b, prob.img_iota
        im["sky_qh"], im["sky_qw"], im["sky_off"] = prob.img_sky_qh, prob.img_sky_qw, prob.img_sky_off
    patches = np.zeros(max(P, 1), dtype=np.dtype([("src", "<i4"), ("img", "<i4"), ("x0", "<i4"), ("y0", "<i4"),
                                                   ("w", "<i4"), ("h", "<i4"), ("pix_off", "<i8")]))
    patches = patches[:P] if P else patches[:0]
    patches["src"], patches["img"] = prob.patch_src, prob.patch_img
    patches["x0"], patches["y0"] = prob.patch_x0, prob.patch_y0
    patches["w"], patches["h"] = prob.patch_w, prob.patch_h
    patches["pix_off"] = prob.patch_off
    patches = np.ascontiguousarray(patches)
    pr = F.CelPrior()
    pr.star_prob = float(prob.prior_a)
    J = prob.prior_cw.shape[1]
    if J > F.N_COLOUR_COMPONENTS:
        raise ValueError("at most 8 colour prior components")
    for i in range(2):
        pr.r[i][0], pr.r[i][1] = float(prob.prior_r[i, 0]), float(prob.prior_r[i, 1])
        for j in range(F.N_COLOUR_COMPONENTS):
            if j < J:
                pr.c_w[i][j] = float(prob.prior_cw[i, j])
                for k in range(4):
                    pr.c_mean[i][j][k] = float(prob.prior_cmean[i, j, k])
                    for l in range(4):
                        pr.c_cov[i][j][k][l] = float(prob.prior_ccov[i, j, k, l])
            else:
                pr.c_w[i][j] = 0.0
                for k in range(4):
                    pr.c_cov[i][j][k][k] = 1.0
    pr.radius[0], pr.radius[1] = float(prob.prior_radius[0]), float(prob.prior_radius[1])
    pr.profile[0], pr.profile[1] = float(prob.prior_profile[0]), float(prob.prior_profile[1])
    pr.axis[0], pr.axis[1] = float(prob.prior_axis[0]), float(prob.prior_axis[1])
    pf = F.CelProfiles()
    pf.n_exp, pf.n_dev = len(prob.exp_alpha), len(prob.dev_alpha)
    if pf.n_exp > F.MAX_PROFILE or pf.n_dev > F.MAX_PROFILE:
        raise ValueError("at most 8 components per profile")
    for j in range(pf.n_exp):
        pf.exp_alpha[j], pf.exp_tau[j] = float(prob.exp_alpha[j]), float(prob.exp_tau[j])
    for j in range(pf.n_dev):
        pf.dev_alpha[j], pf.dev_tau[j] = float(prob.dev_alpha[j]), float(prob.dev_tau[j])
    knots = np.ascontiguousarray(prob.sky_knots, dtype=np.float64)
    return images, knots, patches, pr, pf


def _problem_struct(ctx, prob, pixels_device):
    """The cel_problem of a problem (host tables by value, pixels on the device); returns it
    with the objects that keep its memory alive."""
    dev = ctx.device
    images, knots, patches, prior, profiles = host_tables(prob)
    if pixels_device is not None:
        if not (pixels_device.is_cuda and pixels_device.dtype == torch.float32 and pixels_device.is_contiguous()):
            raise ValueError("pixels_device must be a contiguous cuda float32 tensor")
        pixels = pixels_device
    else:
        pixels = torch.as_tensor(np.ascontiguousarray(prob.pixels, dtype=np.float32)).to(dev)
    cp = F.CelProblem()
    cp.n_sources = int(prob.n_sources)
    cp.n_images = int(len(prob.img_band))
    cp.n_patches = int(len(prob.patch_src))
    cp.images = images.ctypes.data_as(C.POINTER(F.CelImage))
    cp.sky_knots = knots.ctypes.data_as(C.POINTER(C.c_double))
    cp.n_sky_knots = int(knots.size)
    cp.patches = patches.ctypes.data_as(C.POINTER(F.CelPatch))
    cp.pixels = C.c_void_p(pixels.data_ptr())
    cp.n_pixels = int(pixels.numel())
    cp.prior = C.pointer(prior)
    cp.profiles = C.pointer(profiles)
    ppsf = getattr(prob, "patch_psf", None)
    if ppsf is not None:
        ppsf = np.ascontiguousarray(ppsf, dtype=np.float64)
        if ppsf.shape != (cp.n_patches, F.MAX_PSF, 6):
            raise ValueError(f"patch_psf must be [{cp.n_patches}, {F.MAX_PSF}, 6]")
        cp.patch_psf = ppsf.ctypes.data_as(C.POINTER(C.c_double))
    return cp, (images, knots, patches, prior, profiles, pixels, ppsf)


class Plan:
    """A prepared problem (cel_prepare).  Pixels are read once, during construction."""

    def __init__(self, ctx: Context, prob, stream=None, pixels_device=None):
        """pixels_device: optional float32 cuda tensor holding the packed pixels (else
        prob.pixels is copied to the device)."""
        self.ctx = ctx
        dev = ctx.device
        cp, keep = _problem_struct(ctx, prob, pixels_device)
        h = C.c_void_p()
        with torch.cuda.device(dev):
            st = stream if stream is not None else _stream(dev)
            F.check("cel_prepare", F.lib.cel_prepare(ctx.h, C.byref(cp), C.byref(h), st))
        self.h = h
        self._lib = F.lib
        self.S = int(prob.n_sources)
        self._refresh()

    def append(self, prob, pixels_device=None):
        """cel_plan_append: add a problem's sources, images and patches after the plan's
        own (ids offset).  Returns the id of the part's first source."""
        first = self.S
        cp, keep = _problem_struct(self.ctx, prob, pixels_device)
        with torch.cuda.device(self.ctx.device):
            F.check("cel_plan_append", F.lib.cel_plan_append(self.ctx.h, self.h, C.byref(cp), _stream(self.ctx.device)))
        self.S += int(prob.n_sources)
        self._refresh()
        return first

    def _refresh(self):
        nu, nc, nw = C.c_int64(), C.c_int32(), C.c_int64()
        col = np.zeros(max(self.S, 1), dtype=np.int32)
        F.check("cel_plan_info", F.lib.cel_plan_info(self.h, C.byref(nu), C.byref(nc),
                                                     col.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nw), None))
        self.n_units = int(nu.value)
        self.n_colours = int(nc.value)
        self.n_work_items = int(nw.value)
        self.colours = col[:self.S].copy()

    def device_bytes(self):
        """Device bytes the plan holds now (cel_plan_info)."""
        b = C.c_int64()
        F.check("cel_plan_info", F.lib.cel_plan_info(self.h, None, None, None, None, C.byref(b)))
        return int(b.value)

    def close(self):
        lib = getattr(self, "_lib", None)
        if getattr(self, "h", None) and lib is not None:
            lib.cel_plan_free(self.h)
        self.h = None

    def __del__(self):
        self.close()

    # -- helpers ---------------------------------------------------------------------------
    def _theta(self, theta):
        t = torch.as_tensor(theta, dtype=torch.float64, device=self.ctx.device)
        if t.shape != (self.S, F.N_THETA):
            raise ValueError(f"theta must be [{self.S}, {F.N_THETA}]")
        return t.contiguous()

    def phase_times(self, reset=True):
        """cel_phase_times: (ms[tables, maps, pixels, finalise], n_evaluations) since the last reset."""
        ms = (C.c_double * 4)()
        n = C.c_int64()
        F.check("cel_phase_times", F.lib.cel_phase_times(self.h, ms, C.byref(n), int(bool(reset))))
        return list(ms), int(n.value)

    def tune(self, theta, chunk_pixels=None, pixels_per_lane=None, map_pixels_per_lane=None):
        """cel_tune: times the gradient evaluation at theta over work-item sizes, pixel-pass
        pixels per lane and moment-map variants (each argument a list of candidates; None:
        the library's defaults; []: keep the plan's value), keeps the fastest settings for
        this plan and returns them as a dict."""
        th = self._theta(theta)
        space = None
        if not (chunk_pixels is None and pixels_per_lane is None and map_pixels_per_lane is None):
            space = F.CelTuneSpace()
            for name, vals, dflt in (("chunk", chunk_pixels, [256, 512, 1024, 2048]),
                                     ("pixels_per_lane", pixels_per_lane, [1, 2, 4]),
                                     ("map", map_pixels_per_lane, [1, 2, 4, 8, -1])):
                vals = dflt if vals is None else list(vals)
                arr = getattr(space, "chunk_pixels" if name == "chunk" else
                              "map_pixels_per_lane" if name == "map" else "pixels_per_lane")
                if len(vals) > len(arr):
                    raise ValueError(f"at most {len(arr)} candidates for {name}")
                for i, v in enumerate(vals):
                    arr[i] = int(v)
                setattr(space, "n_" + name, len(vals))
        out = F.CelTuning()
        F.check("cel_tune", F.lib.cel_tune(self.ctx.h, self.h, _ptr(th), C.byref(space) if space is not None else None,
                                           C.byref(out), _stream(self.ctx.device)))
        self._refresh()
        return dict(chunk_pixels=out.chunk_pixels, pixels_per_lane=out.pixels_per_lane,
                    map_pixels_per_lane=out.map_pixels_per_lane, n_timed=out.n_timed, ms_per_eval=out.ms_per_eval)

    def _out(self, *shape):
        return torch.empty(shape, dtype=torch.float64, device=self.ctx.device)


def elbo_eval(plan: Plan, theta):
    """cel_elbo_eval: returns (elbo_total [1], elbo_local [S]) device tensors."""
    th = plan._theta(theta)
    tot, loc = plan._out(1), plan._out(plan.S)
    F.check("cel_elbo_eval", F.lib.cel_elbo_eval(plan.ctx.h, plan.h, _ptr(th), _ptr(tot), _ptr(loc),
                                                 _stream(plan.ctx.device)))
    return tot, loc


def elbo_grad(plan: Plan, theta):
    """cel_elbo_grad: returns (elbo_total [1], elbo_local [S], grad [S,32]) device tensors."""
    th = plan._theta(theta)
    tot, loc, g = plan._out(1), plan._out(plan.S), plan._out(plan.S, F.N_THETA)
    F.check("cel_elbo_grad", F.lib.cel_elbo_grad(plan.ctx.h, plan.h, _ptr(th), _ptr(tot), _ptr(loc), _ptr(g),
                                                 _stream(plan.ctx.device)))
    return tot, loc, g


def elbo_grad_static(plan: Plan, theta, out=None):
    """cel_elbo_grad_static: cel_elbo_grad with its scratch in the library's static device
    buffer (no allocation inside the call).  out: optional (total [1], local [S], grad
    [S,32]) float64 cuda tensors to write into (else they are allocated here, by torch,
    before the call).  Returns (total, local, grad)."""
    th = plan._theta(theta)
    tot, loc, g = out if out is not None else (plan._out(1), plan._out(plan.S), plan._out(plan.S, F.N_THETA))
    F.check("cel_elbo_grad_static", F.lib.cel_elbo_grad_static(plan.ctx.h, plan.h, _ptr(th), _ptr(tot), _ptr(loc),
                                                               _ptr(g), _stream(plan.ctx.device)))
    return tot, loc, g


def elbo_grad_plain(plan: Plan, theta):
    """cel_elbo_grad_plain: one launch per source; same outputs as elbo_grad."""
    th = plan._theta(theta)
    tot, loc, g = plan._out(1), plan._out(plan.S), plan._out(plan.S, F.N_THETA)
    F.check("cel_elbo_grad_plain", F.lib.cel_elbo_grad_plain(plan.ctx.h, plan.h, _ptr(th), _ptr(tot), _ptr(loc),
                                                             _ptr(g), _stream(plan.ctx.device)))
    return tot, loc, g


def _mask(plan, mask):
    if mask is None:
        return None, None
    mk = np.ascontiguousarray(np.asarray(mask).astype(np.uint8))
    if mk.shape != (plan.S,):
        raise ValueError("mask must have one entry per source")
    return mk, mk.ctypes.data_as(C.POINTER(C.c_uint8))


def elbo_hessian(plan: Plan, theta, mask=None):
    """cel_elbo_hessian: returns (hess [S,27,27], grad [S,32], elbo_local [S]) device tensors
    (rows of unmasked sources are zero)."""
    th = plan._theta(theta)
    h = torch.zeros((plan.S, F.N_PARAM, F.N_PARAM), dtype=torch.float64, device=plan.ctx.device)
    g, loc = plan._out(plan.S, F.N_THETA), plan._out(plan.S)
    keep, m = _mask(plan, mask)
    F.check("cel_elbo_hessian", F.lib.cel_elbo_hessian(plan.ctx.h, plan.h, _ptr(th), m, _ptr(h), _ptr(g), _ptr(loc),
                                                       _stream(plan.ctx.device)))
    return h, g, loc


def newton_step(plan: Plan, theta, radius, mask=None):
    """cel_newton_step: theta [S,32] and radius [S] device float64 tensors updated in place.
    mask: host bool/uint8 array [S] or None.  Returns (status [S] int32, elbo_local [S])."""
    if not (isinstance(theta, torch.Tensor) and theta.is_cuda and theta.dtype == torch.float64
            and theta.is_contiguous() and theta.shape == (plan.S, F.N_THETA)):
        raise ValueError("theta must be a contiguous cuda float64 tensor [S,32]")
    if not (isinstance(radius, torch.Tensor) and radius.is_cuda and radius.dtype == torch.float64
            and radius.shape == (plan.S,)):
        raise ValueError("radius must be a cuda float64 tensor [S]")
    st = torch.empty(plan.S, dtype=torch.int32, device=plan.ctx.device)
    loc = plan._out(plan.S)
    m = None
    if mask is not None:
        mk = np.ascontiguousarray(np.asarray(mask).astype(np.uint8))
        if mk.shape != (plan.S,):
            raise ValueError("mask must have one entry per source")
        m = mk.ctypes.data_as(C.POINTER(C.c_uint8))
    F.check("cel_newton_step", F.lib.cel_newton_step(plan.ctx.h, plan.h, _ptr(theta), _ptr(radius), m, _ptr(st),
                                                     _ptr(loc), _stream(plan.ctx.device)))
    return st, loc


def loglik(plan: Plan, z_fixed, z_cand, mask=None):
    """cel_loglik: exact Poisson log-likelihood of each candidate point of each selected
    source, the others at z_fixed.  z_fixed [S,16] and z_cand [C,S,16] device float64 tensors
    (layout in include/celmi.h); mask: host bool/uint8 array [S] or None.  Returns ll [C,S]
    (rows of unselected sources NaN)."""
    for t, shape in ((z_fixed, (plan.S, F.N_Z)), (z_cand, None)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("z_fixed / z_cand must be contiguous cuda float64 tensors")
        if shape is not None and tuple(t.shape) != shape:
            raise ValueError("z_fixed must be [S,16]")
    if z_cand.dim() != 3 or tuple(z_cand.shape[1:]) != (plan.S, F.N_Z):
        raise ValueError("z_cand must be [C,S,16]")
    n = int(z_cand.shape[0])
    ll = torch.full((n, plan.S), float("nan"), dtype=torch.float64, device=plan.ctx.device)
    keep, m = _mask(plan, mask)
    F.check("cel_loglik", F.lib.cel_loglik(plan.ctx.h, plan.h, _ptr(z_fixed), n, _ptr(z_cand), m, _ptr(ll),
                                           _stream(plan.ctx.device)))
    return ll


def mcmc_step(plan: Plan, z_fixed, z_init, opts, key, mask=None, want_samples=False):
    """cel_mcmc_step: one MCMC update of the selected sources (annealed importance sampling
    with slice-sampling-within-Gibbs transitions, then further chains and the type draw).
    z_fixed [S,16] and z_init [2,N',S,16] cuda float64 tensors; opts: dict with n_temps,
    n_runs, n_post, max_step_out, max_shrink, gamma (host sequence of n_temps + 1), width
    (16 per-coordinate slice widths), box, seed; key: the generator key's second word.
    Returns dict(z [S,16], p_star [S], log_evidence [S,2], samples [S,2,N',B',16] or None,
    rhat [S,2,16] (the chains' potential scale reduction; NaN rows for unselected sources),
    report)."""
    for t in (z_fixed, z_init):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("z_fixed / z_init must be contiguous cuda float64 tensors")
    Np, Bp, T = int(opts["n_runs"]), int(opts["n_post"]), int(opts["n_temps"])
    if tuple(z_fixed.shape) != (plan.S, F.N_Z) or tuple(z_init.shape) != (2, Np, plan.S, F.N_Z):
        raise ValueError("z_fixed must be [S,16] and z_init [2,n_runs,S,16]")
    gam = np.ascontiguousarray(np.asarray(opts["gamma"], dtype=np.float64))
    if gam.shape != (T + 1,):
        raise ValueError("gamma must hold n_temps + 1 temperatures")
    o = F.CelMcmcOpts()
    o.n_temps, o.n_runs, o.n_post = T, Np, Bp
    o.max_step_out, o.max_shrink = int(opts["max_step_out"]), int(opts["max_shrink"])
    o.gamma = gam.ctypes.data_as(C.POINTER(C.c_double))
    for k in range(F.N_Z):
        o.width[k] = float(opts["width"][k]) if k < len(opts["width"]) else 0.0
    o.box, o.seed = float(opts["box"]), int(opts["seed"])
    dev = plan.ctx.device
    z_out = z_fixed.clone()
    p_star = torch.full((plan.S,), float("nan"), dtype=torch.float64, device=dev)
    log_ev = torch.full((plan.S, 2), float("nan"), dtype=torch.float64, device=dev)
    smp = torch.zeros((plan.S, 2, Np, Bp, F.N_Z), dtype=torch.float64, device=dev) if want_samples else None
    rhat = torch.full((plan.S, 2, F.N_Z), float("nan"), dtype=torch.float64, device=dev)
    rep = F.CelMcmcReport()
    keep, m = _mask(plan, mask)
    F.check("cel_mcmc_step", F.lib.cel_mcmc_step(plan.ctx.h, plan.h, _ptr(z_fixed), m, _ptr(z_init), C.byref(o),
                                                 int(key), _ptr(z_out), _ptr(p_star), _ptr(log_ev), _ptr(smp),
                                                 _ptr(rhat), C.byref(rep), _stream(dev)))
    return dict(z=z_out, p_star=p_star, log_evidence=log_ev, samples=smp, rhat=rhat,
                report=dict(rounds=rep.rounds, n_chains=rep.n_chains, evaluations=rep.evaluations,
                            candidate_pixels=rep.candidate_pixels))


def log_prior(plan: Plan, z):
    """cel_log_prior: log p(w | a) of point values z [..., 16] (contiguous cuda float64);
    returns a tensor of z's leading shape."""
    if not (isinstance(z, torch.Tensor) and z.is_cuda and z.dtype == torch.float64 and z.is_contiguous()
            and z.shape[-1] == F.N_Z):
        raise ValueError("z must be a contiguous cuda float64 tensor [..., 16]")
    out = torch.empty(z.shape[:-1], dtype=torch.float64, device=plan.ctx.device)
    F.check("cel_log_prior", F.lib.cel_log_prior(plan.ctx.h, plan.h, int(out.numel()), _ptr(z), _ptr(out),
                                                 _stream(plan.ctx.device)))
    return out


def sweep(plan: Plan, theta, n_sweeps=3, max_newton_iters=50, use_graph=True, radius=None, status=None,
          start_colour=0, max_classes=0):
    """cel_sweep: theta updated in place.  Returns (radius, status, report dict).

    Checkpoint / resume: with max_classes = k the call stops after k colour classes;
    report["next_colour"] and report["sweeps_done"] are the cursor.  Pass the returned
    radius and status back with start_colour = next_colour and the passes still due to
    continue exactly as one uninterrupted call."""
    if not (isinstance(theta, torch.Tensor) and theta.is_cuda and theta.dtype == torch.float64
            and theta.is_contiguous() and theta.shape == (plan.S, F.N_THETA)):
        raise ValueError("theta must be a contiguous cuda float64 tensor [S,32]")
    if start_colour and (radius is None or status is None):
        raise ValueError("a resumed sweep needs the radius and status of the interrupted one")
    radius = plan._out(plan.S) if radius is None else radius
    st = torch.zeros(plan.S, dtype=torch.int32, device=plan.ctx.device) if status is None else status
    for t, dt in ((radius, torch.float64), (st, torch.int32)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.shape == (plan.S,)):
            raise ValueError("radius / status must be contiguous cuda tensors [S] (float64 / int32)")
    o = F.CelSweepOpts(int(n_sweeps), int(max_newton_iters), int(bool(use_graph)), int(start_colour), int(max_classes))
    rep = F.CelSweepReport()
    F.check("cel_sweep", F.lib.cel_sweep(plan.ctx.h, plan.h, _ptr(theta), _ptr(radius), _ptr(st), C.byref(o),
                                         C.byref(rep), _stream(plan.ctx.device)))
    return radius, st, dict(elbo=rep.elbo_total, n_colours=rep.n_colours, n_newton_steps=rep.n_newton_steps,
                            seconds=rep.seconds, sweeps_done=rep.sweeps_done, next_colour=rep.next_colour)


def psf_fit_at(ctx: Context, eigen, coef, size, fit_img, fit_xy, n_comp=3, n_iter=30):
    """cel_psf_fit: Gaussian-mixture fits of spatially varying PSFs.  eigen [N,E,side,side],
    coef [N,E,6], size [N,2] (W, H), fit_img [n] int, fit_xy [n,2] (host arrays or cuda
    tensors).  Returns a cuda float64 tensor [n, 4, 6]."""
    dev = ctx.device
    as_dev = lambda a, dt: torch.as_tensor(np.asarray(a) if not isinstance(a, torch.Tensor) else a,
                                           dtype=dt).to(dev).contiguous()
    eig, cf, sz = as_dev(eigen, torch.float64), as_dev(coef, torch.float64), as_dev(size, torch.float64)
    fi, fx = as_dev(fit_img, torch.int32), as_dev(fit_xy, torch.float64)
    if eig.dim() != 4 or eig.shape[2] != eig.shape[3] or cf.shape != (eig.shape[0], eig.shape[1], 6) \
            or sz.shape != (eig.shape[0], 2) or fx.shape != (fi.shape[0], 2):
        raise ValueError("psf_fit_at: eigen [N,E,s,s], coef [N,E,6], size [N,2], fit_img [n], fit_xy [n,2]")
    m = F.CelPsfModel(int(eig.shape[0]), int(eig.shape[1]), int(eig.shape[2]), eig.data_ptr(), cf.data_ptr(),
                      sz.data_ptr())
    n = int(fi.shape[0])
    out = torch.zeros((n, F.MAX_PSF, 6), dtype=torch.float64, device=dev)
    F.check("cel_psf_fit", F.lib.cel_psf_fit(ctx.h, C.byref(m), n, _ptr(fi), _ptr(fx), int(n_comp), int(n_iter),
                                             _ptr(out), _stream(dev)))
    return out


def patch_psf_fits(ctx: Context, prob, n_comp=3, n_iter=30):
    """The PSF mixture of every patch of a problem with eigen-PSFs (prob.psf_eigen,
    prob.psf_coef): cel_psf_fit at the centre of each patch.  Returns host float64
    [P, 4, 6], ready for prob.patch_psf."""
    x = prob.patch_x0 + (prob.patch_w - 1) / 2.0
    y = prob.patch_y0 + (prob.patch_h - 1) / 2.0
    size = np.stack([prob.img_W, prob.img_H], 1).astype(np.float64)
    out = psf_fit_at(ctx, prob.psf_eigen, prob.psf_coef, size, prob.patch_img.astype(np.int32),
                     np.stack([x, y], 1), n_comp, n_iter)
    return out.cpu().numpy()


def last_device_error(ctx: Context):
    """cel_last_device_error: CEL_DEVERR_* bits found since the last call (then cleared).
    Synchronises the context's device first."""
    torch.cuda.synchronize(ctx.device)
    code = C.c_int32()
    F.check("cel_last_device_error", F.lib.cel_last_device_error(ctx.h, C.byref(code)))
    return int(code.value)


def save_state(path, theta, radius=None, status=None, cursor=None):
    """Checkpoint the caller-owned optimisation state to an .npz file (host copies)."""
    import numpy as _np
    arrs = dict(theta=theta.detach().cpu().numpy())
    if radius is not None:
        arrs["radius"] = radius.detach().cpu().numpy()
    if status is not None:
        arrs["status"] = status.detach().cpu().numpy()
    if cursor is not None:
        arrs["cursor"] = _np.asarray([cursor.get("sweeps_done", 0), cursor.get("next_colour", 0)], _np.int64)
    _np.savez(path, **arrs)


def load_state(path, device):
    """Inverse of save_state: (theta, radius or None, status or None, cursor dict or None)."""
    import numpy as _np
    with _np.load(path, allow_pickle=False) as z:
        th = torch.as_tensor(z["theta"]).to(device).contiguous()
        r = torch.as_tensor(z["radius"]).to(device).contiguous() if "radius" in z else None
        st = torch.as_tensor(z["status"]).to(device).contiguous() if "status" in z else None
        cur = dict(sweeps_done=int(z["cursor"][0]), next_colour=int(z["cursor"][1])) if "cursor" in z else None
    return th, r, st, cur
