"""Continuous-batching request loop over the celmi library (sky-region cataloging requests).

Each request is a region: its own sources, patches, pixels and initial parameters.  The
loop keeps a set of resident requests whose variational state (theta, trust radii) stays
in device memory.  At every device step:
  1. requests that have arrived are admitted, oldest first, while twice the estimated
     device footprint of the requests laid out in the plan stays within the HBM budget (the
     plan's arrays grow by doubling); a request that does not fit waits, it is never failed
     for lack of memory.  Admission appends the request to the resident plan
     (cel_plan_append): only the request is prepared, so it costs the same whatever is
     resident;
  2. one trust-region Newton round runs, in one batched cel_newton_step, on every resident
     request's current colour class (a request cycles through its classes);
  3. requests that have completed their rounds leave: their parameters and objective are
     copied to the host and the latency (arrival to result on the host) is recorded;
     cancelled requests leave without a result (a request may be cancelled while pending
     or after a given number of rounds).  A request that leaves stays laid out, masked
     out, until such requests hold more than half of the plan's sources; the resident
     requests are then laid out again in a new plan.
Work of different requests shares launches; a request's results do not depend on which
others are resident (every per-source reduction has a fixed order).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api

VARIANTS_EXACT = 2           # Newton with the exact Hessian: iterate, trial
VARIANTS_FD = 56             # Newton with a difference Hessian: iterate, 54 differences, trial
# bytes of one component table (device.h: Table<float>; Table<double> is twice as large):
# header 16, star 4 x 8, star cut radii 4, galaxy cut radii 4 x 16, star exponent rows
# 4 x 4, padding 4, galaxy exponent records 4 x 16 x 8, galaxy 4 x 16 x 4,
# second-derivative terms 4 x 16 x 8, PSF offsets 4 x 2, row recurrence factors 4 x 17,
# padding 12
TABLE_F = 4 * (16 + 4 * 8 + 4 + 4 * 16 + 4 * 4 + 4 + 4 * 16 * 8 + 4 * 16 * 4 + 4 * 16 * 8 + 4 * 17 + 20)
TABLE_D = 2 * TABLE_F
CHUNK = 512                  # pixels per work item (the library's default)
IMAGE_RECORD = 280           # sizeof(cel_image)
PRIOR_RECORDS = 8192         # prior and profile tables, rounded up


def _al(b):
    return (int(b) + 255) // 256 * 256


def neighbour_entries(prob):
    """Entries of the patch overlap lists: ordered pairs of patches of different sources
    whose rectangles intersect in the same image."""
    e = 0
    for n in np.unique(prob.patch_img):
        ps = np.nonzero(prob.patch_img == n)[0]
        x0, y0 = prob.patch_x0[ps].astype(np.int64), prob.patch_y0[ps].astype(np.int64)
        x1, y1 = x0 + prob.patch_w[ps], y0 + prob.patch_h[ps]
        src = prob.patch_src[ps]
        inter = ((x0[:, None] < x1[None, :]) & (x0[None, :] < x1[:, None]) & (y0[:, None] < y1[None, :])
                 & (y0[None, :] < y1[:, None]) & (src[:, None] != src[None, :]))
        e += int(inter.sum())
    return e


def footprint_bytes(prob, variants=VARIANTS_EXACT, fp64=False, chunk=CHUNK):
    """Device bytes a request's own plan holds once Newton steps have run (an upper bound of
    cel_plan_info's device_bytes): the plan's tables and lists, pixels, data constants and
    moment maps, `variants` component tables (float64 ones when fp64: the Hessian on float64
    pixels) with their slot rows and per-source outputs, and the Newton scratch (Hessian
    slots and matrices).  Every block counted rounded up to 256 bytes."""
    S, N, P = int(prob.n_sources), int(len(prob.img_band)), int(len(prob.patch_src))
    sizes = prob.patch_w.astype(np.int64) * prob.patch_h
    U = int(sizes.sum())
    T = int(((sizes + chunk - 1) // chunk).sum())
    E = neighbour_entries(prob)
    C = 16                                   # colour classes (each adds three aligned lists)
    # (work items 16 bytes, their launch order 4, moment-map work items 32: at most one per
    # work item, a patch's overlap box being no larger than the patch)
    pack = (_al(P * 48) + _al(N * IMAGE_RECORD) + _al(E * 4) + _al(T * 16) + _al(T * 4) + _al(T * 32) + _al((S + 1) * 4)
            + _al(N * 4) + PRIOR_RECORDS + _al(P * 8) + _al(len(prob.sky_knots) * 8) + _al(S * 8) + _al(S * 4)
            + (S + P + T) * 4 + 3 * C * 256)
    pixels = _al(U * 8) + _al(2 * P * 8) + _al(P * 8) + 256 + _al(U * 8)          # (count, sky), constants, maps
    if fp64:
        pixels += 2 * _al(U * 16)
    # the plan keeps the one-variant tables and sums made at preparation beside those of the
    # Newton steps
    tables = _al(P * TABLE_F) + (_al(variants * P * TABLE_D) if fp64 else _al(variants * P * TABLE_F))
    sums = sum(_al(nv * T * 128) + 2 * _al(nv * S * 8) + _al(nv * S * 256) for nv in (1, variants))
    newton = (_al(S * 256) + 2 * _al(S * 8) + 2 * _al(S) + 256 + _al(T * 640) + _al(S * 4) + _al(P * 4)
              + _al(T * 4) + _al(S * 5832) + _al(S * 24320))
    return pack + pixels + tables + sums + newton + SLACK


SLACK = 1 << 16              # blocks beyond those counted above (alignment of small lists)


SHARED = ("prior_a", "prior_r", "prior_cw", "prior_cmean", "prior_ccov", "prior_radius", "prior_profile",
          "prior_axis", "exp_alpha", "exp_tau", "dev_alpha", "dev_tau")


def same_model(a, b):
    """True when two requests share the prior and the galaxy profile mixtures."""
    return all(np.array_equal(np.asarray(getattr(a, k)), np.asarray(getattr(b, k))) for k in SHARED)


def merge(probs):
    """One problem holding the given requests side by side (ids offset; images, patches,
    sky knots and pixels concatenated).  All requests must share the prior and profiles
    (ValueError otherwise)."""
    base = probs[0]
    for p in probs[1:]:
        if not same_model(base, p):
            raise ValueError("requests with different priors or profiles cannot share a plan")
    S_off, N_off, K_off, X_off = 0, 0, 0, 0
    cols = {k: [] for k in ("img_band", "img_H", "img_W", "img_npsf", "img_psf", "img_A", "img_b", "img_iota",
                            "img_sky_qh", "img_sky_qw", "img_sky_off", "sky_knots", "patch_src", "patch_img",
                            "patch_x0", "patch_y0", "patch_w", "patch_h", "patch_off", "theta0")}
    for p in probs:
        for k in ("img_band", "img_H", "img_W", "img_npsf", "img_psf", "img_A", "img_b", "img_iota", "img_sky_qh",
                  "img_sky_qw", "patch_x0", "patch_y0", "patch_w", "patch_h", "theta0", "sky_knots"):
            cols[k].append(getattr(p, k))
        cols["img_sky_off"].append(p.img_sky_off + K_off)
        cols["patch_src"].append(p.patch_src + S_off)
        cols["patch_img"].append(p.patch_img + N_off)
        cols["patch_off"].append(p.patch_off + X_off)
        S_off += p.n_sources
        N_off += len(p.img_band)
        K_off += len(p.sky_knots)
        X_off += len(p.pixels)
    out = _Merged()
    for k, v in cols.items():
        setattr(out, k, np.concatenate(v) if v else v)
    out.n_sources = S_off
    for k in SHARED:
        setattr(out, k, getattr(base, k))
    out.pixels = np.zeros(0, np.float32)   # pixels are passed on the device
    return out


class _Merged:
    pass


@dataclass
class Request:
    rid: int
    prob: object
    arrival: float                     # seconds since the loop started
    rounds: int = 10
    cancel_after_rounds: int = None    # cancel once this many rounds are done (None: never)
    cancelled: bool = False
    # device state
    theta: torch.Tensor = None
    radius: torch.Tensor = None
    pixels: torch.Tensor = None
    colours: np.ndarray = None
    n_colours: int = 1
    done_rounds: int = 0
    admitted: float = None
    finished: float = None
    result_theta: np.ndarray = None
    result_local: np.ndarray = None
    result_status: np.ndarray = None
    footprint: int = 0
    units: int = 0
    offset: int = 0
    in_plan: bool = False             # laid out in the current merged plan


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    steps: int = 0
    deferred_admissions: int = 0
    admissions: int = 0
    rebuilds: int = 0             # re-layouts of the resident set (after most of a plan left)
    cancelled: int = 0
    units_evaluated: int = 0
    wall: float = 0.0
    admit_s: list = field(default_factory=list)          # seconds per admission
    admit_resident: list = field(default_factory=list)   # sources in the plan before it
    admit_sources: list = field(default_factory=list)    # sources of the admitted request

    def summary(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        out = dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                   mean_ms=float(lat.mean() * 1e3), completed=len(self.latencies),
                   req_per_s=len(self.latencies) / max(self.wall, 1e-9), steps=self.steps,
                   admissions=self.admissions, deferred_admissions=self.deferred_admissions,
                   rebuilds=self.rebuilds, cancelled=self.cancelled,
                   units_per_s=self.units_evaluated / max(self.wall, 1e-9), wall_s=self.wall)
        if self.admit_s:
            a = np.array(self.admit_s) * 1e3
            res = np.array(self.admit_resident, dtype=np.float64)
            own = np.array(self.admit_sources, dtype=np.float64)
            out["admission_ms"] = dict(p50=float(np.percentile(a, 50)), p99=float(np.percentile(a, 99)),
                                       mean=float(a.mean()))
            # admission time against the resident set and against the request's own size:
            # least-squares slopes of ms on sources (a cost independent of the resident set
            # has a resident slope near zero)
            if len(a) > 2 and np.ptp(res) > 0 and np.ptp(own) > 0:
                X = np.column_stack([np.ones_like(a), res, own])
                coef = np.linalg.lstsq(X, a, rcond=None)[0]
                out["admission_ms"].update(ms_per_resident_source=float(coef[1]),
                                           ms_per_request_source=float(coef[2]),
                                           resident_sources_max=int(res.max()))
        return out


class Server:
    """Continuous-batching loop on one device.

    Admission appends the request to the resident plan (cel_plan_append: the request alone is
    prepared and spliced in, so an admission costs what the request costs, whatever is
    resident).  The parameters and trust radii of everything laid out in the plan live in
    one device array each, grown by doubling.  A request that finishes or is cancelled stays
    laid out, masked out of the Newton rounds, until such requests hold more than half of
    the plan's sources; the resident requests are then laid out again in a new plan (its cost
    amortised over the requests that left)."""

    def __init__(self, device=0, hbm_budget_bytes=16 << 30, rounds=10, **ctx_opts):
        self.ctx = api.Context(device, **ctx_opts)
        self.dev = self.ctx.device
        self.variants = VARIANTS_FD if ctx_opts.get("hessian_fd") else VARIANTS_EXACT
        self.fp64 = bool(ctx_opts.get("hessian_fp64") or ctx_opts.get("pixel_fp64"))
        self.budget = int(hbm_budget_bytes)
        self.rounds = int(rounds)
        self.resident: list[Request] = []
        self.plan = None
        self.laid: list[Request] = []       # requests laid out in the plan, in order
        self.theta_buf = self.radius_buf = None
        self.stats = Stats()

    # -- admission and layout --------------------------------------------------------------
    def _rows(self):
        return self.plan.S if self.plan is not None else 0

    def _ensure_rows(self, n, used):
        """Room for n rows of parameters and radii, the first `used` kept."""
        cap = 0 if self.theta_buf is None else self.theta_buf.shape[0]
        if n <= cap:
            return
        new_cap = max(n, 2 * cap, 64)
        th = torch.empty((new_cap, 32), dtype=torch.float64, device=self.dev)
        ra = torch.empty(new_cap, dtype=torch.float64, device=self.dev)
        if used:
            th[:used] = self.theta_buf[:used]
            ra[:used] = self.radius_buf[:used]
        self.theta_buf, self.radius_buf = th, ra

    def _lay_out(self, r, theta=None, radius=None):
        """Append request r to the plan (or start one); its state from theta/radius or its
        initial parameters."""
        p = r.prob
        if r.pixels is None:
            r.pixels = torch.as_tensor(np.ascontiguousarray(p.pixels, np.float32)).to(self.dev)
        if self.plan is None:
            self.plan = api.Plan(self.ctx, p, pixels_device=r.pixels)
            first = 0
        else:
            first = self.plan.append(p, pixels_device=r.pixels)
        n = p.n_sources
        self._ensure_rows(first + n, first)
        self.theta_buf[first:first + n] = (torch.as_tensor(p.theta0, dtype=torch.float64, device=self.dev)
                                           if theta is None else theta)
        self.radius_buf[first:first + n] = 1.0 if radius is None else radius
        r.offset = first
        r.colours = self.plan.colours[first:first + n]
        r.n_colours = int(r.colours.max()) + 1 if n else 1
        r.in_plan = True
        self.laid.append(r)

    def _admit(self, r, now):
        t0 = time.perf_counter()
        before = self._rows()
        r.admitted = now
        r.rounds = self.rounds
        r.units = int(np.sum(r.prob.patch_w.astype(np.int64) * r.prob.patch_h))
        self._lay_out(r)
        self.resident.append(r)
        self.stats.admissions += 1
        self.stats.admit_s.append(time.perf_counter() - t0)
        self.stats.admit_resident.append(before)
        self.stats.admit_sources.append(r.prob.n_sources)

    def _relayout(self):
        """A new plan holding the resident requests only (their state carried over)."""
        keep = [(r, self.theta_buf[r.offset:r.offset + r.prob.n_sources].clone(),
                 self.radius_buf[r.offset:r.offset + r.prob.n_sources].clone()) for r in self.resident]
        for r in self.laid:
            r.in_plan = False
        self.plan = None
        self.laid = []
        self.theta_buf = self.radius_buf = None
        for r, th, ra in keep:
            self._lay_out(r, th, ra)
        self.stats.rebuilds += 1

    def _cancel(self, r):
        r.cancelled = True
        r.pixels = None
        self.stats.cancelled += 1

    def _leave(self, gone):
        self.resident = [r for r in self.resident if r not in gone]
        for r in gone:
            r.pixels = None

    def step(self, now, pending):
        """Admit what fits from `pending` (arrived requests, oldest first), run one Newton
        round for every resident request, retire finished and cancelled ones.  Returns the
        retired requests."""
        cancelled = [r for r in pending if r.cancel_after_rounds is not None and r.cancel_after_rounds <= 0]
        for r in cancelled:
            pending.remove(r)
        gone = [r for r in self.resident
                if r.cancel_after_rounds is not None and r.done_rounds >= r.cancel_after_rounds]
        if gone:
            self._leave(gone)
        cancelled += gone
        for r in cancelled:
            self._cancel(r)
        # requests that left but are still laid out count until the next re-layout; the
        # plan's arrays grow by doubling, so twice the laid-out footprint is held to the budget
        idle = sum(r.prob.n_sources for r in self.laid if r not in self.resident)
        if self.plan is not None and 2 * idle > self.plan.S:
            self._relayout()
        used = sum(r.footprint for r in self.laid)
        while pending:
            r = pending[0]
            r.footprint = r.footprint or footprint_bytes(r.prob, self.variants, self.fp64)
            if 2 * (used + r.footprint) > self.budget and self.resident:
                self.stats.deferred_admissions += 1
                break
            pending.pop(0)
            self._admit(r, now)
            used += r.footprint
        if not self.resident:
            return cancelled
        S = self.plan.S
        mask = np.zeros(S, bool)
        for r in self.resident:
            c = r.done_rounds % r.n_colours
            mask[r.offset:r.offset + r.prob.n_sources] = r.colours == c
        theta, radius = self.theta_buf[:S], self.radius_buf[:S]
        status, local = api.newton_step(self.plan, theta, radius, mask)
        self.stats.steps += 1
        self.stats.units_evaluated += sum(r.units for r in self.resident)
        finished = []
        for r in self.resident:
            r.done_rounds += 1
            if r.done_rounds >= r.rounds:
                finished.append(r)
        if finished:
            theta_h = theta.cpu().numpy()
            tot_local = local.cpu().numpy()
            st = status.cpu().numpy()
            t_done = time.perf_counter()
            for r in finished:
                sl = slice(r.offset, r.offset + r.prob.n_sources)
                r.result_theta = theta_h[sl].copy()
                r.result_local = tot_local[sl]
                r.result_status = st[sl]
                r.finished = t_done
            self._leave(finished)
        return finished + cancelled

    def run(self, requests, realtime=True):
        """Serve `requests` (each with .arrival seconds from start).  Returns the stats
        summary; results are left on the Request objects."""
        order = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = time.perf_counter()
        pending, i, done = [], 0, 0
        while done < len(order):
            now = time.perf_counter() - t0 if realtime else float("inf")
            while i < len(order) and order[i].arrival <= now:
                pending.append(order[i])
                i += 1
            if not pending and not self.resident:
                if realtime and i < len(order):
                    time.sleep(max(0.0, order[i].arrival - now))
                continue
            fin = self.step(now, pending)
            for r in fin:
                if not r.cancelled:
                    self.stats.latencies.append((r.finished - t0) - r.arrival if realtime else r.finished - t0)
                done += 1
        torch.cuda.synchronize(self.dev)
        self.stats.wall = time.perf_counter() - t0
        return self.stats.summary()


def solo(prob, rounds=10, device=0, **ctx_opts):
    """The same rounds for one request alone (reference for the mixed runs)."""
    srv = Server(device, rounds=rounds, **ctx_opts)
    r = Request(0, prob, 0.0)
    srv.run([r], realtime=False)
    return r
