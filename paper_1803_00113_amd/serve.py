"""Continuous-batching request loop over the celmi library (sky-region cataloging requests).

Each request is a region: its own sources, patches, pixels and initial parameters.  The
loop keeps a set of resident requests whose variational state (theta, trust radii) stays
in device memory.  At every device step:
  1. requests that have arrived are admitted, oldest first, while the estimated device
     footprint of the resident set stays within the HBM budget (a request that does not
     fit waits; it is never failed for lack of memory);
     Under a burst of arrivals (the last two rebuilds less than two intervals apart),
     admissions are held while the last rebuild of the merged plan is younger than
     `min_rebuild_interval_s`: a rebuild costs a few milliseconds of host work, and arrivals
     a few milliseconds apart then share one; outside bursts an arrival is admitted at once;
  2. if a request was admitted, the resident requests are merged into one plan (their
     pixel arrays are concatenated on the device; sources of different requests never
     overlap, so the merged colouring restricted to a request equals its own), and their
     parameters and trust radii into one device array each;
  3. one trust-radius Newton round runs, in one batched cel_newton_step, on every resident
     request's current colour class (a request cycles through its classes);
  4. requests that have completed their rounds leave: their parameters and objective are
     copied to the host and the latency (arrival to result on the host) is recorded;
     cancelled requests leave without a result (a request may be cancelled while pending
     or after a given number of rounds).  A request that leaves stays in the merged plan,
     masked out, until the next admission rebuilds it (or until such requests hold more
     than half of the plan's sources), so that leaving costs no rebuild.
Work of different requests shares launches; a request's results do not depend on which
others are resident (every per-source reduction has a fixed order).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api

TABLE_BYTES = 1536           # per patch and variant, float32 component table (upper bound)
VARIANTS_EXACT = 2           # Newton with the exact Hessian: iterate, trial
VARIANTS_FD = 56             # Newton with a difference Hessian: iterate, 54 differences, trial


def footprint_bytes(prob, variants=VARIANTS_EXACT):
    """Estimated device bytes a request needs inside a merged plan (pixels, per-pixel
    arrays, Newton tables and slots, Hessian slots and matrices, per-source scratch)."""
    units = int(np.sum(prob.patch_w.astype(np.int64) * prob.patch_h))
    P = int(len(prob.patch_src))
    S = int(prob.n_sources)
    items = int(np.sum((prob.patch_w.astype(np.int64) * prob.patch_h + 511) // 512))
    return (units * (4 + 8 + 8) + P * variants * TABLE_BYTES + items * (variants * 16 + 80) * 8
            + S * variants * (8 + 8 + 32 * 8) + S * (32 * 8 * 3 + 27 * 27 * 8) + P * 64)


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
    held_admissions: int = 0      # steps whose arrivals waited for the rebuild interval
    rebuilds: int = 0
    cancelled: int = 0
    units_evaluated: int = 0
    wall: float = 0.0

    def summary(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                    mean_ms=float(lat.mean() * 1e3), completed=len(self.latencies),
                    req_per_s=len(self.latencies) / max(self.wall, 1e-9), steps=self.steps,
                    deferred_admissions=self.deferred_admissions, held_admissions=self.held_admissions,
                    rebuilds=self.rebuilds,
                    cancelled=self.cancelled,
                    units_per_s=self.units_evaluated / max(self.wall, 1e-9), wall_s=self.wall)


class Server:
    """Continuous-batching loop on one device."""

    def __init__(self, device=0, hbm_budget_bytes=16 << 30, rounds=10, min_rebuild_interval_s=0.01, **ctx_opts):
        self.ctx = api.Context(device, **ctx_opts)
        self.dev = self.ctx.device
        self.variants = VARIANTS_FD if ctx_opts.get("hessian_fd") else VARIANTS_EXACT
        self.budget = int(hbm_budget_bytes)
        self.rounds = int(rounds)
        self.resident: list[Request] = []
        self.plan = None
        self.theta = self.radius = None   # merged state of the requests laid out in the plan
        self.in_plan: list[Request] = []
        self.dirty = False
        self.min_rebuild_interval = float(min_rebuild_interval_s)
        self.last_rebuild = self.prev_rebuild = -float("inf")
        self.stats = Stats()

    # -- admission and merging ---------------------------------------------------------------
    def _attach(self, r: Request, now):
        p = r.prob
        r.theta = torch.as_tensor(p.theta0, dtype=torch.float64, device=self.dev).contiguous()
        r.radius = torch.full((p.n_sources,), 1.0, dtype=torch.float64, device=self.dev)
        r.pixels = torch.as_tensor(np.ascontiguousarray(p.pixels, np.float32)).to(self.dev)
        r.admitted = now
        r.rounds = self.rounds
        r.units = int(np.sum(p.patch_w.astype(np.int64) * p.patch_h))

    def _cancel(self, r):
        r.cancelled = True
        r.theta = r.radius = r.pixels = None
        self.stats.cancelled += 1

    def _rebuild(self):
        # the state of requests already in the plan comes from the merged arrays
        for r in self.resident:
            if r.in_plan:
                sl = slice(r.offset, r.offset + r.prob.n_sources)
                r.theta, r.radius = self.theta[sl], self.radius[sl]
        self.plan = None
        self.theta = self.radius = None
        self.in_plan = []
        if not self.resident:
            return
        merged = merge([r.prob for r in self.resident])
        pixels = torch.cat([r.pixels for r in self.resident])
        self.plan = api.Plan(self.ctx, merged, pixels_device=pixels)
        off = 0
        for r in self.resident:
            r.colours = self.plan.colours[off:off + r.prob.n_sources]
            r.n_colours = int(r.colours.max()) + 1 if r.prob.n_sources else 1
            r.offset = off
            r.in_plan = True
            off += r.prob.n_sources
        self.theta = torch.cat([r.theta for r in self.resident]).contiguous()
        self.radius = torch.cat([r.radius for r in self.resident]).contiguous()
        for r in self.resident:
            r.theta = r.radius = None
        self.in_plan = list(self.resident)
        self.stats.rebuilds += 1

    def _leave(self, gone):
        """Requests leaving the resident set stay in the plan, masked out; a rebuild is
        asked for once they hold more than half of its sources."""
        self.resident = [r for r in self.resident if r not in gone]
        idle = sum(r.prob.n_sources for r in self.in_plan if r not in self.resident)
        if self.plan is not None and 2 * idle > self.plan.S:
            self.dirty = True

    def step(self, now, pending):
        """Admit what fits from `pending` (arrived requests, oldest first), run one Newton
        round for every resident request, retire finished and cancelled ones.  Returns the
        retired requests."""
        changed = False
        # cancellations: pending requests are dropped, resident ones leave the plan
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
        # (requests that left but stay in the plan do not count: an admission rebuilds the
        # plan without them, after the old one is released)
        used = sum(r.footprint for r in self.resident)
        burst = self.last_rebuild - self.prev_rebuild < 2 * self.min_rebuild_interval
        hold = bool(pending) and bool(self.resident) and burst and now - self.last_rebuild < self.min_rebuild_interval
        if hold:
            self.stats.held_admissions += 1
        while pending and not hold:
            r = pending[0]
            r.footprint = r.footprint or footprint_bytes(r.prob, self.variants)
            if used + r.footprint > self.budget and self.resident:
                self.stats.deferred_admissions += 1
                break
            pending.pop(0)
            self._attach(r, now)
            self.resident.append(r)
            used += r.footprint
            changed = True
        if changed or self.dirty:
            self._rebuild()
            self.dirty = False
            self.prev_rebuild, self.last_rebuild = self.last_rebuild, now
        if not self.resident:
            return cancelled
        S = self.plan.S
        mask = np.zeros(S, bool)
        for r in self.resident:
            c = r.done_rounds % r.n_colours
            mask[r.offset:r.offset + r.prob.n_sources] = r.colours == c
        status, local = api.newton_step(self.plan, self.theta, self.radius, mask)
        self.stats.steps += 1
        self.stats.units_evaluated += sum(r.units for r in self.resident)
        finished = []
        for r in self.resident:
            r.done_rounds += 1
            if r.done_rounds >= r.rounds:
                finished.append(r)
        if finished:
            theta_h = self.theta.cpu().numpy()
            tot_local = local.cpu().numpy()
            st = status.cpu().numpy()
            t_done = time.perf_counter()
            for r in finished:
                sl = slice(r.offset, r.offset + r.prob.n_sources)
                r.result_theta = theta_h[sl].copy()
                r.result_local = tot_local[sl]
                r.result_status = st[sl]
                r.finished = t_done
                r.pixels = None
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
