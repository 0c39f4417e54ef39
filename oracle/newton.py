"""Reference trust-region Newton block step, overlap colouring and block coordinate ascent.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 4.3: each source is a block; a block is improved by Newton's method with a
Euclidean-ball trust region (the subproblem of Nocedal & Wright, Numerical Optimization,
ch. 4), with a dense Hessian.  Section 4.4: sources that do not overlap can be optimised
in parallel with the same result as serially, so blocks are grouped by a colouring of the
overlap graph.  The paper prints no trust-region constants; the ones below are this
implementation's reading:
  initial radius 1, maximum radius 100, accept if rho > 0.1, shrink to 0.25*|p| if
  rho < 0.25, double (capped) if rho > 0.75 and the step reached the boundary;
  converged when |g|_inf <= gtol * max(1, |L_s| / n_pix), or the model's predicted gain
  <= ftol * max(1, |L_s|), or the radius < 1e-8; colour classes in ascending colour, greedy
  colouring in ascending source id; the radius is reset to its initial value at the start
  of every sweep.
"""
from __future__ import annotations

import math

import numpy as np

from . import elbo as E

ST_SKIPPED, ST_ACCEPTED, ST_REJECTED, ST_CONVERGED, ST_NONFINITE = 0, 1, 2, 3, 4

DEFAULTS = dict(radius0=1.0, radius_max=100.0, eta=0.1, gtol=1e-6, ftol=1e-9, radius_min=1e-8,
                max_iter=50, n_sweeps=3)


def tr_subproblem(g, H, delta, hard_tol=1e-12):
    """argmax_p g.p + 1/2 p^T H p subject to |p| <= delta.

    Optimality (Nocedal & Wright, Theorem 4.1): (B + lam I) p = g with B = -H, lam >= 0,
    lam (delta - |p|) = 0 and B + lam I positive semidefinite.  Uses the eigenvectors of B;
    the boundary multiplier is found by bisection on |p(lam)| = delta.  In the hard case
    (g orthogonal to the lowest eigenvector) the step is completed along that eigenvector,
    oriented so its largest-magnitude entry is positive.  Returns (p, lam, hard).
    Pinned by KKT residuals, brute force in 2-D and the interior Newton step."""
    g = np.asarray(g, dtype=np.float64)
    B = -0.5 * (np.asarray(H, dtype=np.float64) + np.asarray(H, dtype=np.float64).T)
    lam_e, Q = np.linalg.eigh(B)
    gt = Q.T @ g
    lmin = lam_e[0]
    if lmin > 0:
        p = Q @ (gt / lam_e)
        if np.linalg.norm(p) <= delta:
            return p, 0.0, False

    def norm_p(lam):
        return math.sqrt(float(np.sum((gt / (lam_e + lam)) ** 2)))

    lo = max(0.0, -lmin)
    gnorm = float(np.linalg.norm(g))
    low = np.abs(lam_e - lmin) <= 1e-12 * max(1.0, abs(lmin))
    if np.all(np.abs(gt[low]) <= hard_tol * max(gnorm, 1e-300)):
        rest = ~low
        denom = lam_e[rest] + lo
        p_rest = Q[:, rest] @ (gt[rest] / denom) if np.any(rest) else np.zeros_like(g)
        nr = float(np.linalg.norm(p_rest))
        if nr <= delta:
            q = Q[:, np.nonzero(low)[0][0]].copy()
            if q[np.argmax(np.abs(q))] < 0:
                q = -q
            return p_rest + math.sqrt(max(delta * delta - nr * nr, 0.0)) * q, lo, True
    # |p(lam)| decreases from +inf (or |p(lo)|) to 0 on (lo, inf); bracket and bisect
    hi = lo + gnorm / delta + 1.0
    while norm_p(hi) > delta:
        hi = lo + 2.0 * (hi - lo)
    a, b = lo, hi
    for _ in range(400):
        mid = 0.5 * (a + b)
        if mid == a or mid == b:
            break
        if norm_p(mid) > delta:
            a = mid
        else:
            b = mid
    lam = b
    return Q @ (gt / (lam_e + lam)), lam, False


def overlap_graph(model):
    """Sources are adjacent when any of their patches intersect in the same image."""
    S = model.S
    adj = [set() for _ in range(S)]
    for p, cov in enumerate(model.cover):
        if cov is None:
            continue
        s = model.psrc[p]
        for q in cov:
            t = model.psrc[q]
            if t != s:
                adj[s].add(int(t))
    return [sorted(a) for a in adj]


def greedy_colouring(adj):
    """Ascending source id, smallest colour unused by already-coloured neighbours."""
    colour = np.full(len(adj), -1, dtype=np.int64)
    for s in range(len(adj)):
        used = {colour[t] for t in adj[s] if colour[t] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[s] = c
    return colour


def newton_step_source(model, theta, s, radius, opts=None, info=None):
    """One trust-region Newton step on source s with every other source fixed.
    Returns (theta_s_new[32], radius_new, status, L_s at the returned point).  A dict passed
    as `info` receives the step's local model: L, g, H (when formed), the subproblem's
    solution p and its predicted gain."""
    o = dict(DEFAULTS, **(opts or {}))
    theta = np.asarray(theta, dtype=np.float64)
    L, g = E.local_value_grad(model, theta, s)
    if info is not None:
        info.update(L=L, g=g)
    ts = theta[s].copy()
    if not (np.isfinite(L) and np.all(np.isfinite(g)) and np.all(np.isfinite(ts))):
        return ts, radius, ST_NONFINITE, L
    npix = E.n_active_pixels(model, s)
    if np.max(np.abs(g)) <= o["gtol"] * max(1.0, abs(L) / max(npix, 1)) or radius < o["radius_min"]:
        return ts, radius, ST_CONVERGED, L
    H = E.local_hessian(model, theta, s)
    p, _, _ = tr_subproblem(g, H, radius)
    pred = float(g @ p + 0.5 * p @ H @ p)
    if info is not None:
        info.update(H=H, p=p, pred=pred)
    if pred <= o["ftol"] * max(1.0, abs(L)):
        return ts, radius, ST_CONVERGED, L
    trial = theta.copy()
    trial[s, :E.N_PARAM] += p
    Lt = E.elbo(model, trial, sources=[s], with_total=False)[1][s].item()
    pn = float(np.linalg.norm(p))
    if not np.isfinite(Lt):
        return ts, 0.25 * pn, ST_REJECTED, L
    rho = (Lt - L) / pred
    if rho < 0.25:
        radius = 0.25 * pn
    elif rho > 0.75 and pn >= 0.99 * radius:
        radius = min(2.0 * radius, o["radius_max"])
    if rho > o["eta"]:
        return trial[s].copy(), radius, ST_ACCEPTED, Lt
    return ts, radius, ST_REJECTED, L


def newton_step(model, theta, radius, mask=None, opts=None):
    """Step every source in `mask` (pairwise non-overlapping) from the same iterate.
    Returns (theta, radius, status[S], elbo_local[S] (nan where skipped))."""
    theta = np.array(theta, dtype=np.float64)
    radius = np.array(radius, dtype=np.float64)
    S = model.S
    mask = np.ones(S, bool) if mask is None else np.asarray(mask, bool)
    status = np.zeros(S, np.int32)
    loc = np.full(S, np.nan)
    new = theta.copy()
    for s in np.nonzero(mask)[0]:
        new[s], radius[s], status[s], loc[s] = newton_step_source(model, theta, s, radius[s], opts)
    return new, radius, status, loc


def sweep(model, theta, opts=None, radius=None):
    """Block coordinate ascent: for each sweep and colour class (ascending), Newton steps on
    the class until every member has converged or max_iter steps were taken.
    Returns (theta, radius, status, report)."""
    o = dict(DEFAULTS, **(opts or {}))
    theta = np.array(theta, dtype=np.float64)
    S = model.S
    colour = greedy_colouring(overlap_graph(model))
    status = np.zeros(S, np.int32)
    iters = np.zeros(S, np.int64)
    n_steps = 0
    for sw in range(o["n_sweeps"]):
        radius = np.full(S, o["radius0"])
        for c in range(int(colour.max()) + 1 if S else 0):
            active = colour == c
            for it in range(o["max_iter"]):
                if not active.any():
                    break
                theta, radius, st, _ = newton_step(model, theta, radius, active, o)
                n_steps += 1
                status[active] = st[active]
                iters[active] += 1
                active = active & (st != ST_CONVERGED) & (st != ST_NONFINITE)
    total = E.elbo(model, theta)[0].item()
    return theta, radius, status, dict(elbo=total, colours=colour, iters=iters, n_steps=n_steps)
