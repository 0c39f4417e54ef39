"""Reference MCMC source step: annealed importance sampling with slice-sampling-within-Gibbs
transitions, float64, plain Python.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): the product path never imports this.

Section 3 of the paper samples one light source s at a time with its neighbours' latent
variables held fixed (equation eqzs).  For each source type a (galaxy 0, star 1) it runs N'
independent annealed importance samplers (Section 3.1) from the prior pi_0 = p(w | a) to
the target pi(w) = p(x | w, a, z_-s) p(w | a) through pi_t = pi_0^(1 - gamma_t) pi^gamma_t,
t = 1..T, each transition a slice-sampling-within-Gibbs sweep that leaves pi_t invariant;
the log weight of a run is sum_t (gamma_t - gamma_{t-1}) log p(x | w^(t-1)), and the mean of
the weights estimates p(x | a, z_-s).  Each run's last state then starts a chain of B'
further slice-sampling sweeps at the target (Section 3.2).  Bayes' rule with the prior
p(a) gives p(a = 1 | x, z_-s); a type is drawn from it and one of the N' B' samples of
that type is drawn uniformly (the procedure summarised at the end of Section 3.2).

Slice sampling (the univariate update of Neal, "Slice sampling", Annals of Statistics
2003, with the "stepping out" and "shrinkage" procedures): y = log f(x0) + log U; an
interval of width w placed at random around x0 is stepped out at most m - 1 times, split
at random between the two sides, while its ends lie in the slice; points drawn uniformly
from the interval are accepted once inside the slice, the interval shrinking towards x0
after each rejection.

Readings of what the paper leaves open (stated once, used by the HIP sampler alike):
  * coordinates of w in the point layout of oracle.likelihood (u, log r, colours; for a
    galaxy also angle, log radius, profile weight, axis ratio), updated in that order;
    slice widths per coordinate and the stepping-out limit m are inputs;
  * the position's prior is uniform on a square of half-width `box` pixels around the
    source's fixed (detected) position; its density is the same for both types and left
    out of both the target and the evidence;
  * the angle is periodic (the light kernel has period pi): an accepted angle is mapped to
    [0, pi);
  * temperatures gamma_t = (t / T)^power unless a schedule gamma_0..gamma_T is given;
  * the log target of a point outside the support (either factor -infinity) is -infinity,
    whatever gamma;
  * shrinkage stops after `max_shrink` rejections, keeping x0;
  * random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
    as easy as 1, 2, 3", SC 2011) keyed by (seed, gibbs_key); a 64-bit output x becomes
    the uniform ((x >> 11) + 1/2) 2^-53 in (0, 1).  Counters: the stepping-out triple of
    coordinate i in sweep t of chain c is (0, 16 t + i, c, 0) (outputs: threshold, interval
    position, split); shrinkage draw k of that update is (1 + k, 16 t + i, c, 0); the type
    and sample choice of source s is (0, 0, s, 1).  Chain c of source s, type a, run r is
    (2 s + a) N' + r;
  * the initial states w^(0) ~ pi_0 are inputs (drawn by the caller).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import likelihood as LK

MASK64 = (1 << 64) - 1
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
GALAXY_COORDS = (0, 1, 3, 4, 5, 6, 7, 8, 9, 10, 11)
STAR_COORDS = (0, 1, 3, 4, 5, 6, 7)
ANGLE = 8
NEG_INF = -math.inf


def philox4x64(ctr, key, rounds=10):
    """Philox4x64-10 block: four 64-bit words from a 256-bit counter and a 128-bit key."""
    c = [int(v) & MASK64 for v in ctr]
    k = [int(v) & MASK64 for v in key]
    for _ in range(rounds):
        p0, p1 = PHILOX_M[0] * c[0], PHILOX_M[1] * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & MASK64, (p0 >> 64) ^ c[3] ^ k[1], p0 & MASK64]
        k = [(k[0] + PHILOX_W[0]) & MASK64, (k[1] + PHILOX_W[1]) & MASK64]
    return c


def uniform(x):
    """A 64-bit word as a uniform number in (0, 1): ((x >> 11) + 1/2) 2^-53."""
    return ((int(x) >> 11) + 0.5) * 2.0 ** -53


def schedule(T, power):
    """gamma_0 .. gamma_T = (t / T)^power."""
    return [(t / T) ** power for t in range(T + 1)]


def slice_update(logf, x0, fx0, width, m, draws, max_shrink=200, stats=None):
    """One univariate slice-sampling update of x0 (log density logf, logf(x0) = fx0), with
    stepping out (width, at most m - 1 steps) and shrinkage.  draws(k) returns the
    uniforms: draws(0) -> (U_threshold, U_position, U_split); draws(1 + j) -> U of shrinkage
    draw j.  Returns (x1, logf(x1))."""
    uy, uw, uj = draws(0)
    y = fx0 + math.log(uy)
    L = x0 - width * uw
    R = L + width
    J = math.floor(m * uj)
    K = (m - 1) - J
    n_eval = 0
    while J > 0:
        n_eval += 1
        if not (y < logf(L)):
            break
        L -= width
        J -= 1
    while K > 0:
        n_eval += 1
        if not (y < logf(R)):
            break
        R += width
        K -= 1
    for j in range(max_shrink):
        x1 = L + draws(1 + j)[0] * (R - L)
        f1 = logf(x1)
        n_eval += 1
        if y < f1:
            if stats is not None:
                stats.append(n_eval)
            return x1, f1
        if x1 < x0:
            L = x1
        else:
            R = x1
    if stats is not None:
        stats.append(n_eval)
    return x0, fx0


class SourceTarget:
    """log pi_t of source s at a point w: log p(w | a) + gamma log p(x | w, a, z_-s), with
    the position inside the box; the likelihood and prior from oracle.likelihood."""

    def __init__(self, model, z_fixed, s, box):
        self.model, self.z_fixed, self.s, self.box = model, np.asarray(z_fixed, np.float64), s, box

    def parts(self, w):
        if abs(w[0] - self.z_fixed[self.s, 0]) > self.box or abs(w[1] - self.z_fixed[self.s, 1]) > self.box:
            return NEG_INF, NEG_INF
        lp = LK.log_prior(self.model, w)
        if lp == NEG_INF:
            return NEG_INF, NEG_INF
        return lp, LK.log_likelihood(self.model, self.z_fixed, self.s, w)


def combine(lp, ll, gamma):
    """log pi_t = log pi_0 + gamma log-likelihood; -infinity if either factor is."""
    return NEG_INF if (lp == NEG_INF or ll == NEG_INF) else lp + gamma * ll


def run_chain(target, w0, coords, chain, key, opts, stats=None, periodic=(ANGLE,)):
    """One annealed importance sampling run over the coordinates `coords` of the point w
    (start w0 ~ pi_0; target.parts(w) gives (log pi_0(w), log-likelihood(w))), followed by
    B' slice-sampling sweeps at the target.  Returns (log weight, samples [B', len(w0)])."""
    T, Bp, power = opts["n_temps"], opts["n_post"], opts["gamma_power"]
    widths, m, max_shrink = opts["width"], opts["max_step_out"], opts["max_shrink"]
    gam = list(opts["gamma"]) if opts.get("gamma") is not None else schedule(T, power)
    w = np.array(w0, dtype=np.float64)
    lp, ll = target.parts(w)
    logw = 0.0
    samples = np.zeros((Bp, len(w)))
    for t in range(1, T + Bp + 1):
        if t <= T:
            logw += (gam[t] - gam[t - 1]) * ll
            g = gam[t]
        else:
            g = 1.0
        for i, ci in enumerate(coords):
            def draws(k, _t=t, _i=i):
                out = philox4x64((k, 16 * _t + _i, chain, 0), key)
                return uniform(out[0]), uniform(out[1]), uniform(out[2])

            def logf(x, _ci=ci):
                v = w.copy()
                v[_ci] = x
                lp_, ll_ = target.parts(v)
                logf.last = (lp_, ll_)
                return combine(lp_, ll_, g)

            logf.last = None
            fx0 = combine(lp, ll, g)
            x1, f1 = slice_update(logf, w[ci], fx0, widths[ci], m, draws, max_shrink, stats)
            if x1 != w[ci] or f1 != fx0:
                w[ci] = x1
                lp, ll = logf.last
                if ci in periodic:
                    w[ci] = x1 - math.pi * math.floor(x1 / math.pi)   # period pi
        if t > T:
            samples[t - T - 1] = w
    return logw, samples


def source_step(model, z_fixed, s, z_init, opts, key, stats=None):
    """The MCMC update of source s (equation eqzs) with every other source at z_fixed.
    z_init [2, N', 16]: the start points of the runs per type (draws from the prior).
    Returns dict(z (the new point), p_star = p(a = 1 | x, z_-s), log_evidence [2],
    logw [2, N'], samples [2, N', B', 16], rhat [2, 16]: the N' chains' potential scale
    reduction per type and coordinate)."""
    Np, Bp = opts["n_runs"], opts["n_post"]
    target = SourceTarget(model, z_fixed, s, opts["box"])
    logw = np.zeros((2, Np))
    samples = np.zeros((2, Np, Bp, 16))
    for a in (0, 1):
        for r in range(Np):
            chain = (2 * s + a) * Np + r
            w0 = np.array(z_init[a, r], dtype=np.float64)
            w0[2] = float(a)
            logw[a, r], samples[a, r] = run_chain(target, w0, STAR_COORDS if a == 1 else GALAXY_COORDS, chain,
                                                  key, opts, stats)
    log_ev = np.zeros(2)
    for a in (0, 1):
        mx = logw[a].max()
        log_ev[a] = mx + math.log(np.exp(logw[a] - mx).sum()) - math.log(Np) if np.isfinite(mx) else NEG_INF
    A = float(model.prior_a)
    d = math.log(A) - math.log(1 - A) + log_ev[1] - log_ev[0]
    p_star = 1.0 / (1.0 + math.exp(-d)) if d > -700 else 0.0
    out = philox4x64((0, 0, s, 1), key)
    a_star = 1 if uniform(out[0]) < p_star else 0
    j = min(int(math.floor(uniform(out[1]) * Np * Bp)), Np * Bp - 1)
    z = samples[a_star, j // Bp, j % Bp].copy()
    return dict(z=z, p_star=p_star, log_evidence=log_ev, logw=logw, samples=samples, a=a_star, index=j,
                rhat=np.array([rhat(samples[a]) for a in (0, 1)]))


def rhat(samples):
    """Potential scale reduction factor of m chains of n draws, per coordinate (Gelman and
    Rubin, "Inference from iterative simulation using multiple sequences", Statistical
    Science 1992), the convergence and mixing criterion with which Section 3.2 monitors the
    N' chains of B' steps.  samples [m, n, d] -> [d].  With chain means mean_j, their mean
    g, chain variances s_j^2 (divisor n - 1): B = n / (m - 1) sum_j (mean_j - g)^2,
    W = mean_j s_j^2, V = (n - 1) / n W + B / n, R = sqrt(V / W).  Reading: the basic form,
    without the degrees-of-freedom correction; each coordinate on its own scale (the angle
    as stored, in [0, pi)); a coordinate that does not move in any chain (W = 0) gives
    0 / 0 = NaN, one with W = 0 < B gives +infinity; fewer than 2 chains or 2 draws: NaN."""
    x = np.asarray(samples, dtype=np.float64)
    m, n = x.shape[0], x.shape[1]
    if m < 2 or n < 2:
        return np.full(x.shape[2:], np.nan)
    means = x.mean(axis=1)
    g = means.mean(axis=0)
    B = n / (m - 1) * ((means - g) ** 2).sum(axis=0)
    W = x.var(axis=1, ddof=1).mean(axis=0)
    V = (n - 1) / n * W + B / n
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.sqrt(V / W)


DEFAULTS = dict(n_temps=200, n_runs=25, n_post=25, max_step_out=8, max_shrink=200, gamma_power=4.0, box=2.0,
                width=(0.5, 0.5, 0.0, 0.3, 0.2, 0.2, 0.2, 0.2, 0.5, 0.3, 0.2, 0.2, 0.0, 0.0, 0.0, 0.0))
