"""Write the stored oracle values under tests/golden/.  Calls only oracle/ and the seeded
generator synth/; nothing here touches the HIP library.

The paper prints no worked numeric example of the objective, its gradient or a Newton step
(its printed numbers are accuracy and run-time results on survey data that is not
available here), so these files hold the oracle's own values on the seeded workloads:
they let the GPU tests compare the HIP path with the oracle at sizes where the oracle takes
minutes, and pin the oracle against unintended change.  Each .npz records a hash of the
generated inputs (input_sha256, see tests/golden/inputs_hash.py); a test first checks that
the generator still produces the same inputs.

  config1       config1_oracle.json: ELBO, L_s and gradient, 1 star + 1 galaxy
  skew_sweep    skew_sweep.npz: two oracle sweeps (float64) on the skewed small field
  config2       config2_oracle.npz: global ELBO, every L_s and gradient, 1000 sources
  config3       config3_oracle.npz: every gradient of 4096 sources; central differences
                (h = 1e-4) of L_s in all 27 coordinates for 128 sampled sources
  config4       config4_oracle.npz: every L_s and gradient of the 600-source field at the
                initial point, its global ELBO, and one oracle Newton step (with its local
                model g, H, p, predicted gain) for the first 48 sources of colour class 0
  config4_sweep config4_sweep.npz: three oracle sweeps of the field (float64)
  mcmc          mcmc_oracle.npz: the oracle's MCMC source step (annealed importance
                sampling, slice sampling, type draw, the chains' potential scale
                reduction) of both sources of a small problem
  eigen         eigen_oracle.npz: the field with a spatially varying PSF (E = 4 eigen-
                images of 51 x 51 knots) and a 192 x 256 sky knot grid: the oracle's PSF
                fit of every patch, every L_s and gradient and the global ELBO

Run from the repository root:  python -m tests.golden.make_golden NAME [NAME ...]
(per-source work runs in a process pool; CEL_GOLDEN_PROCS sets its size, default 8).
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np
import torch

from oracle import elbo as E
from oracle import newton as NW
from oracle import mcmc as MC
from oracle import psf as OP
from synth import gen
from tests.golden.inputs_hash import inputs_hash

HERE = os.path.dirname(os.path.abspath(__file__))
PROCS = int(os.environ.get("CEL_GOLDEN_PROCS", "8"))
FD_H = 1e-4
N_FD = 128
N_STEP = 48

_M = None      # the model shared with forked workers


def _pool():
    return mp.get_context("fork").Pool(PROCS, initializer=torch.set_num_threads, initargs=(1,))


def _value_grad(s):
    v, g = E.local_value_grad(_M, _M.prob.theta0, s)
    return v, g


def _fd_row(s):
    f = E.local_objective(_M, _M.prob.theta0, s)
    base = torch.as_tensor(_M.prob.theta0[s, :E.N_PARAM], dtype=torch.float64)
    out = np.zeros(E.N_PARAM)
    for k in range(E.N_PARAM):
        e = torch.zeros(E.N_PARAM, dtype=torch.float64)
        e[k] = FD_H
        out[k] = (f(base + e).item() - f(base - e).item()) / (2 * FD_H)
    return out


def _step(s):
    info = {}
    th, r, st, loc = NW.newton_step_source(_M, _M.prob.theta0, s, 1.0, info=info)
    z = np.zeros((E.N_PARAM, E.N_PARAM))
    return th, r, st, loc, info.get("g", np.zeros(E.N_PARAM)), info.get("H", z), \
        info.get("p", np.zeros(E.N_PARAM)), info.get("pred", np.nan)


def _total_part(srcs):
    """Owned pixel terms of the patches of `srcs` (the global ELBO's pixel sum, split)."""
    th = torch.as_tensor(_M.prob.theta0, dtype=torch.float64)
    nat = E.natural(th)
    acc = 0.0
    for s in srcs:
        for p in _M.patches_of[s]:
            Ev, Vv = E.patch_rate(_M, nat, p)
            T = E.pixel_terms(_M.pixels(p), Ev, Vv)
            acc += T[E.owned_mask(_M, p)].sum().item()
    return acc


def _global_elbo(pool, S):
    parts = pool.map(_total_part, [list(range(k, min(S, k + 25))) for k in range(0, S, 25)])
    kl = E.kl_terms(_M, E.natural(torch.as_tensor(_M.prob.theta0, dtype=torch.float64)))["total"].sum().item()
    return float(sum(parts) - kl)


def _all_value_grad(pool, S):
    res = pool.map(_value_grad, range(S), chunksize=4)
    loc = np.array([r[0] for r in res])
    g = np.zeros((S, gen.N_THETA))
    g[:, :E.N_PARAM] = np.array([r[1] for r in res])
    return loc, g


def _save(name, prob, **arrs):
    path = os.path.join(HERE, name)
    np.savez_compressed(path, input_sha256=np.array(inputs_hash(prob)), workload=np.array(prob.name), **arrs)
    print(f"wrote {path}", flush=True)


def make_config1():
    prob = gen.config1()
    m = E.Model(prob)
    total, local, grad = E.elbo_total_and_grad(m, prob.theta0)
    out = dict(workload=prob.name, seed=gen.SEED_BASE + 1, elbo_total=total, elbo_local=local.tolist(),
               grad=grad.tolist())
    with open(os.path.join(HERE, "config1_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


def make_skew_sweep():
    prob = gen.config_skew()
    m = E.Model(prob)
    th, r, st, rep = NW.sweep(m, prob.theta0, dict(n_sweeps=2, max_iter=15))
    _save("skew_sweep.npz", prob, theta=th, status=st, elbo=np.array(rep["elbo"]), colours=rep["colours"],
          n_sweeps=np.array(2), max_iter=np.array(15))


def make_config2():
    global _M
    prob = gen.config2()
    _M = E.Model(prob)
    with _pool() as pool:
        loc, g = _all_value_grad(pool, prob.n_sources)
        total = _global_elbo(pool, prob.n_sources)
    _save("config2_oracle.npz", prob, elbo_total=np.array(total), elbo_local=loc, grad=g)


def make_config3():
    global _M
    prob = gen.config3()
    _M = E.Model(prob)
    fd_src = np.sort(np.random.default_rng(gen.SEED_BASE + 3).choice(prob.n_sources, N_FD, replace=False))
    with _pool() as pool:
        loc, g = _all_value_grad(pool, prob.n_sources)
        fd = np.array(pool.map(_fd_row, fd_src.tolist()))
    _save("config3_oracle.npz", prob, elbo_local=loc, grad=g, fd_sources=fd_src, fd_grad=fd, fd_h=np.array(FD_H))


def make_config4():
    global _M
    prob = gen.config4()
    _M = E.Model(prob)
    colours = NW.greedy_colouring(NW.overlap_graph(_M))
    step_src = np.nonzero(colours == 0)[0][:N_STEP]
    with _pool() as pool:
        loc, g = _all_value_grad(pool, prob.n_sources)
        total = _global_elbo(pool, prob.n_sources)
        res = pool.map(_step, step_src.tolist())
    _save("config4_oracle.npz", prob, elbo_total=np.array(total), elbo_local=loc, grad=g, colours=colours,
          step_sources=step_src, step_theta=np.array([r[0] for r in res]), step_radius=np.array([r[1] for r in res]),
          step_status=np.array([r[2] for r in res], np.int32), step_local=np.array([r[3] for r in res]),
          step_g=np.array([r[4] for r in res]), step_H=np.array([r[5] for r in res]),
          step_p=np.array([r[6] for r in res]), step_pred=np.array([r[7] for r in res]))


def _class_step(args):
    s, radius = args
    th, r, st, loc = NW.newton_step_source(_M, _THETA, s, radius)
    return th, r, st


_THETA = None


def make_config4_sweep(n_sweeps=3, max_iter=50):
    """The oracle's block-coordinate ascent (oracle.newton.sweep) on the field, with the
    sources of a colour class stepped in a process pool: they do not overlap, so each
    step depends only on the class's common iterate (parallel equals serial)."""
    global _M, _THETA
    prob = gen.config4()
    _M = E.Model(prob)
    o = dict(NW.DEFAULTS)
    colours = NW.greedy_colouring(NW.overlap_graph(_M))
    S = prob.n_sources
    theta = prob.theta0.copy()
    status = np.zeros(S, np.int32)
    n_steps = 0
    t0 = time.time()
    for sw in range(n_sweeps):
        radius = np.full(S, o["radius0"])
        for c in range(int(colours.max()) + 1):
            active = colours == c
            for it in range(max_iter):
                if not active.any():
                    break
                _THETA = theta
                idx = np.nonzero(active)[0]
                with _pool() as pool:
                    res = pool.map(_class_step, [(int(s), radius[s]) for s in idx], chunksize=1)
                new = theta.copy()
                for s, (th, r, st) in zip(idx, res):
                    new[s], radius[s], status[s] = th, r, st
                theta = new
                n_steps += 1
                active = active.copy()
                for s, (_, _, st) in zip(idx, res):
                    if st in (NW.ST_CONVERGED, NW.ST_NONFINITE):
                        active[s] = False
            print(f"sweep {sw} class {c}: {n_steps} steps, {time.time() - t0:.0f} s", flush=True)
    prob.theta0 = theta              # _global_elbo evaluates the model's problem at theta0
    with _pool() as pool:
        total = _global_elbo(pool, S)
    prob = gen.config4()             # hash of the unmodified inputs
    _save("config4_sweep.npz", prob, theta=theta, status=status, elbo=np.array(total), colours=colours,
          n_steps=np.array(n_steps), n_sweeps=np.array(n_sweeps), max_iter=np.array(max_iter))


def _fit_patch(p):
    prob = _M.prob
    n = int(prob.patch_img[p])
    x = prob.patch_x0[p] + (prob.patch_w[p] - 1) / 2.0
    y = prob.patch_y0[p] + (prob.patch_h[p] - 1) / 2.0
    img = OP.psf_image(prob.psf_eigen[n], prob.psf_coef[n], float(prob.img_W[n]), float(prob.img_H[n]), x, y)
    return OP.fit_mixture(img, EIGEN_K, EIGEN_ITER)


EIGEN_K, EIGEN_ITER = 3, 30


def make_eigen():
    """The field workload with a spatially varying PSF (eigen-images) and a 192 x 256 sky
    grid: the oracle's PSF fit of every patch (3 components, 30 iterations), then every L_s
    and gradient and the global ELBO with those PSFs."""
    global _M
    prob = gen.config_eigen()
    _M = E.Model(prob)
    with _pool() as pool:
        fits = pool.map(_fit_patch, range(prob.n_patches), chunksize=16)
    psf = np.zeros((prob.n_patches, OP.MAX_PSF, 6))
    psf[:, :EIGEN_K] = np.array(fits)
    _M = E.Model(prob, patch_psf=psf)
    with _pool() as pool:
        loc, g = _all_value_grad(pool, prob.n_sources)
        total = _global_elbo(pool, prob.n_sources)
    _save("eigen_oracle.npz", prob, patch_psf=psf, psf_k=np.array(EIGEN_K), psf_iter=np.array(EIGEN_ITER),
          elbo_total=np.array(total), elbo_local=loc, grad=g)


MCMC_T = 4
MCMC_OPTS = dict(n_temps=MCMC_T, n_runs=3, n_post=2, seed=7, gamma=[(t / MCMC_T) ** 4 for t in range(MCMC_T + 1)])
MCMC_KEY = 3
MCMC_INIT_SEED = 5


def mcmc_problem():
    """The small problem of the stored MCMC step: 1 star + 1 galaxy, bands g and r, patches
    cropped to 12 x 12, the sources at their true points."""
    prob = gen.crop_patches(gen.subset(gen.config1(), images=[1, 2]), 12)
    return prob, gen.truth_point(prob)


def _mcmc_source(s):
    prob, z = mcmc_problem()
    opts = dict(MC.DEFAULTS, **MCMC_OPTS)
    init = gen.prior_draws(prob, z, opts["n_runs"], seed=MCMC_INIT_SEED, box=opts["box"])
    return MC.source_step(E.Model(prob), z, s, init[:, :, s], opts, key=(opts["seed"], MCMC_KEY))


def make_mcmc():
    """The oracle's MCMC step of both sources of the small problem (T = 4, N' = 3, B' = 2)."""
    prob, _ = mcmc_problem()
    with _pool() as pool:
        res = pool.map(_mcmc_source, range(prob.n_sources))
    opts = dict(MC.DEFAULTS, **MCMC_OPTS)
    _save("mcmc_oracle.npz", prob, samples=np.array([r["samples"] for r in res]),
          log_evidence=np.array([r["log_evidence"] for r in res]), p_star=np.array([r["p_star"] for r in res]),
          z=np.array([r["z"] for r in res]), a=np.array([r["a"] for r in res]),
          logw=np.array([r["logw"] for r in res]), rhat=np.array([r["rhat"] for r in res]),
          n_temps=np.array(opts["n_temps"]), n_runs=np.array(opts["n_runs"]),
          n_post=np.array(opts["n_post"]), gamma=np.array(opts["gamma"]), width=np.array(opts["width"]),
          box=np.array(opts["box"]), max_step_out=np.array(opts["max_step_out"]),
          max_shrink=np.array(opts["max_shrink"]), seed=np.array(opts["seed"]), key=np.array(MCMC_KEY),
          init_seed=np.array(MCMC_INIT_SEED))


MAKERS = dict(config1=make_config1, skew_sweep=make_skew_sweep, config2=make_config2, config3=make_config3,
              config4=make_config4, config4_sweep=make_config4_sweep, eigen=make_eigen, mcmc=make_mcmc)

if __name__ == "__main__":
    for name in sys.argv[1:] or ["config1"]:
        t = time.time()
        MAKERS[name]()
        print(f"{name}: {time.time() - t:.0f} s", flush=True)
