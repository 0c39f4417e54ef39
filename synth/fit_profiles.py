"""Fit the galaxy light-profile constants (alpha_j, tau_j) used by the galaxy light kernel.

The model writes each extremal galaxy profile as a scale mixture of zero-mean bivariate
normals, sum_j alpha_j N(0, tau_j Sigma_s), whose weights and scales are fixed constants
(Section 2.1.2, equation hsi).  The paper does not print them, so this script fits them:
an isotropic mixture is fitted by least squares to the Sersic profile of index n (n=1
exponential, 6 components; n=4 de Vaucouleurs, 8 components) with half-light radius 1.
The result is then normalised so that sum(alpha) = 1 exactly (the kernel is a density)
and the scales are rescaled so the mixture's half-light radius is exactly 1, which is how
the model defines e_radius (Section 2.1.2).

Run:  python -m synth.fit_profiles   (writes synth/profiles.json)
The output is input data for both the reference and the HIP path; it holds no method
arithmetic, only the constants.
"""
import json
import math
import os

import numpy as np
from scipy.optimize import brentq, least_squares
from scipy.special import gamma, gammaincinv

HERE = os.path.dirname(os.path.abspath(__file__))


def sersic_unit_flux(r, n):
    """Sersic surface brightness with half-light radius 1, normalised to unit total flux."""
    b = gammaincinv(2 * n, 0.5)
    z = 2 * math.pi * n * math.exp(b) * b ** (-2 * n) * gamma(2 * n)
    return np.exp(-b * (r ** (1.0 / n) - 1.0)) / z


def mog_iso(r, alpha, tau):
    return np.sum(alpha[:, None] * np.exp(-r[None, :] ** 2 / (2 * tau[:, None]))
                  / (2 * math.pi * tau[:, None]), axis=0)


def fit(n, k, rmax):
    r = np.geomspace(1e-3, rmax, 600)
    target = sersic_unit_flux(r, n)
    # weight by annulus area in log-radius (r^2 dlogr) so the fit tracks enclosed flux
    wts = r * np.sqrt(np.gradient(np.log(r)))
    init_tau = np.geomspace(1e-3 if n == 4 else 5e-3, 4.0 if n == 4 else 2.0, k)

    def resid(x):
        alpha = np.exp(x[:k])
        tau = np.exp(x[k:])
        return wts * (mog_iso(r, alpha, tau) - target) * 50.0

    x0 = np.concatenate([np.log(np.full(k, 1.0 / k)), np.log(init_tau)])
    sol = least_squares(resid, x0, method="lm", max_nfev=200000, xtol=1e-14, ftol=1e-14)
    alpha = np.exp(sol.x[:k])
    tau = np.exp(sol.x[k:])
    order = np.argsort(tau)
    alpha, tau = alpha[order], tau[order]
    alpha = alpha / alpha.sum()

    # half-light radius of an isotropic mixture: sum_j alpha_j exp(-R^2 / (2 tau_j)) = 1/2
    def light_outside(scale):
        return np.sum(alpha * np.exp(-1.0 / (2 * tau * scale))) - 0.5

    scale = brentq(light_outside, 1e-3, 1e3, xtol=1e-15, rtol=1e-15)
    tau = tau * scale
    return alpha, tau


def main():
    exp_a, exp_t = fit(1, 6, 8.0)
    dev_a, dev_t = fit(4, 8, 8.0)
    out = {
        "comment": "Isotropic Gaussian-mixture approximations of Sersic n=1 (exp) and n=4 (dev) "
                   "profiles with half-light radius 1; sum(alpha)=1. Written by synth/fit_profiles.py.",
        "exp": {"alpha": exp_a.tolist(), "tau": exp_t.tolist()},
        "dev": {"alpha": dev_a.tolist(), "tau": dev_t.tolist()},
    }
    with open(os.path.join(HERE, "profiles.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
