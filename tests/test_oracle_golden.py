"""Regression pins of the oracle against its own stored values (tests/golden/, written by
tests/golden/make_golden.py, which calls only the oracle and the generator), and checks
that the generator still produces the inputs those values were made from."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import elbo as E
from synth import gen
from tests.golden.inputs_hash import load_golden

HERE = os.path.join(os.path.dirname(__file__), "golden")


def test_oracle_matches_stored_values():
    with open(os.path.join(HERE, "config1_oracle.json")) as f:
        ref = json.load(f)
    prob = gen.config1()
    total, local, grad = E.elbo_total_and_grad(E.Model(prob), prob.theta0)
    assert abs(total - ref["elbo_total"]) <= 1e-12 * abs(ref["elbo_total"])
    assert np.allclose(local, ref["elbo_local"], rtol=1e-12)
    assert np.allclose(grad, ref["grad"], rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("k,name", [(2, "config2_oracle.npz"), (4, "config4_oracle.npz")])
def test_full_size_stored_values_reproduce(k, name):
    """The stored full-size values come from the current oracle on the current inputs: the
    hash of the generated inputs matches and three sampled sources' L_s and gradients are
    reproduced."""
    prob = gen.make_config(k)
    ref = load_golden(name, prob)
    m = E.Model(prob)
    torch.set_num_threads(4)
    for s in np.random.default_rng(k).choice(prob.n_sources, 3, replace=False):
        v, g = E.local_value_grad(m, prob.theta0, int(s))
        assert abs(v - ref["elbo_local"][s]) <= 1e-12 * abs(v)
        assert np.allclose(g, ref["grad"][s, :27], rtol=1e-10, atol=1e-8)
    assert np.all(ref["grad"][:, 27:] == 0)


def test_adjoint_stored_gradient_matches_its_central_differences():
    """The oracle's reverse-mode gradient on the 4096-source workload against its own central
    differences (h = 1e-4, float64) for 128 sources x 27 coordinates (Section 4.2's
    objective; the finite differences pin the derivative).  The truncation error is
    h^2 |d^3 L_s| / 6: on the flux means of bright sources, whose third derivative scales
    with the source's expected counts, it reaches 2e-6 of the gradient's scale (median
    4e-9); the rounding error eps |L_s| / h is below 1e-7.  Bound: 1e-5, ten times below
    the GPU's tolerance."""
    with np.load(os.path.join(HERE, "config3_oracle.npz"), allow_pickle=False) as z:
        g, fd, src = z["grad"], z["fd_grad"], z["fd_sources"]
    og = g[src, :27]
    floor = 0.01 * np.abs(og).max(axis=1, keepdims=True)
    err = np.abs(fd - og) / np.maximum(np.abs(og), floor)
    assert err.max() <= 1e-5, err.max()


def test_skew_sweep_stored_values_are_consistent():
    """The stored sweep of the skewed field was made from the current inputs, and its
    reported ELBO is the oracle's objective at its stored end point."""
    prob = gen.config_skew()
    ref = load_golden("skew_sweep.npz", prob)
    tot = E.elbo(E.Model(prob), ref["theta"])[0].item()
    assert abs(tot - float(ref["elbo"])) <= 1e-12 * abs(tot)
    assert tot > E.elbo(E.Model(prob), prob.theta0)[0].item()
