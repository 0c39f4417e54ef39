"""Regression pin: the oracle still produces the stored values on the 1-star + 1-galaxy
workload (values written by tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

from oracle import elbo as E
from synth import gen


def test_oracle_matches_stored_values():
    with open(os.path.join(os.path.dirname(__file__), "golden", "config1_oracle.json")) as f:
        ref = json.load(f)
    prob = gen.config1()
    total, local, grad = E.elbo_total_and_grad(E.Model(prob), prob.theta0)
    assert abs(total - ref["elbo_total"]) <= 1e-12 * abs(ref["elbo_total"])
    assert np.allclose(local, ref["elbo_local"], rtol=1e-12)
    assert np.allclose(grad, ref["grad"], rtol=1e-10, atol=1e-9)
