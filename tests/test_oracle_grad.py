"""Pins of the oracle's gradient and of structural invariants of the objective."""
import math

import numpy as np
import pytest
import torch

from oracle import elbo as E
from synth import gen


@pytest.fixture(scope="module")
def c1():
    p = gen.config1()
    return p, E.Model(p)


def test_gradient_matches_central_differences(c1):
    """Central finite differences (h = 1e-4) of the float64 global ELBO against the reverse-
    mode gradient, every used coordinate of both sources; FD truncation ~h^2."""
    prob, m = c1
    th = prob.theta0.copy()
    _, _, g = E.elbo_total_and_grad(m, th)
    h = 1e-4
    for s in range(2):
        for k in range(E.N_PARAM):
            tp, tm = th.copy(), th.copy()
            tp[s, k] += h
            tm[s, k] -= h
            fd = (E.elbo(m, tp)[0].item() - E.elbo(m, tm)[0].item()) / (2 * h)
            assert abs(fd - g[s, k]) <= 1e-6 * max(1.0, abs(g[s, k])), (s, k, fd, g[s, k])
    assert np.all(g[:, E.N_PARAM:] == 0)


def test_local_gradient_equals_global_gradient():
    """dL/dtheta_s = dL_s/dtheta_s: pixels outside s's patches and other sources' KL do not
    depend on theta_s (the objective is a sum over pixels and sources, Section 4.4)."""
    prob = gen.crop_patches(gen.subset(gen.config2(n_sources=8), images=[0, 1, 7]), 24)
    m = E.Model(prob)
    _, loc, g = E.elbo_total_and_grad(m, prob.theta0)
    for s in range(prob.n_sources):
        v, gs = E.local_value_grad(m, prob.theta0, s)
        assert abs(v - loc[s]) <= 1e-12 * abs(v)
        assert np.allclose(gs, g[s, :E.N_PARAM], rtol=1e-10, atol=1e-9)


def test_hessian_symmetric_and_matches_fd_of_gradient(c1):
    """The forward-over-reverse Hessian is symmetric and equals central differences of the
    gradient (h = 1e-4)."""
    prob, m = c1
    s = 1
    H = E.local_hessian(m, prob.theta0, s)
    assert np.abs(H - H.T).max() <= 1e-9 * np.abs(H).max()
    h = 1e-4
    for k in (0, 2, 3, 9, 16, 23, 24, 25, 26):
        tp, tm = prob.theta0.copy(), prob.theta0.copy()
        tp[s, k] += h
        tm[s, k] -= h
        col = (E.local_value_grad(m, tp, s)[1] - E.local_value_grad(m, tm, s)[1]) / (2 * h)
        assert np.allclose(col, H[:, k], rtol=1e-5, atol=1e-5 * np.abs(H).max())


def test_relabelling_sources_leaves_elbo_unchanged():
    """The global ELBO is a sum over sources and pixels: permuting source ids changes only
    the summation order."""
    prob = gen.crop_patches(gen.subset(gen.config2(n_sources=9), images=[2, 6]), 30)
    m = E.Model(prob)
    tot = E.elbo(m, prob.theta0)[0].item()
    perm = np.random.default_rng(1).permutation(prob.n_sources)
    # build the permuted problem: new id k is old source perm[k]
    import copy
    q = copy.copy(prob)
    inv = np.argsort(perm)
    q.patch_src = inv[prob.patch_src].astype(np.int32)
    order = np.lexsort((prob.patch_img, q.patch_src))
    for f in ("patch_src", "patch_img", "patch_x0", "patch_y0", "patch_w", "patch_h"):
        setattr(q, f, getattr(q if f == "patch_src" else prob, f)[order])
    sizes = q.patch_w.astype(np.int64) * q.patch_h
    q.patch_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    q.pixels = np.concatenate([prob.patch_pixels(p).ravel() for p in order]).astype(np.float32)
    q.theta0 = prob.theta0[perm]
    tq = E.elbo(E.Model(q), q.theta0)[0].item()
    assert abs(tq - tot) <= 1e-12 * abs(tot)


def test_translation_and_shape_invariances(c1):
    """Integer translation of sources and patches on a constant sky leaves the ELBO
    unchanged; angle + pi gives the same Sigma_s; a round galaxy (axis -> 1) has zero
    derivative with respect to the angle (Section 2.1.2)."""
    prob, m = c1
    th = prob.theta0.copy()
    base = E.elbo(m, th)[0].item()
    import copy
    q = copy.copy(prob)
    q.patch_x0 = prob.patch_x0 + 3
    q.patch_y0 = prob.patch_y0 - 2
    q.img_W = prob.img_W + 10
    q.img_H = prob.img_H + 10
    tq = th.copy()
    tq[:, 0] += 3
    tq[:, 1] -= 2
    assert abs(E.elbo(E.Model(q), tq)[0].item() - base) <= 1e-12 * abs(base)
    tr = th.copy()
    tr[1, 23] += math.pi
    assert abs(E.elbo(m, tr)[0].item() - base) <= 1e-12 * abs(base)
    tround = th.copy()
    tround[1, 26] = 40.0
    _, _, g = E.elbo_total_and_grad(m, tround)
    assert abs(g[1, 23]) <= 1e-9 * np.abs(g[1]).max()
