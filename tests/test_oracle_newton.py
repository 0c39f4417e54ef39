"""Pins of the oracle's trust-region subproblem, Newton step, colouring and sweep."""
import math

import numpy as np
import pytest

from oracle import elbo as E
from oracle import newton as NW
from synth import gen


def _rand_sym(rng, n, shift=0.0):
    A = rng.normal(size=(n, n))
    return 0.5 * (A + A.T) + shift * np.eye(n)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("delta", [0.05, 1.0, 30.0])
def test_tr_kkt(seed, delta):
    """Nocedal & Wright Theorem 4.1 conditions for the returned step (Section 4.3's
    Euclidean-ball trust region)."""
    rng = np.random.default_rng(seed)
    n = 27
    H = _rand_sym(rng, n, shift=-3.0 if seed % 2 else 0.0)
    g = rng.normal(size=n)
    p, lam, hard = NW.tr_subproblem(g, H, delta)
    B = -H
    assert lam >= 0
    assert np.linalg.norm(p) <= delta * (1 + 1e-10)
    assert np.linalg.norm((B + lam * np.eye(n)) @ p - g) <= 1e-9 * max(1, np.linalg.norm(g))
    assert lam * (delta - np.linalg.norm(p)) <= 1e-8 * max(1, lam * delta)
    assert np.linalg.eigvalsh(B + lam * np.eye(n)).min() >= -1e-9


def test_tr_interior_is_newton_step():
    """Concave model with a large radius: the step is the Newton step -H^{-1} g."""
    rng = np.random.default_rng(2)
    X = rng.normal(size=(27, 27))
    H = -(X @ X.T + np.eye(27))
    g = rng.normal(size=27)
    p, lam, _ = NW.tr_subproblem(g, H, 1e6)
    assert lam == 0.0
    assert np.allclose(p, -np.linalg.solve(H, g), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_tr_2d_brute_force(seed):
    """2-D subproblems against a brute-force maximum over a polar grid of the disk."""
    rng = np.random.default_rng(100 + seed)
    H = _rand_sym(rng, 2)
    g = rng.normal(size=2)
    delta = 0.7
    p, _, _ = NW.tr_subproblem(g, H, delta)
    model = lambda P: P @ g + 0.5 * np.einsum("ni,ij,nj->n", P, H, P)
    r = np.linspace(0, delta, 1001)
    t = np.linspace(0, 2 * math.pi, 2001)
    R, T = np.meshgrid(r, t)
    P = np.stack([(R * np.cos(T)).ravel(), (R * np.sin(T)).ravel()], 1)
    best = model(P).max()
    got = model(p[None])[0]
    assert got >= best - 1e-9
    assert got - best <= 1e-4 * max(1, abs(best))


def test_tr_hard_case():
    """g orthogonal to the lowest eigenvector of -H with a radius larger than the
    restricted Newton step: the step reaches the boundary along that eigenvector,
    oriented so its largest entry is positive."""
    Q = np.linalg.qr(np.random.default_rng(4).normal(size=(5, 5)))[0]
    lam = np.array([-2.0, 1.0, 2.0, 3.0, 4.0])
    B = Q @ np.diag(lam) @ Q.T
    g = Q[:, 1:] @ np.array([0.3, -0.2, 0.1, 0.05])
    delta = 3.0
    p, l, hard = NW.tr_subproblem(g, -B, delta)
    assert hard and abs(l - 2.0) < 1e-12
    assert abs(np.linalg.norm(p) - delta) < 1e-10
    q0 = Q[:, 0] if Q[np.argmax(np.abs(Q[:, 0])), 0] > 0 else -Q[:, 0]
    assert p @ q0 > 0
    # model value equals the best over +-q0 completions
    model = lambda P: P @ g - 0.5 * P @ B @ P
    alt = p - 2 * (p @ q0) * q0
    assert abs(model(p) - model(alt)) < 1e-9


def _tiny(n_sources=6, side=18, images=(0, 2, 5)):
    return gen.crop_patches(gen.subset(gen.config2(n_sources=n_sources), images=list(images)), side)


def test_colouring_separates_overlapping_sources():
    prob = _tiny(12)
    m = E.Model(prob)
    adj = NW.overlap_graph(m)
    col = NW.greedy_colouring(adj)
    groups = prob.truth["group"]
    for s in range(prob.n_sources):
        for t in adj[s]:
            assert col[s] != col[t]
            assert groups[s] == groups[t]           # groups never touch
        assert col[s] == min(set(range(len(adj) + 1)) - {col[t] for t in adj[s] if t < s})


def test_newton_step_parallel_equals_serial_and_increases_objective():
    """Sources of one colour class do not overlap, so stepping them from the same iterate
    equals stepping them one after another (Section 4.4).  Accepted steps never decrease
    L_s (Section 4.3)."""
    prob = _tiny(8)
    m = E.Model(prob)
    col = NW.greedy_colouring(NW.overlap_graph(m))
    mask = col == 0
    assert mask.sum() >= 2
    radius = np.full(prob.n_sources, 1.0)
    th_par, r_par, st_par, loc_par = NW.newton_step(m, prob.theta0, radius, mask)
    th_ser = prob.theta0.copy()
    r_ser = radius.copy()
    for s in np.nonzero(mask)[0]:
        th_ser[s], r_ser[s], st, loc = NW.newton_step_source(m, th_ser, s, r_ser[s])
        assert st == st_par[s] and loc == loc_par[s]
    assert np.array_equal(th_ser, th_par) and np.array_equal(r_ser, r_par)
    before = E.elbo(m, prob.theta0, sources=list(np.nonzero(mask)[0]), with_total=False)[1].numpy()
    for s in np.nonzero(mask)[0]:
        if st_par[s] == NW.ST_ACCEPTED:
            assert loc_par[s] > before[s]
    assert not mask[~mask].any()
    assert np.array_equal(th_par[~mask], prob.theta0[~mask])


@pytest.mark.slow
def test_isolated_source_converges_in_one_sweep():
    """For a source overlapping no other, one subsolver call reaches a local maximum
    (Section 4.3): a second sweep does not move it, and Newton needs at most tens of
    iterations."""
    full = gen.config2(n_sources=6)
    # a single source taken out of its group has no neighbour in the sub-problem
    prob = gen.crop_patches(gen.subset(full, sources=[0], images=[1, 2]), 20)
    m = E.Model(prob)
    th1, _, st1, rep1 = NW.sweep(m, prob.theta0, dict(n_sweeps=1))
    assert rep1["iters"][0] <= 50
    th2, _, st2, rep2 = NW.sweep(m, th1, dict(n_sweeps=1))
    assert np.abs(th2 - th1).max() < 1e-3
    assert rep2["elbo"] >= rep1["elbo"] - 1e-9 * abs(rep1["elbo"])
    assert rep1["elbo"] > E.elbo(m, prob.theta0)[0].item()
