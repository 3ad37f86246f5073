"""CPU checks of the input generator and of the oracle on double-integrator runs."""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_02403_amd import inputs as I


def test_geometric_inputs_are_valid():
    for seed in range(3):
        p = I.problem_2d(seed)
        q = I.problem_3d(seed, n=4096)
        for prob in (p, q):
            assert I.on_grid(prob.samples) and I.on_grid(prob.boxes) and I.on_grid(prob.x_init)
            assert I.on_grid(prob.goal_center)
            s = I.to_grid(prob.samples.T)
            b = I.to_grid(prob.boxes)
            d = prob.dim
            assert not np.any(I._in_any_box(s, b))
            assert np.any(I._in_ball(s, I.to_grid(prob.goal_center), prob.goal_radius))
            assert not np.any(I._in_any_box(I.to_grid(prob.x_init)[None, :], b))
            for lo, hi in zip(b[:, :d], b[:, d:]):
                assert not I._box_touches_ball(lo, hi, I.to_grid(prob.goal_center), prob.goal_radius)
                assert np.all(lo >= 0) and np.all(hi <= I.QSCALE) and np.all(lo <= hi)
    a, b = I.problem_2d(5), I.problem_2d(5)
    assert np.array_equal(a.samples, b.samples) and np.array_equal(a.boxes, b.boxes)


def test_di_inputs_are_valid():
    s = I.di_samples(0, 4096)
    assert s.shape == (6, 4096) and I.on_grid(s)
    v = I.to_grid(s[3:].T)
    assert np.all(np.sum(v * v, axis=1) <= I.QSCALE ** 2)
    assert np.all(s[:3] >= 0) and np.all(s[:3] <= 1)
    p = I.di_problem(3, s)
    assert p.x_init.shape == (6,) and np.all(p.x_init[3:] == 0)
    assert np.all(np.abs(p.x_init[:3] - 0.05) <= 0.03 + 1e-6)
    assert np.any(I._in_ball(I.to_grid(s[:3].T), I.to_grid(p.goal_center), p.goal_radius))
    b = I.to_grid(p.boxes)
    assert not np.any(I._in_any_box(I.to_grid(p.x_init[:3])[None, :], b))


def test_clustered_samples_are_valid():
    for dim in (2, 3):
        s = I.clustered_samples(11, dim, 500, 0.05)
        assert s.shape == (dim, 500) and s.dtype == np.float32 and I.on_grid(s)
        assert np.all(s >= 0) and np.all(s <= 0.05)
    assert np.array_equal(I.clustered_samples(4, 3, 64, 0.1), I.clustered_samples(4, 3, 64, 0.1))


def test_poisson_stream_rate():
    t = I.poisson_arrivals(20000, 2000.0, seed=7)
    assert np.all(np.diff(t) > 0)
    assert abs(20000 / t[-1] - 2000.0) < 60.0


@pytest.mark.parametrize("seed,lam", [(0, 0.5), (1, 1.0), (2, 0.25)])
def test_di_tree_invariants(seed, lam):
    """Double-integrator run: each tree edge is a neighbour pair whose optimal
    trajectory passes the 16-point check, costs add up along edges, and the
    group index follows Algorithm 1 line 3."""
    s = I.di_samples(1, 2048)
    prob = I.di_problem(seed, s, lam=lam, r=2.4)
    tab = O.neighbors(s, O.DI, prob.r)
    a = O.plan(prob, prob.r, tab)
    n = prob.n
    X = np.concatenate([s.astype(np.float64).T, prob.x_init.astype(np.float64)[None, :]])
    inn = np.nonzero(a.parent >= 0)[0]
    assert len(inn) > 50
    for x in inn:
        y = int(a.parent[x])
        J, tau = O.di_cost(X[y], X[x])
        assert J < prob.r
        assert a.cost[x] == pytest.approx(a.cost[y] + J, rel=1e-12, abs=0)
        ok, _ = O.edge_free(prob, y, int(x), tau)
        assert ok
    delta = lam * prob.r
    for x in np.nonzero(a.group_iter >= 0)[0]:
        if x == n:
            continue
        i = a.added_iter[x] + 1
        while not (a.cost[x] <= i * delta):
            i += 1
        assert a.group_iter[x] == i
    if a.status == O.OK:
        assert a.path_cost <= a.iters * delta
        assert a.path[0] == n


def test_di_lambda0_never_beats_dijkstra():
    s = I.di_samples(2, 1024)
    prob = I.di_problem(4, s, lam=0.0, r=2.6)
    tab = O.neighbors(s, O.DI, prob.r)
    a = O.plan(prob, prob.r, tab)
    d = O.dijkstra(prob, prob.r, tab)
    inn = np.isfinite(a.cost)
    assert np.all(a.cost[inn] >= d[inn] * (1 - 1e-12))
