"""Pins of the oracle's Dubins airplane cost (Section V-A: a planar Dubins
car with an altitude single integrator, bounded turning rate, Euclidean
length cost) against facts fixed outside the oracle's code:

* closed forms: a straight run, a quarter turn, a U-turn, a pure climb;
* symmetries of the problem: reversing a path (headings turned by pi),
  mirroring the plane (left and right swap), rigid motions;
* the path reaches the goal pose (forward kinematics written here, as
  complex exponentials);
* brute force: for each of the six word families, every path found by
  numeric root finding of its end-pose equations from a grid of starts is at
  least as long as the oracle's, and the shortest found equals it;
* length >= straight-line distance; cost = sqrt(planar^2 + climb^2);
* the lazy check: constructed edges whose points (taken from the forward
  kinematics here) enter a trunk, graze it, or leave the unit cube.
"""

import math

import numpy as np
import pytest
from scipy.optimize import least_squares

from oracle import oracle as O

RHO = 0.05


def turns(theta):
    return (theta / (2 * math.pi)) % 1.0


def state(x, y, z, theta):
    return np.array([x, y, z, turns(theta)])


def walk(x0, y0, th0, word, seg, s=None, rho=RHO):
    """Forward kinematics: pose after planar arc length s (default: all)."""
    z = complex(x0, y0)
    th = th0
    left = sum(seg) if s is None else s
    for d, l in zip(word, seg):
        l = min(l, left)
        if l <= 0:
            continue
        if d == 0:
            z += l * np.exp(1j * th)
        else:
            th2 = th + d * l / rho
            z += d * rho * 1j * (np.exp(1j * th) - np.exp(1j * th2))
            th = th2
        left -= l
    return z.real, z.imag, th


def planar(x0, x1):
    return O.dubins_cost(x0, x1, RHO)[1]


def test_closed_forms():
    D = 0.2
    c, pl, w, sg = O.dubins_cost(state(0.1, 0.1, 0.5, 0.0), state(0.1 + D, 0.1, 0.5, 0.0), RHO)
    assert abs(pl - D) < 1e-12 and abs(c - D) < 1e-12
    # quarter turn to the left: end at (rho, rho) heading +y
    pl = planar(state(0.2, 0.2, 0.5, 0.0), state(0.2 + RHO, 0.2 + RHO, 0.5, math.pi / 2))
    assert abs(pl - math.pi * RHO / 2) < 1e-12
    # U-turn: end 2 rho to the left, heading reversed
    pl = planar(state(0.3, 0.3, 0.5, 0.0), state(0.3, 0.3 + 2 * RHO, 0.5, math.pi))
    assert abs(pl - math.pi * RHO) < 1e-12
    # climb on a straight run: the cost is the 3D segment length
    c, pl, _, _ = O.dubins_cost(state(0.1, 0.5, 0.1, 0.0), state(0.4, 0.5, 0.5, 0.0), RHO)
    assert abs(pl - 0.3) < 1e-12 and abs(c - 0.5) < 1e-12


def random_pairs(count, seed=0, span=0.4):
    rng = np.random.default_rng(seed)
    a = np.column_stack([rng.uniform(0.3, 0.7, (count, 3)), rng.uniform(0, 1, count)])
    b = a.copy()
    b[:, :3] += rng.uniform(-span / 2, span / 2, (count, 3))
    b[:, 3] = rng.uniform(0, 1, count)
    return a, b


def test_arrival_and_lower_bounds():
    a, b = random_pairs(300)
    for x0, x1 in zip(a, b):
        c, pl, w, sg = O.dubins_cost(x0, x1, RHO)
        x, y, th = walk(x0[0], x0[1], 2 * math.pi * x0[3], w, sg)
        assert abs(x - x1[0]) < 1e-9 and abs(y - x1[1]) < 1e-9
        dth = (th - 2 * math.pi * x1[3]) % (2 * math.pi)
        assert min(dth, 2 * math.pi - dth) < 1e-9
        assert abs(pl - sum(sg)) < 1e-12 and all(v >= 0 for v in sg)
        assert pl >= math.hypot(x1[0] - x0[0], x1[1] - x0[1]) - 1e-12
        assert abs(c - math.hypot(pl, x1[2] - x0[2])) <= 1e-12 * c
        assert c >= np.linalg.norm(x1[:3] - x0[:3]) - 1e-12


def test_symmetries():
    a, b = random_pairs(200, seed=1)
    rng = np.random.default_rng(5)
    for x0, x1 in zip(a, b):
        L = planar(x0, x1)
        # reversal: the path flown backwards joins the reversed headings
        r0 = x1.copy(); r0[3] = (x1[3] + 0.5) % 1.0
        r1 = x0.copy(); r1[3] = (x0[3] + 0.5) % 1.0
        assert abs(planar(r0, r1) - L) < 1e-9
        # mirror y -> 1 - y, theta -> -theta
        m0 = x0.copy(); m0[1] = 1 - x0[1]; m0[3] = (-x0[3]) % 1.0
        m1 = x1.copy(); m1[1] = 1 - x1[1]; m1[3] = (-x1[3]) % 1.0
        assert abs(planar(m0, m1) - L) < 1e-9
        # rotation about (0.5, 0.5) and a translation
        phi = rng.uniform(0, 2 * math.pi)
        t = rng.uniform(-0.1, 0.1, 2)
        def move(x):
            z = complex(x[0] - 0.5, x[1] - 0.5) * np.exp(1j * phi)
            return np.array([z.real + 0.5 + t[0], z.imag + 0.5 + t[1], x[2], (x[3] + phi / (2 * math.pi)) % 1.0])
        assert abs(planar(move(x0), move(x1)) - L) < 1e-9


WORDS = [(1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (1, -1, 1), (-1, 1, -1)]


def brute_force(x0, x1):
    """Shortest path among the six families found by root finding of the
    end-pose equations (unknowns: the three segment lengths)."""
    th0, th1 = 2 * math.pi * x0[3], 2 * math.pi * x1[3]
    best = math.inf
    for word in WORDS:
        hi = [2 * math.pi * RHO if d else 2.0 for d in word]

        def resid(l):
            x, y, th = walk(x0[0], x0[1], th0, word, l)
            return [x - x1[0], y - x1[1], RHO * (math.cos(th) - math.cos(th1)), RHO * (math.sin(th) - math.sin(th1))]
        for g in np.linspace(0.1, 0.9, 3):
            for h in np.linspace(0.1, 0.9, 3):
                for k in np.linspace(0.1, 0.9, 3):
                    start = [g * hi[0], h * hi[1], k * hi[2]]
                    sol = least_squares(resid, start, bounds=([0, 0, 0], hi), xtol=1e-15, ftol=1e-15, gtol=1e-15)
                    if np.max(np.abs(sol.fun)) < 1e-10:
                        best = min(best, float(np.sum(sol.x)))
    return best


def test_brute_force_shortest():
    a, b = random_pairs(12, seed=3, span=0.25)
    # include configurations where the turning words matter (close and behind)
    a = np.vstack([a, [0.5, 0.5, 0.5, 0.0], [0.5, 0.5, 0.5, 0.25]])
    b = np.vstack([b, [0.48, 0.52, 0.5, 0.5], [0.55, 0.45, 0.5, 0.8]])
    for x0, x1 in zip(a, b):
        L = planar(x0, x1)
        bf = brute_force(x0, x1)
        assert L <= bf + 1e-9, (x0, x1, L, bf)
        assert abs(L - bf) < 1e-8, (x0, x1, L, bf)


def dubins_prob(samples, boxes, step=0.005):
    from paper_1705_02403_amd import inputs as I
    s = np.ascontiguousarray(np.asarray(samples, np.float32).T)
    return I.Problem(kind="dubins", dim=4, pdim=3, samples=s, x_init=s[:, 0].copy(),
                     goal_center=np.zeros(3, np.float32), goal_radius=0.05,
                     boxes=np.asarray(boxes, np.float32).reshape(-1, 6), lam=0.5, step=step, r=0.3,
                     turn_radius=RHO)


def grid(v):
    return np.rint(np.asarray(v, np.float64) * (1 << 20)) / (1 << 20)


def test_lazy_check_constructed():
    # straight run along x at y = z = 0.5 from 0.2 to 0.4537 (L / step is
    # not an integer, so the point count is not a rounding decision)
    a = grid([0.2, 0.5, 0.5, 0.0])
    b = grid([0.4537, 0.5, 0.5, 0.0])
    trunk = grid([0.3, 0.49, 0.0, 0.31, 0.51, 0.8])
    p = dubins_prob([a, b], [trunk])
    ok, mg = O.edge_free(p, 0, 1)
    assert not ok and mg > 0
    # the trunk stops just below the flight level: free, clearance = the gap
    low = grid([0.3, 0.49, 0.0, 0.31, 0.51, 0.5 - 2 ** -10])
    ok, mg = O.edge_free(dubins_prob([a, b], [low]), 0, 1)
    assert ok and abs(mg - 2 ** -10) < 1e-9
    # with L / step an integer the margin reports the point-count boundary
    ok, mg = O.edge_free(dubins_prob([a, grid([0.45, 0.5, 0.5, 0.0])], [trunk]), 0, 1)
    assert not ok and mg == 0.0
    # a trunk thinner than the point spacing between two points is missed,
    # one that covers a point is hit: points at multiples of L/(K-1)
    L = float(b[0] - a[0])
    K = math.ceil(L / 0.005) + 1
    xs = [a[0] + k * L / (K - 1) for k in range(K)]
    thin = grid([xs[10] + 0.001, 0.49, 0.0, xs[10] + 0.002, 0.51, 0.8])
    assert O.edge_free(dubins_prob([a, b], [thin]), 0, 1)[0]
    on = grid([xs[10] - 0.0001, 0.49, 0.0, xs[10] + 0.0001, 0.51, 0.8])
    assert not O.edge_free(dubins_prob([a, b], [on]), 0, 1)[0]
    # a U-turn (right circle of centre (0.03, 0.45)) from near the wall at
    # x = 0 swings to x = -0.02: it leaves the cube
    u0 = grid([0.03, 0.4, 0.5, 0.5])  # heading -x
    u1 = grid([0.03, 0.4 + 2 * RHO, 0.5, 0.0])
    ok, mg = O.edge_free(dubins_prob([u0, u1], []), 0, 1)
    c, pl, w, sg = O.dubins_cost(u0, u1, RHO)
    xmin = min(walk(u0[0], u0[1], math.pi, w, sg, s)[0] for s in np.linspace(0, pl, 400))
    assert xmin < 0.0 and not ok
    # every point of a curved edge agrees with the forward kinematics
    c0 = grid([0.3, 0.3, 0.2, 0.1])
    c1 = grid([0.42, 0.36, 0.3, 0.6])
    c, pl, w, sg = O.dubins_cost(c0, c1, RHO)
    K = math.ceil(c / 0.005) + 1
    for k in range(1, K - 1):
        pt = O.dubins_point(c0, c1, k, K, RHO)
        x, y, _ = walk(c0[0], c0[1], 2 * math.pi * c0[3], w, sg, pl * k / (K - 1))
        assert abs(pt[0] - x) < 1e-12 and abs(pt[1] - y) < 1e-12
        assert abs(pt[2] - (c0[2] + (c1[2] - c0[2]) * k / (K - 1))) < 1e-15
