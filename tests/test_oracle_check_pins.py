"""CPU pins of the oracle's double-integrator lazy check and of its CSR transpose.

The double-integrator check (Algorithm 1's lazy check of the one chosen edge;
Section V-A's double integrator) tests the optimal trajectory at the times
t_k = k tau/(K-1), k = 0..K-1: a point inside a closed box or outside the
closed workspace [0,1]^3 is a collision, and the two end points are the
states' own positions.  It is checked here against
  * an independent reference that evaluates the trajectory through the cubic
    Hermite basis (not the oracle's power-basis coefficients) on thousands of
    random edges, and
  * constructed edges whose decisions are fixed by exact values: boxes
    touching an end state (closed faces), boxes around each interior point
    and between consecutive points (the time grid), and the workspace faces.
The transpose that turns in-rows into out-rows (line 4 walks out-rows) is
checked against a numpy sort-based transpose.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_02403_amd import inputs as I


def hermite_points(py, vy, px, vx, tau, K):
    """Positions at t_k = k tau/(K-1) of the cubic with p(0)=py, p'(0)=vy,
    p(tau)=px, p'(tau)=vx, from the Hermite basis in s = t/tau."""
    s = np.arange(K, dtype=np.float64) / (K - 1)
    h00 = 2 * s ** 3 - 3 * s ** 2 + 1
    h10 = s ** 3 - 2 * s ** 2 + s
    h01 = -2 * s ** 3 + 3 * s ** 2
    h11 = s ** 3 - s ** 2
    P = (h00[:, None] * py[None, :] + (h10 * tau)[:, None] * vy[None, :]
         + h01[:, None] * px[None, :] + (h11 * tau)[:, None] * vx[None, :])
    P[0], P[-1] = py, px
    return P


def ref_check(P, boxes):
    """(free, margin): collision when a point leaves [0,1]^3 or lies in a
    closed box; margin is the least distance of any point from deciding
    otherwise (L-inf, position units)."""
    out = np.max(np.maximum(-P, P - 1.0), axis=1)  # > 0 outside the workspace
    hit = bool(np.any(out > 0))
    margin = float(np.min(np.abs(out)))
    for b in boxes.astype(np.float64):
        lo, hi = b[:3], b[3:]
        sd = np.max(np.maximum(lo[None, :] - P, P - hi[None, :]), axis=1)  # <= 0 inside
        hit |= bool(np.any(sd <= 0))
        margin = min(margin, float(np.min(np.abs(sd))))
    return not hit, margin


def di_prob(samples, x_init, boxes, K=16):
    return I.Problem(kind="di", dim=6, pdim=3, samples=np.ascontiguousarray(samples, np.float32),
                     x_init=np.asarray(x_init, np.float32), goal_center=np.array([0.95] * 3, np.float32),
                     goal_radius=0.05, boxes=np.ascontiguousarray(boxes, np.float32).reshape(-1, 6),
                     lam=0.5, traj_points=K, r=2.0)


def test_di_check_matches_hermite_reference_on_random_edges():
    """>= 2000 random edges against 40 random boxes each (plus box-free and
    dense variants); every decision whose margin exceeds FP64 rounding agrees."""
    s = I.di_samples(3, 512)
    X = s.astype(np.float64).T
    rng = np.random.default_rng(5)
    compared, hits = 0, 0
    for w in range(8):
        m = (0, 40, 120, 40)[w % 4]
        boxes = []
        for _ in range(m):
            side = rng.uniform(0.05, 0.2, size=3)
            lo = rng.uniform(0, 1 - side)
            boxes.append(np.concatenate([lo, lo + side]))
        boxes = I.from_grid(I.to_grid(np.array(boxes).reshape(-1, 6)))
        prob = di_prob(s, s[:, 0], boxes)
        for _ in range(300):
            y, x = rng.integers(0, s.shape[1], size=2)
            if y == x:
                continue
            J, tau = O.di_cost(X[y], X[x])
            P = hermite_points(X[y, :3], X[y, 3:], X[x, :3], X[x, 3:], tau, 16)
            want, margin = ref_check(P, boxes)
            if margin <= 1e-9:
                continue
            got, _ = O.edge_free(prob, int(y), int(x), tau)
            assert got == want, (w, y, x)
            compared += 1
            hits += int(not want)
    assert compared >= 2000
    assert 0.1 * compared < hits < 0.9 * compared  # both outcomes well represented


def straight_edge(K):
    """Rest-to-rest edge along x from (0.25, .5, .5) to (0.5, .5, .5): the
    trajectory is p0 + a (3 s^2 - 2 s^3), exact positions known in closed form."""
    y = np.array([0.25, 0.5, 0.5, 0, 0, 0], np.float32)
    x = np.array([0.5, 0.5, 0.5, 0, 0, 0], np.float32)
    s = np.stack([y, x], axis=1)  # samples 0 (y) and 1 (x)
    J, tau = O.di_cost(y.astype(np.float64), x.astype(np.float64))
    assert tau == pytest.approx(np.sqrt(6 * 0.25), rel=1e-12)  # rest-to-rest closed form
    sk = np.arange(K) / (K - 1)
    xs = 0.25 + 0.25 * (3 * sk ** 2 - 2 * sk ** 3)
    return s, tau, xs


def box_x(lo, hi):
    return np.array([[lo, 0.4, 0.4, hi, 0.6, 0.6]])


@pytest.mark.parametrize("K", [5, 16])
def test_di_check_time_grid_and_closed_boxes(K):
    s, tau, xs = straight_edge(K)
    g = 2.0 ** -20
    root = s[:, 0]

    def free(boxes):
        prob = di_prob(s, root, I.from_grid(I.to_grid(boxes)) if boxes.size else boxes, K)
        return O.edge_free(prob, 0, 1, tau)[0]

    assert free(np.zeros((0, 6)))
    # closed faces at the two end states: touching either end is a collision
    assert not free(box_x(0.5, 0.6))
    assert not free(box_x(0.1, 0.25))
    assert free(box_x(0.5 + g, 0.6))
    assert free(box_x(0.1, 0.25 - g))
    # a thin box around each interior point is hit; one strictly between two
    # consecutive points is not (only the K points are tested)
    for k in range(1, K - 1):
        prob_hit = di_prob(s, root, box_x(xs[k] - 1e-6, xs[k] + 1e-6), K)
        assert not O.edge_free(prob_hit, 0, 1, tau)[0], k
        a, b = xs[k] + 1e-6, xs[k + 1] - 1e-6
        prob_gap = di_prob(s, root, box_x(a, b), K)
        assert O.edge_free(prob_gap, 0, 1, tau)[0], k


def test_di_check_workspace_bound_is_closed():
    """End states exactly on the faces of [0,1]^3 are inside the workspace;
    a trajectory that overshoots a face between its points collides, and the
    same manoeuvre shifted into the cube does not."""
    y = np.array([0.0, 0.5, 0.5, 0, 0, 0], np.float32)
    x = np.array([1.0, 0.5, 0.5, 0, 0, 0], np.float32)
    s = np.stack([y, x], axis=1)
    J, tau = O.di_cost(y.astype(np.float64), x.astype(np.float64))
    assert O.edge_free(di_prob(s, y, np.zeros((0, 6))), 0, 1, tau)[0]
    # leave at rest, arrive with velocity -1 (resp. +1): the cubic first runs
    # past the arrival point, by ~0.31 in position -- beyond x = 1 (resp. 0)
    # near the upper (lower) face, inside the cube from the middle
    for py, px, vx, free in [(0.9, 0.98, -1.0, False), (0.1, 0.02, 1.0, False), (0.5, 0.58, -1.0, True)]:
        yy = np.array([py, 0.5, 0.5, 0.0, 0, 0], np.float32)
        xx = np.array([px, 0.5, 0.5, vx, 0, 0], np.float32)
        J2, tau2 = O.di_cost(yy.astype(np.float64), xx.astype(np.float64))
        P = hermite_points(yy[:3].astype(np.float64), yy[3:].astype(np.float64),
                           xx[:3].astype(np.float64), xx[3:].astype(np.float64), tau2, 16)
        want, margin = ref_check(P, np.zeros((0, 6)))
        assert want == free and margin > 1e-3
        assert O.edge_free(di_prob(np.stack([yy, xx], axis=1), yy, np.zeros((0, 6))), 0, 1, tau2)[0] == free


def np_transpose(n, rp, col):
    src = np.repeat(np.arange(n), np.diff(rp))
    order = np.lexsort((src, col))
    out_col = src[order]
    out_ptr = np.concatenate([[0], np.cumsum(np.bincount(col, minlength=n))])
    return out_ptr, out_col


@pytest.mark.parametrize("n,deg,seed", [(1, 0, 0), (7, 3, 1), (500, 40, 2), (4096, 9, 3)])
def test_transpose_matches_sort_based_transpose(n, deg, seed):
    rng = np.random.default_rng(seed)
    rows = []
    for x in range(n):
        k = int(rng.integers(0, deg + 1)) if n > 1 else 0
        cand = np.setdiff1d(rng.choice(n, size=min(k, n), replace=False), [x])
        rows.append(np.sort(cand))
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    col = (np.concatenate(rows) if rp[-1] else np.zeros(0)).astype(np.int32)
    op, oc = O.transpose(n, rp, col)
    wp, wc = np_transpose(n, rp, col)
    np.testing.assert_array_equal(op, wp)
    np.testing.assert_array_equal(oc, wc)


def test_transpose_of_di_table_gives_out_neighbours():
    """Out-row y of the transposed DI table lists exactly the x with
    c(y -> x) < r, ascending (the out-neighbour set line 4 walks)."""
    s = I.di_samples(4, 300)
    r = 2.4
    tab = O.neighbors(s, O.DI, r)
    op, oc = O.transpose(s.shape[1], tab.row_ptr, tab.col)
    X = s.astype(np.float64).T
    for y in range(0, 300, 37):
        want = [x for x in range(300) if x != y and O.di_cost(X[y], X[x])[0] < r]
        assert list(oc[op[y]:op[y + 1]]) == want
