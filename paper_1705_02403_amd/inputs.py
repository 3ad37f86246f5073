"""Seeded synthetic planning problems.

This module only draws inputs; it holds none of the planner's arithmetic (no
costs, radii, neighbour tests or collision checks along edges).  Both the HIP
library and the CPU oracle are fed from here.

Every coordinate is a multiple of 2^-20 (``QSCALE``), which FP32 represents
exactly on [-1, 1]; the planner's Euclidean distances, goal tests and box
tests are then exact integer arithmetic on both sides.

State spaces (Section II, Problem 1; Section V-A for the double integrator):

* ``euclid``: X = [0,1]^d, d in {2, 3}; boxes and samples live in all d dims.
* ``di``: 6D double integrator, position in [0,1]^3 and velocity in the unit
  ball; boxes and the goal ball constrain the 3 position dims only.

Box worlds follow the workloads' recipe: per box and per axis a side
U[smin, smax] and a lower corner U[0, 1-side]; a box containing the start or
touching the closed goal ball is redrawn.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

QBITS = 20
QSCALE = 1 << QBITS  # grid units per unit length


def to_grid(x) -> np.ndarray:
    """Float coordinates -> int64 grid units (round to nearest)."""
    return np.rint(np.asarray(x, dtype=np.float64) * QSCALE).astype(np.int64)


def from_grid(k) -> np.ndarray:
    """int64 grid units -> FP32 coordinates (exact)."""
    return (np.asarray(k, dtype=np.float64) / QSCALE).astype(np.float32)


def on_grid(x) -> bool:
    """True when every value is an exact multiple of 2^-20."""
    a = np.asarray(x, dtype=np.float64) * QSCALE
    return bool(np.all(a == np.rint(a)))


@dataclasses.dataclass
class Problem:
    """One planning query (Problem 1): sample set, start, goal ball, boxes.

    ``samples`` is SoA FP32 ``[dim][n]``; ``boxes`` is FP32 ``[m][2*pdim]`` with
    the lower corner first.  ``goal_radius`` is an FP32 value held as a Python
    float.  ``r`` is set for workloads whose radius is a fixed constant (the
    double integrator); Euclidean workloads derive it from Theorem 1 with
    ``r_factor`` = (1+eta)^(1/d).
    """

    kind: str
    dim: int
    pdim: int
    samples: np.ndarray
    x_init: np.ndarray
    goal_center: np.ndarray
    goal_radius: float
    boxes: np.ndarray
    lam: float
    step: float = 0.0
    traj_points: int = 16
    r: Optional[float] = None
    r_factor: float = 1.1
    seed: int = 0
    sample_seed: int = 0
    turn_radius: float = 0.0  # Dubins airplane: least turning radius

    @property
    def n(self) -> int:
        return int(self.samples.shape[1])

    @property
    def m(self) -> int:
        return int(self.boxes.shape[0])

    def with_boxes(self, boxes: np.ndarray) -> "Problem":
        return dataclasses.replace(self, boxes=np.ascontiguousarray(boxes, np.float32))


# ---------------------------------------------------------------------------
# drawing helpers (grid units)
# ---------------------------------------------------------------------------

def _in_any_box(p_q: np.ndarray, boxes_q: np.ndarray) -> np.ndarray:
    """p_q [k, pd] int64, boxes_q [m, 2pd] int64 -> bool [k] (closed boxes)."""
    if boxes_q.shape[0] == 0:
        return np.zeros(p_q.shape[0], dtype=bool)
    pd = p_q.shape[1]
    lo = boxes_q[None, :, :pd]
    hi = boxes_q[None, :, pd:]
    p = p_q[:, None, :]
    inside = np.all((p >= lo) & (p <= hi), axis=2)
    return np.any(inside, axis=1)


def _in_ball(p_q: np.ndarray, c_q: np.ndarray, radius: float) -> np.ndarray:
    d = p_q - c_q[None, :]
    dd = np.sum(d * d, axis=1).astype(np.float64)
    rq = float(radius) * float(radius) * float(QSCALE) * float(QSCALE)
    return dd <= rq


def _box_touches_ball(lo: np.ndarray, hi: np.ndarray, c_q: np.ndarray, radius: float) -> bool:
    gap = np.maximum(np.maximum(lo - c_q, 0), c_q - hi)
    dd = float(np.sum(gap * gap))
    return dd <= float(radius) * float(radius) * float(QSCALE) * float(QSCALE)


def draw_boxes(rng: np.random.Generator, m: int, pdim: int, smin: float, smax: float,
               start_q: np.ndarray, goal_q: np.ndarray, goal_radius: float) -> np.ndarray:
    """m boxes (int64 grid units [m, 2*pdim]) avoiding the start and the goal ball.

    Each attempt draws the sides U[smin, smax] per axis, then the lower
    corner U[0, 1 - side] per axis (2*pdim uniform doubles from `rng`, in that
    order) and is rejected when the box contains the start or touches the goal
    ball.  Attempts are evaluated a block at a time; the generator is then
    left exactly where drawing the accepted attempts one by one leaves it."""
    if m <= 0:
        return np.zeros((0, 2 * pdim), dtype=np.int64)
    out = []
    have = 0
    lim = float(goal_radius) * float(goal_radius) * float(QSCALE) * float(QSCALE)
    while have < m:
        k = 2 * (m - have) + 8
        state = rng.bit_generator.state
        d = rng.random(2 * pdim * k).reshape(k, 2 * pdim)
        side = smin + (smax - smin) * d[:, :pdim]
        lo = (1.0 - side) * d[:, pdim:]
        lo_q = to_grid(lo)
        hi_q = np.minimum(to_grid(lo + side), QSCALE)
        holds_start = np.all((start_q[:pdim] >= lo_q) & (start_q[:pdim] <= hi_q), axis=1)
        gap = np.maximum(np.maximum(lo_q - goal_q, 0), goal_q - hi_q)
        touches = np.sum(gap * gap, axis=1).astype(np.float64) <= lim
        ok = np.flatnonzero(~holds_start & ~touches)[: m - have]
        used = int(ok[-1]) + 1 if len(ok) == m - have else k
        rng.bit_generator.state = state
        rng.random(2 * pdim * used)  # consume exactly the attempts made
        out.append(np.concatenate([lo_q[ok], hi_q[ok]], axis=1))
        have += len(ok)
    return np.concatenate(out).astype(np.int64)


def draw_positions(rng: np.random.Generator, k: int, pdim: int) -> np.ndarray:
    return rng.integers(0, QSCALE + 1, size=(k, pdim), dtype=np.int64)


def draw_velocities(rng: np.random.Generator, k: int) -> np.ndarray:
    """k velocities uniform in the closed unit ball (rejection from the cube)."""
    out = np.zeros((0, 3), dtype=np.int64)
    q2 = QSCALE * QSCALE
    while out.shape[0] < k:
        need = k - out.shape[0]
        v = rng.integers(-QSCALE, QSCALE + 1, size=(2 * need + 16, 3), dtype=np.int64)
        ok = np.sum(v * v, axis=1) <= q2
        out = np.concatenate([out, v[ok]])
    return out[:k]


def _ensure_goal_sample(rng, pos_q: np.ndarray, goal_q: np.ndarray, goal_radius: float,
                        boxes_q: Optional[np.ndarray]) -> None:
    """If no position lies in the closed goal ball, replace the last one by a draw
    from goal ball (and outside the boxes when given)."""
    if np.any(_in_ball(pos_q, goal_q, goal_radius)):
        return
    pd = pos_q.shape[1]
    rq = int(math.ceil(goal_radius * QSCALE))
    lo = np.maximum(goal_q - rq, 0)
    hi = np.minimum(goal_q + rq, QSCALE)
    while True:
        p = rng.integers(lo, hi + 1, size=(64, pd), dtype=np.int64)
        ok = _in_ball(p, goal_q, goal_radius)
        if boxes_q is not None:
            ok &= ~_in_any_box(p, boxes_q)
        if np.any(ok):
            pos_q[-1] = p[np.argmax(ok)]
            return


def draw_free_positions(rng, n: int, pdim: int, boxes_q: np.ndarray) -> np.ndarray:
    """n grid positions uniform in [0,1]^pdim minus the closed boxes."""
    out = np.zeros((0, pdim), dtype=np.int64)
    while out.shape[0] < n:
        need = n - out.shape[0]
        p = draw_positions(rng, int(need * 1.6) + 64, pdim)
        out = np.concatenate([out, p[~_in_any_box(p, boxes_q)]])
    return out[:n]


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def geometric_problem(seed: int, dim: int, n: int, m: int, smin: float, smax: float,
                      lam: float = 0.5, step: float = 0.005, goal_radius: float = 0.05,
                      r_factor: float = 1.1, start: float = 0.05, goal: float = 0.95) -> Problem:
    """Euclidean box world (the 2D / 3D workloads): samples rejected from boxes,
    start at (start,...), goal ball of radius 0.05 at (goal,...)."""
    rng = np.random.default_rng(seed)
    start_q = to_grid(np.full(dim, start))
    goal_q = to_grid(np.full(dim, goal))
    gr = float(np.float32(goal_radius))
    boxes_q = draw_boxes(rng, m, dim, smin, smax, start_q, goal_q, gr)
    pos_q = draw_free_positions(rng, n, dim, boxes_q)
    _ensure_goal_sample(rng, pos_q, goal_q, gr, boxes_q)
    return Problem(kind="euclid", dim=dim, pdim=dim,
                   samples=np.ascontiguousarray(from_grid(pos_q.T)),
                   x_init=from_grid(start_q), goal_center=from_grid(goal_q),
                   goal_radius=gr, boxes=np.ascontiguousarray(from_grid(boxes_q)),
                   lam=float(lam), step=float(step), r=None, r_factor=float(r_factor),
                   seed=int(seed), sample_seed=int(seed))


def problem_2d(seed: int, n: int = 2000, lam: float = 0.5) -> Problem:
    """2D geometric workload: 20 boxes, sides U[0.05, 0.15], step 0.005."""
    return geometric_problem(seed, 2, n, 20, 0.05, 0.15, lam=lam, step=0.005)


def problem_3d(seed: int, n: int = 16384, lam: float = 0.5) -> Problem:
    """3D geometric workload: 60 boxes, sides U[0.05, 0.2], step 0.002."""
    return geometric_problem(seed, 3, n, 60, 0.05, 0.2, lam=lam, step=0.002)


DI_RADIUS = 1.75          # connection radius of the double-integrator workload
DI_START = (0.05, 0.05, 0.05)
DI_GOAL = (0.95, 0.95, 0.95)


def di_samples(sample_seed: int, n: int, goal_radius: float = 0.05) -> np.ndarray:
    """SoA FP32 [6][n] double-integrator samples: position uniform in the unit
    cube, velocity uniform in the unit ball; at least one position in the goal
    ball.  Independent of any box world, so one sample set serves many queries."""
    rng = np.random.default_rng(10_000_019 + int(sample_seed))
    pos = draw_positions(rng, n, 3)
    vel = draw_velocities(rng, n)
    gr = float(np.float32(goal_radius))
    _ensure_goal_sample(rng, pos, to_grid(np.array(DI_GOAL)), gr, None)
    return np.ascontiguousarray(from_grid(np.concatenate([pos, vel], axis=1).T))


def di_problem(seed: int, samples: np.ndarray, m: int = 40, smin: float = 0.05, smax: float = 0.2,
               lam: float = 0.5, r: float = DI_RADIUS, jitter: float = 0.03,
               traj_points: int = 16, sample_seed: int = 0) -> Problem:
    """6D double-integrator query on a given sample set: start at rest near
    (0.05,0.05,0.05) jittered by U[-jitter, jitter] per axis, goal ball of radius
    0.05 about (0.95,0.95,0.95) over position (any velocity), m boxes."""
    rng = np.random.default_rng(20_000_003 + int(seed))
    start_p = np.array(DI_START) + rng.uniform(-jitter, jitter, size=3)
    start_q = np.concatenate([to_grid(start_p), np.zeros(3, np.int64)])
    goal_q = to_grid(np.array(DI_GOAL))
    gr = float(np.float32(0.05))
    boxes_q = draw_boxes(rng, m, 3, smin, smax, start_q, goal_q, gr)
    return Problem(kind="di", dim=6, pdim=3, samples=samples,
                   x_init=from_grid(start_q), goal_center=from_grid(goal_q), goal_radius=gr,
                   boxes=np.ascontiguousarray(from_grid(boxes_q)), lam=float(lam), step=0.0,
                   traj_points=int(traj_points), r=float(r), seed=int(seed),
                   sample_seed=int(sample_seed))


def problem_di(seed: int, n: int = 16384, sample_seed: Optional[int] = None, lam: float = 0.5,
               r: float = DI_RADIUS) -> Problem:
    """Headline workload: 6D double integrator, n samples, 40 boxes, lambda 0.5."""
    ss = (seed % 8) if sample_seed is None else sample_seed
    return di_problem(seed, di_samples(ss, n), lam=lam, r=r, sample_seed=ss)


# Dubins airplane workload (Section V-A's forest problem, synthetic): state
# (x, y, z, h) with position in [0,1]^3 and heading 2 pi h, h in [0,1).
DUBINS_START = (0.05, 0.05, 0.5, 0.125)  # heading 45 degrees, towards the goal
DUBINS_GOAL = (0.95, 0.95, 0.5)
DUBINS_TURN = 0.05     # least turning radius
DUBINS_RADIUS = 0.27   # connection radius on the path length (mean in-degree near 7 ln n at n = 5000)
DUBINS_STEP = 0.005    # spacing of the lazy check's points along a path


def dubins_samples(sample_seed: int, n: int, goal_radius: float = 0.05) -> np.ndarray:
    """SoA FP32 [4][n] states: position uniform in the unit cube, heading
    uniform in [0, 1) turns, at least one position in the goal ball.  Free of
    any box world, so one set serves many forests."""
    rng = np.random.default_rng(30_000_001 + int(sample_seed))
    pos = draw_positions(rng, n, 3)
    head = rng.integers(0, QSCALE, size=(n, 1), dtype=np.int64)
    gr = float(np.float32(goal_radius))
    _ensure_goal_sample(rng, pos, to_grid(np.array(DUBINS_GOAL)), gr, None)
    return np.ascontiguousarray(from_grid(np.concatenate([pos, head], axis=1).T))


def draw_forest(rng: np.random.Generator, m: int, start_q: np.ndarray, goal_q: np.ndarray,
                goal_radius: float, side=(0.02, 0.06), height=(0.3, 0.9), clear: float = 0.1) -> np.ndarray:
    """m tree trunks: boxes standing on the ground (z from 0), footprints with
    sides U[side] per axis and heights U[height]; a trunk whose footprint
    comes within `clear` of the start's planar position, or that touches the
    goal ball, is redrawn (the airplane cannot turn away from a trunk closer
    than about two turning radii)."""
    out = []
    while len(out) < m:
        sx, sy = rng.uniform(side[0], side[1], size=2)
        hz = rng.uniform(height[0], height[1])
        lo = np.array([rng.uniform(0.0, 1.0 - sx), rng.uniform(0.0, 1.0 - sy), 0.0])
        hi = lo + np.array([sx, sy, hz])
        lo_q, hi_q = to_grid(lo), to_grid(hi)
        gap = np.maximum(np.maximum(lo_q[:2] - start_q[:2], 0), start_q[:2] - hi_q[:2]).astype(np.float64)
        if float(np.sum(gap * gap)) <= (clear * QSCALE) ** 2:
            continue
        if _box_touches_ball(lo_q, hi_q, goal_q, goal_radius):
            continue
        out.append(np.concatenate([lo_q, hi_q]))
    return np.array(out, dtype=np.int64).reshape(m, 6)


def dubins_problem(seed: int, samples: np.ndarray, m: int = 150, lam: float = 0.5,
                   r: float = DUBINS_RADIUS, turn_radius: float = DUBINS_TURN, step: float = DUBINS_STEP,
                   jitter: float = 0.03, sample_seed: int = 0) -> Problem:
    """Dubins airplane query in a synthetic forest of m trunks: start near
    (0.05, 0.05, 0.5) (position jittered by U[-jitter, jitter] per axis) with
    heading 45 degrees, goal ball of radius 0.05 about (0.95, 0.95, 0.5) over
    position (any heading)."""
    rng = np.random.default_rng(40_000_003 + int(seed))
    start_p = np.array(DUBINS_START[:3]) + rng.uniform(-jitter, jitter, size=3)
    start_q = np.concatenate([to_grid(start_p), to_grid([DUBINS_START[3]])])
    goal_q = to_grid(np.array(DUBINS_GOAL))
    gr = float(np.float32(0.05))
    boxes_q = draw_forest(rng, m, start_q, goal_q, gr)
    return Problem(kind="dubins", dim=4, pdim=3, samples=samples,
                   x_init=from_grid(start_q), goal_center=from_grid(goal_q), goal_radius=gr,
                   boxes=np.ascontiguousarray(from_grid(boxes_q)), lam=float(lam), step=float(step),
                   traj_points=0, r=float(r), seed=int(seed), sample_seed=int(sample_seed),
                   turn_radius=float(turn_radius))


def problem_dubins(seed: int, n: int = 5000, sample_seed: Optional[int] = None, m: int = 150,
                   lam: float = 0.5) -> Problem:
    """Dubins airplane workload: n samples, m trunks, lambda 0.5."""
    ss = (seed % 8) if sample_seed is None else sample_seed
    return dubins_problem(seed, dubins_samples(ss, n), m=m, lam=lam, sample_seed=ss)


def draw_trees(rng: np.random.Generator, trees: int, m: int, start_q: np.ndarray, goal_q: np.ndarray,
               goal_radius: float, clear: float = 0.1) -> np.ndarray:
    """A forest of `trees` trees described by m boxes in all (Section V-B
    varies the resolution of the obstacle representation, not the obstacles):
    each tree is a trunk (footprint half-width U[0.008, 0.02], height
    U[0.3, 0.6]) under a cone canopy (base radius U[0.04, 0.08], height
    U[0.15, 0.3]).  A tree given one box is its bounding box; with k >= 2 boxes
    it is its trunk plus k - 1 slabs that cover the cone (slab j spans the j-th
    of k - 1 equal height bands, as wide as the cone at the band's bottom).
    The m boxes are spread over the trees as evenly as possible.  Trees whose
    bounding box comes within `clear` of the start's planar position, or that
    touch the goal ball, are redrawn."""
    out = []
    per = [m // trees + (1 if t < m % trees else 0) for t in range(trees)]
    for t in range(trees):
        while True:
            w = rng.uniform(0.008, 0.02)
            ht = rng.uniform(0.3, 0.6)
            R = rng.uniform(0.04, 0.08)
            hc = rng.uniform(0.15, 0.3)
            cx = rng.uniform(R, 1.0 - R)
            cy = rng.uniform(R, 1.0 - R)
            blo = to_grid(np.array([cx - R, cy - R, 0.0]))
            bhi = to_grid(np.array([cx + R, cy + R, min(ht + hc, 1.0)]))
            gap = np.maximum(np.maximum(blo[:2] - start_q[:2], 0), start_q[:2] - bhi[:2]).astype(np.float64)
            if float(np.sum(gap * gap)) <= (clear * QSCALE) ** 2 or _box_touches_ball(blo, bhi, goal_q, goal_radius):
                continue
            break
        k = per[t]
        if k == 0:
            continue
        if k == 1:
            out.append(np.concatenate([blo, bhi]))
            continue
        out.append(np.concatenate([to_grid(np.array([cx - w, cy - w, 0.0])), to_grid(np.array([cx + w, cy + w, ht]))]))
        for j in range(k - 1):
            z0 = ht + hc * j / (k - 1)
            z1 = ht + hc * (j + 1) / (k - 1)
            rj = R * (1.0 - j / (k - 1))
            out.append(np.concatenate([to_grid(np.array([cx - rj, cy - rj, min(z0, 1.0)])),
                                       to_grid(np.array([cx + rj, cy + rj, min(z1, 1.0)]))]))
    return np.array(out, dtype=np.int64).reshape(m, 6)


def dubins_forest_problem(seed: int, samples: np.ndarray, m: int, trees: int = 150, lam: float = 0.5,
                          sample_seed: int = 0) -> Problem:
    """Dubins airplane query in a forest of `trees` trees described by m
    boxes (the obstacle-count rows of Table III: one forest, finer boxes)."""
    rng = np.random.default_rng(50_000_017 + int(seed))
    start_p = np.array(DUBINS_START[:3]) + rng.uniform(-0.03, 0.03, size=3)
    start_q = np.concatenate([to_grid(start_p), to_grid([DUBINS_START[3]])])
    goal_q = to_grid(np.array(DUBINS_GOAL))
    gr = float(np.float32(0.05))
    # the same forest at every resolution: its own generator, seeded by `seed` only
    boxes_q = draw_trees(np.random.default_rng(60_000_011 + int(seed)), trees, m, start_q, goal_q, gr)
    return Problem(kind="dubins", dim=4, pdim=3, samples=samples,
                   x_init=from_grid(start_q), goal_center=from_grid(goal_q), goal_radius=gr,
                   boxes=np.ascontiguousarray(from_grid(boxes_q)), lam=float(lam), step=DUBINS_STEP,
                   traj_points=0, r=DUBINS_RADIUS, seed=int(seed), sample_seed=int(sample_seed),
                   turn_radius=DUBINS_TURN)


def collapse_schedule(seed: int, rate: float, t_max: float, pdim: int = 3, side=(0.05, 0.1)):
    """Boxes added over time (Section V-C models a collapsing cave as randomly
    placed boxes added at a rate): a Poisson stream of `rate` boxes per
    second up to t_max, each with sides U[side] per axis placed uniformly in
    the unit cube; returns [(time, box [2*pdim])]."""
    rng = np.random.default_rng(70_000_001 + int(seed))
    out = []
    t = 0.0
    if rate <= 0.0:
        return out
    while True:
        t += rng.exponential(1.0 / rate)
        if t > t_max:
            return out
        sd = rng.uniform(side[0], side[1], size=pdim)
        lo = rng.uniform(0.0, 1.0 - sd)
        out.append((float(t), from_grid(np.concatenate([to_grid(lo), to_grid(lo + sd)]))))


def problem_ids(count: int, first: int = 0) -> List[int]:
    return list(range(first, first + count))


def poisson_arrivals(count: int, rate_hz: float = 2000.0, seed: int = 7) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream: exponential inter-arrival."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))


def batch_specs(count: int = 512, seed: int = 7, sample_seeds: int = 4):
    """Mixed batch: dim in {2, 3, 6}, n log-uniform in [1k, 32k], m in U{10..100}.

    Returns dicts (dim, n, m, sample_seed, problem_seed); n is rounded to a
    multiple of 256 so that problems share resident sample sets."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        dim = int(rng.choice([2, 3, 6]))
        n = int(round(math.exp(rng.uniform(math.log(1024), math.log(32768)))))
        n = max(1024, min(32768, 256 * int(round(n / 256))))
        m = int(rng.integers(10, 101))
        out.append(dict(dim=dim, n=n, m=m, sample_seed=int(rng.integers(0, sample_seeds)),
                        problem_seed=1_000 + k))
    return out


def uniform_samples(dim: int, n: int, sample_seed: int, goal: float = 0.95,
                    goal_radius: float = 0.05) -> np.ndarray:
    """Obstacle-independent Euclidean sample set (SoA FP32 [dim][n], uniform on
    the grid, at least one sample in the goal ball), shared by every box world
    of a replanning stream; samples inside a query's boxes are dead for it."""
    rng = np.random.default_rng(60_000_011 + 977 * int(dim) + int(sample_seed) * 131 + int(n))
    pos = draw_positions(rng, n, dim)
    _ensure_goal_sample(rng, pos, to_grid(np.full(dim, goal)), float(np.float32(goal_radius)), None)
    return np.ascontiguousarray(from_grid(pos.T))


def mixed_problem(spec: dict, samples: np.ndarray, lam: float = 0.5) -> Problem:
    """Query of the mixed replanning stream on a shared sample set: `spec`
    from batch_specs; 2D boxes with sides U[0.05, 0.15] (step 0.005), 3D and
    6D with sides U[0.05, 0.2] (3D step 0.002); the Euclidean radius uses the
    obstacle-free volume (r is a property of the shared roadmap)."""
    dim, m, seed = spec["dim"], spec["m"], spec["problem_seed"]
    if dim == 6:
        return di_problem(seed, samples, m=m, lam=lam, r=di_radius_of(spec["n"]),
                          sample_seed=spec["sample_seed"])
    rng = np.random.default_rng(70_000_003 + int(seed))
    smax, step = (0.15, 0.005) if dim == 2 else (0.2, 0.002)
    start_q = to_grid(np.full(dim, 0.05))
    goal_q = to_grid(np.full(dim, 0.95))
    gr = float(np.float32(0.05))
    boxes_q = draw_boxes(rng, m, dim, 0.05, smax, start_q, goal_q, gr)
    return Problem(kind="euclid", dim=dim, pdim=dim, samples=samples, x_init=from_grid(start_q),
                   goal_center=from_grid(goal_q), goal_radius=gr,
                   boxes=np.ascontiguousarray(from_grid(boxes_q)), lam=float(lam), step=step,
                   r=None, seed=int(seed), sample_seed=int(spec["sample_seed"]))


def di_radius_of(n: int) -> float:
    """Double-integrator radius at n samples: 1.75 at n = 16384, scaled by
    (16384/n)^(1/6)."""
    return DI_RADIUS * (16384.0 / float(n)) ** (1.0 / 6.0)


def clustered_samples(seed: int, dim: int, n: int, extent: float) -> np.ndarray:
    """n grid samples uniform in [0, extent]^dim (SoA FP32): a dense cluster
    whose cells hold far more samples than uniform sets do."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, int(extent * QSCALE) + 1, size=(dim, n), dtype=np.int64)
    return from_grid(k)


def tiny_problem(seed: int, dim: int, n: int, m: int, lam: float, step: float = 0.01,
                 smin: float = 0.1, smax: float = 0.3) -> Problem:
    """Small Euclidean instance for brute-force cross-checks."""
    return geometric_problem(seed, dim, n, m, smin, smax, lam=lam, step=step)


# ---------------------------------------------------------------------------
# learned sampler: parameter initialisation and random draws (both sides use
# these; the method's arithmetic is not here)
# ---------------------------------------------------------------------------
SAMPLER_IN, SAMPLER_HID, SAMPLER_OUT, SAMPLER_COND = 416, 256, 16, 396
SAMPLER_NET = (SAMPLER_HID * SAMPLER_IN + SAMPLER_HID + SAMPLER_HID * SAMPLER_HID + SAMPLER_HID
               + SAMPLER_OUT * SAMPLER_HID + SAMPLER_OUT)
SAMPLER_PARAMS = 2 * SAMPLER_NET


def bf16_round(x) -> np.ndarray:
    """FP32 values rounded to the nearest BF16 value (ties to even), as FP32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def sampler_params(seed: int, out_scale: float = 0.1) -> np.ndarray:
    """Initial parameters of the encoder and decoder (flat FP32, layout of
    include/gmt_sampler.h), BF16-representable.  Uniform He-style weights
    on the 402 real input columns, zero on the padding columns, zero biases,
    output rows beyond the used ones (12 encoder, 6 decoder) zero."""
    rng = np.random.default_rng(30_000_001 + int(seed))
    H, IN, OUT = SAMPLER_HID, SAMPLER_IN, SAMPLER_OUT
    parts = []
    for used in (12, 6):
        a1 = np.sqrt(6.0 / 402.0)
        W1 = rng.uniform(-a1, a1, size=(H, IN))
        W1[:, 6:8] = 0.0
        W1[:, 404:] = 0.0
        a2 = np.sqrt(6.0 / H)
        W2 = rng.uniform(-a2, a2, size=(H, H))
        W3 = np.zeros((OUT, H))
        W3[:used] = rng.uniform(-a2, a2, size=(used, H)) * out_scale
        parts += [W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), np.zeros(OUT)]
    return bf16_round(np.concatenate(parts).astype(np.float32))


def normal_draws(seed: int, count: int, dim: int = 6) -> np.ndarray:
    """Standard normal draws [count][dim] (FP32) for the sampler's noise."""
    rng = np.random.default_rng(40_000_003 + int(seed))
    return rng.standard_normal(size=(count, dim)).astype(np.float32)
