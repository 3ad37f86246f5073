"""Halton sample sets on the 2^-20 grid: the oracle's definition.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): imported by
``tests/`` and the benchmark's reference legs, never by the planning
library.  Plain Python integers, one point at a time, so that each value
can be checked by eye against the definition.

Section V-A: the paper's planner draws its samples from the deterministic,
low-dispersion Halton sequence.  The sequence itself is the textbook one:
point k (k = 1, 2, ...; k = 0, the origin, is skipped) has coordinate j equal
to the radical inverse of k in the j-th prime base,

    phi_b(k) = sum_i d_i b^-(i+1)   where   k = sum_i d_i b^i, 0 <= d_i < b.

Readings (the paper gives only the name of the sequence):

* bases 2, 3, 5, 7, 11, 13 for coordinates 0..5;
* every coordinate is put on the 2^-20 grid by rounding down:
  g = floor(phi * 2^20), exact in integers;
* Euclidean state space [0,1]^d: coordinate g * 2^-20;
* double integrator: position coordinates g * 2^-20, velocity coordinates
  (2g - 2^20) * 2^-20 in [-1, 1); a point whose velocity lies outside the
  closed unit ball is skipped (exact integer test);
* a point whose position lies in a closed obstacle box is skipped (samples
  are drawn from X_free, Algorithm 1's input);
* the set of n samples is the first n points that are not skipped, in index
  order, starting at index `first`.
"""

from __future__ import annotations

from fractions import Fraction
from typing import Sequence, Tuple

import numpy as np

PRIMES = (2, 3, 5, 7, 11, 13)
QBITS = 20
QS = 1 << QBITS


def radical_inverse(k: int, b: int) -> Fraction:
    """phi_b(k) as an exact fraction: the base-b digits of k mirrored about
    the radix point."""
    assert k >= 0 and b >= 2
    x = Fraction(0)
    scale = Fraction(1, b)
    while k > 0:
        k, d = divmod(k, b)
        x += d * scale
        scale /= b
    return x


def grid_coordinate(k: int, b: int) -> int:
    """floor(phi_b(k) * 2^20): the grid integer of the coordinate."""
    f = radical_inverse(k, b) * QS
    return f.numerator // f.denominator


def grid_coordinates(ks: np.ndarray, b: int) -> np.ndarray:
    """floor(phi_b(k) * 2^20) for many k at once, in exact int64 arithmetic:
    phi_b(k) = num / b^L with num the digits of k read in reverse, so the
    grid integer is (num * 2^20) // b^L (below 2^54 for k < 2^31, b <= 13)."""
    k = np.asarray(ks, dtype=np.int64).copy()
    assert np.all(k >= 0) and np.all(k < (1 << 31))
    num = np.zeros_like(k)
    den = np.ones_like(k)
    while np.any(k > 0):
        live = k > 0
        d = k % b
        num = np.where(live, num * b + d, num)
        den = np.where(live, den * b, den)
        k //= b
    return (num << QBITS) // den


def halton_state(k: int, dim: int, di: bool) -> Tuple[int, ...]:
    """Grid integers of point k: positions in [0, 2^20), velocities (double
    integrator, coordinates 3..5) in [-2^20, 2^20)."""
    out = []
    for j in range(dim):
        g = grid_coordinate(k, PRIMES[j])
        out.append(2 * g - QS if (di and j >= 3) else g)
    return tuple(out)


def _in_box(p: Sequence[int], boxes_q: np.ndarray, pd: int) -> bool:
    for b in boxes_q:
        if all(b[a] <= p[a] <= b[pd + a] for a in range(pd)):
            return True
    return False


def accepted(state: Sequence[int], di: bool, boxes_q: np.ndarray, pd: int) -> bool:
    """The skip rules: velocity in the closed unit ball, position outside
    every closed box."""
    if di and sum(v * v for v in state[3:6]) > QS * QS:
        return False
    return not _in_box(state, boxes_q, pd)


def halton_samples(n: int, dim: int, di: bool = False, boxes=None, first: int = 1):
    """The first n accepted Halton points from index `first` on, SoA FP32
    [dim][n] (exact: grid integers times 2^-20), and the index after the last
    point examined."""
    pd = 3 if di else dim
    if boxes is None or len(boxes) == 0:
        bq = np.zeros((0, 2 * pd), np.int64)
    else:
        bq = np.rint(np.asarray(boxes, np.float64).reshape(-1, 2 * pd) * QS).astype(np.int64)
    chunks = [np.zeros((dim, 0), np.int64)]
    got = 0
    k = first
    while got < n:
        ks = np.arange(k, k + max(2 * (n - got), 1024), dtype=np.int64)
        g = np.stack([grid_coordinates(ks, PRIMES[j]) for j in range(dim)])
        if di:
            g[3:6] = 2 * g[3:6] - QS
        keep = np.ones(ks.size, dtype=bool)
        if di:
            keep &= (g[3:6] ** 2).sum(axis=0) <= QS * QS
        for b in bq:
            inside = np.ones(ks.size, dtype=bool)
            for a in range(pd):
                inside &= (g[a] >= b[a]) & (g[a] <= b[pd + a])
            keep &= ~inside
        idx = np.flatnonzero(keep)[: n - got]
        chunks.append(g[:, idx])
        got += idx.size
        k = int(ks[idx[-1]]) + 1 if got == n else int(ks[-1]) + 1
    q = np.concatenate(chunks, axis=1)
    return np.ascontiguousarray((q.astype(np.float64) / QS).astype(np.float32)), k


def halton_samples_literal(n: int, dim: int, di: bool = False, boxes=None, first: int = 1):
    """The same set, one point at a time through the exact fractions (small n)."""
    pd = 3 if di else dim
    if boxes is None or len(boxes) == 0:
        bq = np.zeros((0, 2 * pd), np.int64)
    else:
        bq = np.rint(np.asarray(boxes, np.float64).reshape(-1, 2 * pd) * QS).astype(np.int64)
    rows = []
    k = first
    while len(rows) < n:
        s = halton_state(k, dim, di)
        if accepted(s, di, bq, pd):
            rows.append(s)
        k += 1
    q = np.array(rows, dtype=np.int64).reshape(n, dim).T
    return np.ascontiguousarray((q.astype(np.float64) / QS).astype(np.float32)), k


def halton_radius(d: int, mu: float, n: int, factor: float = 1.1) -> float:
    """Reading for the radius of a Halton set (the paper allows a radius
    below Theorem 1's for low-dispersion samples without a value): twice a
    dispersion bound kappa_d (mu/n)^(1/d), times the margin factor 1.1 of
    Theorem 1's (1+eta)^(1/d).  kappa_2 = 1.5 and kappa_3 = 1.7 bound the
    largest empty ball of the sets measured by ``dispersion`` below.  The
    result is capped at Theorem 1's radius, the paper's value for uniform
    samples, since the reading may only make the radius smaller."""
    import math
    kappa = {2: 1.5, 3: 1.7}[d]
    r_disp = factor * 2.0 * kappa * (mu / n) ** (1.0 / d)
    zeta = math.pi ** (d / 2.0) / math.gamma(d / 2.0 + 1.0)
    r_thm1 = factor * 4.0 * (1.0 / d) ** (1.0 / d) * (mu / zeta) ** (1.0 / d) * (math.log(n) / n) ** (1.0 / d)
    return min(r_disp, r_thm1)


def dispersion(samples) -> float:
    """Radius of the largest empty ball centred in [0,1]^d: the largest
    distance from a Voronoi vertex inside the cube, or from a probe on a face
    of the cube, to its nearest sample (a lower estimate of the exact value
    on the faces)."""
    from scipy.spatial import Voronoi, cKDTree
    s = np.asarray(samples, np.float64)
    d = s.shape[0]
    tree = cKDTree(s.T)
    v = Voronoi(s.T).vertices
    v = v[np.all((v >= 0) & (v <= 1), axis=1)]
    best = float(tree.query(v)[0].max()) if len(v) else 0.0
    lin = np.linspace(0.0, 1.0, 300 if d == 2 else 90)
    for a in range(d):
        for val in (0.0, 1.0):
            g = np.stack(np.meshgrid(*[lin] * (d - 1), indexing="ij")).reshape(d - 1, -1)
            best = max(best, float(tree.query(np.insert(g, a, val, axis=0).T)[0].max()))
    return best
