"""Pins of the oracle's Halton sample sets (Section V-A: the planner samples
the deterministic, low-dispersion Halton sequence) against facts fixed by
the mathematics of radical inverses, not by the oracle's own code:

* the van der Corput values of the first indices in bases 2 and 3;
* the first b^L radical inverses in base b are exactly {j / b^L};
* any N = 2^a 3^c consecutive 2D Halton points from index 1 put exactly one
  point in each cell of the 2^a x 3^c grid (the Chinese-remainder
  stratification of the sequence);
* the grid integer is the floor: an independent floating-point evaluation
  lands inside the cell it names;
* the vectorised integer path equals the exact-fraction definition;
* the skip rules against a brute-force recount of the raw points.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import halton as H


def test_van_der_corput_base_2_and_3():
    assert [H.radical_inverse(k, 2) for k in range(1, 8)] == [
        Fraction(1, 2), Fraction(1, 4), Fraction(3, 4), Fraction(1, 8), Fraction(5, 8), Fraction(3, 8),
        Fraction(7, 8)]
    assert [H.radical_inverse(k, 3) for k in range(1, 9)] == [
        Fraction(1, 3), Fraction(2, 3), Fraction(1, 9), Fraction(4, 9), Fraction(7, 9), Fraction(2, 9),
        Fraction(5, 9), Fraction(8, 9)]
    assert H.radical_inverse(0, 5) == 0


@pytest.mark.parametrize("b", H.PRIMES)
def test_first_b_power_points_are_the_b_adic_grid(b):
    L = 3 if b <= 5 else 2
    N = b ** L
    got = sorted(H.radical_inverse(k, b) for k in range(N))
    assert got == [Fraction(j, N) for j in range(N)]


@pytest.mark.parametrize("a,c", [(3, 2), (5, 3), (2, 4)])
def test_2d_points_stratify_the_mixed_radix_grid(a, c):
    N = 2 ** a * 3 ** c
    cells = set()
    for k in range(1, N + 1):
        x, y = H.radical_inverse(k, 2), H.radical_inverse(k, 3)
        cells.add((int(x * 2 ** a), int(y * 3 ** c)))
    assert len(cells) == N


def test_grid_integer_is_the_floor():
    rng = np.random.default_rng(1)
    ks = rng.integers(1, 1 << 31, size=400)
    for b in H.PRIMES:
        for k in ks[:60]:
            k = int(k)
            # digit sum in floating point, an independent evaluation
            x, scale, m = 0.0, 1.0 / b, k
            while m:
                x += (m % b) * scale
                scale /= b
                m //= b
            g = H.grid_coordinate(k, b)
            assert g <= x * H.QS < g + 1 + 1e-6
            assert 0 <= g < H.QS


def test_vectorised_path_equals_the_fractions():
    rng = np.random.default_rng(2)
    ks = np.concatenate([np.arange(0, 300), rng.integers(1, (1 << 31) - 1, size=300),
                         [(1 << 31) - 1, 13 ** 8, 13 ** 8 - 1, 3 ** 19, 2 ** 30]])
    for b in H.PRIMES:
        want = np.array([H.grid_coordinate(int(k), b) for k in ks], dtype=np.int64)
        np.testing.assert_array_equal(H.grid_coordinates(ks, b), want)


def test_sets_match_the_literal_construction():
    boxes = np.array([[0.1, 0.1, 0.1, 0.5, 0.6, 0.7], [0.4, 0.0, 0.2, 0.9, 0.3, 0.8]], np.float32)
    for n, dim, di, bx, first in [(1, 2, False, None, 1), (777, 2, False, None, 5),
                                  (1500, 3, False, boxes, 17), (900, 6, True, boxes, 1),
                                  (64, 6, True, None, 1000)]:
        a, ka = H.halton_samples(n, dim, di, bx, first)
        b, kb = H.halton_samples_literal(n, dim, di, bx, first)
        np.testing.assert_array_equal(a, b)
        assert ka == kb
    e, k = H.halton_samples(0, 3)
    assert e.shape == (3, 0) and k == 1


def test_skip_rules_against_a_recount():
    """Double integrator with boxes: every kept point is in free space with a
    velocity in the closed ball, and the kept count over the raw points
    examined equals a brute-force count of the raw points that pass."""
    boxes = np.array([[0.2, 0.2, 0.2, 0.6, 0.7, 0.5]], np.float32)
    n = 500
    s, k_end = H.halton_samples(n, 6, True, boxes)
    q = np.rint(s.astype(np.float64) * H.QS).astype(np.int64)
    assert np.all((q[3:] ** 2).sum(axis=0) <= H.QS ** 2)
    lo, hi = np.rint(boxes[0, :3] * H.QS), np.rint(boxes[0, 3:] * H.QS)
    assert not np.any(np.all((q[:3].T >= lo) & (q[:3].T <= hi), axis=1))
    kept = 0
    for k in range(1, k_end):
        pos = [H.radical_inverse(k, b) for b in (2, 3, 5)]
        vel = [2 * H.radical_inverse(k, b) - 1 for b in (7, 11, 13)]
        # grid rounding of the velocity: floor on phi, then 2g - 2^20
        vq = [2 * (int(H.radical_inverse(k, b) * H.QS)) - H.QS for b in (7, 11, 13)]
        pq = [int(p * H.QS) for p in pos]
        in_box = all(lo[a] <= pq[a] <= hi[a] for a in range(3))
        if sum(v * v for v in vq) <= H.QS ** 2 and not in_box:
            kept += 1
        assert abs(vel[0]) <= 1
    assert kept == n
    # the last point examined was kept
    last = H.halton_state(k_end - 1, 6, True)
    assert H.accepted(last, True, np.rint(boxes * H.QS).astype(np.int64), 3)


@pytest.mark.parametrize("d,n", [(2, 1024), (2, 2000), (3, 2000), (3, 4096)])
def test_radius_reading_covers_twice_the_dispersion(d, n):
    """The Halton radius keeps a margin over twice the set's dispersion, and
    lies below Theorem 1's radius for uniform samples at the same n."""
    s, _ = H.halton_samples(n, d)
    D = H.dispersion(s)
    r = H.halton_radius(d, 1.0, n)
    assert 2.0 * D < r / 1.05
    from oracle import oracle as O
    assert r <= O.radius(d, 1.0, n) * (1 + 1e-12)
    if n >= 4096:
        assert r < 0.98 * O.radius(d, 1.0, n)
