"""The block-wise box draw gives the same boxes, and leaves the generator in
the same state, as drawing one attempt at a time (sides first, then the
lower corner, rejecting boxes that hold the start or touch the goal ball)."""
import numpy as np
import pytest

from paper_1705_02403_amd import inputs as I


def one_at_a_time(rng, m, pdim, smin, smax, start_q, goal_q, goal_radius):
    out = []
    while len(out) < m:
        side = rng.uniform(smin, smax, size=pdim)
        lo = rng.uniform(0.0, 1.0 - side)
        lo_q = I.to_grid(lo)
        hi_q = np.minimum(I.to_grid(lo + side), I.QSCALE)
        if np.all((start_q[:pdim] >= lo_q) & (start_q[:pdim] <= hi_q)):
            continue
        gap = np.maximum(np.maximum(lo_q - goal_q, 0), goal_q - hi_q)
        if float(np.sum(gap * gap)) <= goal_radius * goal_radius * float(I.QSCALE) ** 2:
            continue
        out.append(np.concatenate([lo_q, hi_q]))
    if not out:
        return np.zeros((0, 2 * pdim), dtype=np.int64)
    return np.stack(out).astype(np.int64)


WORLDS = [  # pdim, m, side range, start, goal centre, goal radius
    (2, 20, 0.05, 0.15, (0.05, 0.05), (0.95, 0.95), 0.05),
    (3, 60, 0.05, 0.20, (0.05, 0.05, 0.05), (0.95, 0.95, 0.95), 0.05),
    (3, 40, 0.30, 0.60, (0.5, 0.5, 0.5), (0.9, 0.9, 0.9), 0.2),  # many rejections
    (3, 0, 0.05, 0.20, (0.05, 0.05, 0.05), (0.95, 0.95, 0.95), 0.05),
]


@pytest.mark.parametrize("world", WORLDS)
def test_block_draw_equals_one_at_a_time(world):
    pdim, m, smin, smax, st, gc, gr = world
    sq, gq = I.to_grid(np.array(st)), I.to_grid(np.array(gc))
    for seed in range(300):
        a, b = np.random.default_rng(seed), np.random.default_rng(seed)
        x = I.draw_boxes(a, m, pdim, smin, smax, sq, gq, gr)
        y = one_at_a_time(b, m, pdim, smin, smax, sq, gq, gr)
        assert np.array_equal(x, y), seed
        assert a.random() == b.random(), seed  # the same draws consumed
