"""Pins of the oracle's per-iteration records (Algorithm 1 lines 3-9) against
brute force over its tree outputs and neighbour table: which iterations had a
group, the open set when each began, the group, the unexplored out-neighbours
of the group (line 4), those lying in an obstacle, the lazy-check failures and
the nodes added.  The tree outputs themselves are pinned elsewhere (literal
set transcription, heap FMT*, Dijkstra)."""

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_02403_amd import inputs as I


def out_rows(n, table):
    """out-neighbours of every sample: x such that y lies in in-row x"""
    rows = [[] for _ in range(n)]
    for x in range(n):
        for y in table.col[table.row_ptr[x]:table.row_ptr[x + 1]]:
            rows[int(y)].append(x)
    return [np.array(r, np.int64) for r in rows]


def root_neighbours(prob, r):
    """samples within r of the root, by the cost definitions of Section V-A"""
    n = prob.samples.shape[1]
    kind = O.kind_of(prob)
    if kind == O.EUCLID:
        q = np.round(prob.samples.astype(np.float64) * 2.0 ** 20).astype(np.int64)
        x = np.round(np.asarray(prob.x_init, np.float64) * 2.0 ** 20).astype(np.int64)
        d2 = ((q - x[:, None]) ** 2).sum(axis=0).astype(np.float64)
        return np.nonzero(d2 < float(np.float64(r) * np.float64(r)) * 2.0 ** 40)[0]
    xi = np.asarray(prob.x_init, np.float64)
    return np.array([v for v in range(n) if O.di_cost(xi, prob.samples[:, v].astype(np.float64))[0] < r], np.int64)


def in_obstacle(prob):
    q = np.round(prob.samples[:prob.pdim].astype(np.float64) * 2.0 ** 20).astype(np.int64)
    b = np.round(np.asarray(prob.boxes, np.float64).reshape(-1, 2 * prob.pdim) * 2.0 ** 20).astype(np.int64)
    dead = np.zeros(q.shape[1], bool)
    for box in b:
        lo, hi = box[:prob.pdim, None], box[prob.pdim:, None]
        dead |= np.all((q >= lo) & (q <= hi), axis=0)
    return dead


def brute_trace(prob, r, table, pl):
    n = prob.samples.shape[1]
    root = n
    gi, ai = pl.group_iter, pl.added_iter
    outs = out_rows(n, table)
    rootn = root_neighbours(prob, r)
    dead = in_obstacle(prob)
    recs = []
    for i in sorted(set(int(v) for v in gi if v >= 0)):
        added_before = (ai == -1) | ((ai >= 0) & (ai < i))
        open_now = added_before & ((gi == -1) | (gi >= i))
        G = np.nonzero(gi == i)[0]
        unexplored = np.ones(n + 1, bool)
        unexplored[added_before] = False
        unexplored[root] = False
        C = set()
        for g in G:
            nb = rootn if g == root else outs[g]
            C.update(int(x) for x in nb if unexplored[x])
        C = np.array(sorted(C), np.int64)
        added = int((ai == i).sum())
        recs.append((i, int(open_now.sum()), len(G), len(C), int(dead[C].sum()) if len(C) else 0,
                     len(C) - added, added))
    return np.array(recs, np.int32).reshape(-1, 7)


def with_boxes_of(p, seed):
    """the same samples under another seed's boxes: some samples then lie in
    obstacles (the box draws keep the start and goal clear)"""
    q = I.tiny_problem(seed, p.dim, 16, 6, p.lam)
    return dataclasses.replace(p, boxes=q.boxes)


CASES = [
    ("2d", lambda: I.tiny_problem(3, 2, 400, 6, 0.5)),
    ("2d_fmt", lambda: I.tiny_problem(4, 2, 300, 5, 0.0)),
    ("2d_dead", lambda: with_boxes_of(I.tiny_problem(5, 2, 400, 6, 0.5), 11)),
    ("3d_dead", lambda: with_boxes_of(I.tiny_problem(6, 3, 500, 8, 0.5), 12)),
    ("2d_lam1", lambda: I.tiny_problem(7, 2, 300, 6, 1.0)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_trace_matches_brute_force(name, make):
    p = make()
    r = O.euclid_radius(p)
    t = O.neighbors(p.samples, O.EUCLID, r)
    pl = O.plan(p, r, t, trace=True)
    want = brute_trace(p, r, t, pl)
    assert pl.trace.shape == want.shape and np.array_equal(pl.trace, want), name
    # iteration records add up to the tree
    assert pl.trace[:, 2].sum() == (pl.group_iter >= 0).sum()
    assert pl.trace[:, 6].sum() == (pl.added_iter >= 0).sum()
    if name.endswith("_dead"):
        assert pl.trace[:, 4].sum() > 0  # the case exercises candidates in obstacles


def test_trace_double_integrator_brute_force():
    s = I.di_samples(2, 160)
    p = I.di_problem(4, s, r=2.6)
    t = O.neighbors(p.samples, O.DI, p.r)
    pl = O.plan(p, p.r, t, trace=True)
    want = brute_trace(p, p.r, t, pl)
    assert np.array_equal(pl.trace, want)
    assert pl.trace[:, 4].sum() > 0


def test_trace_sink_is_per_call():
    """the record sink is installed for one plan only"""
    p = I.tiny_problem(3, 2, 400, 6, 0.5)
    r = O.euclid_radius(p)
    full = O.plan(p, r, trace=True).trace
    assert len(full) > 3
    plain = O.plan(p, r)
    assert plain.trace is None
    again = O.plan(p, r, trace=True).trace
    assert np.array_equal(full, again)
