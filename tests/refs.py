"""Independent references used by the CPU tests to pin the oracle.

Nothing here is shared with the oracle or the library: disk graphs by numpy
brute force, shortest paths by scipy, the lazy check rewritten with numpy
integers, and a heap-ordered FMT* (one node expanded at a time).
"""

from __future__ import annotations

import heapq
import math

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

QS = 1 << 20


def grid_states(prob) -> np.ndarray:
    """[n+1, dim] int64 grid coordinates, root last."""
    s = np.rint(prob.samples.astype(np.float64).T * QS).astype(np.int64)
    root = np.rint(prob.x_init.astype(np.float64) * QS).astype(np.int64)
    return np.concatenate([s, root[None, :]], axis=0)


def euclid_pairs(prob, r: float):
    """All ordered pairs (u, v), u != v, v a sample, with d2 < fl(r*r)*2^40."""
    P = grid_states(prob)
    n = prob.n
    R2 = float(r) * float(r) * float(QS) * float(QS)
    us, vs, cs = [], [], []
    for u in range(n + 1):
        d = P[:n] - P[u][None, :]
        d2 = np.sum(d * d, axis=1)
        ok = d2.astype(np.float64) < R2
        if u < n:
            ok[u] = False
        idx = np.nonzero(ok)[0]
        us.append(np.full(len(idx), u))
        vs.append(idx)
        cs.append(np.sqrt(d2[idx].astype(np.float64)) / QS)
    return np.concatenate(us), np.concatenate(vs), np.concatenate(cs)


def segment_free(prob, y: int, x: int, P=None) -> bool:
    """Lazy check of the straight edge y -> x on the grid (numpy rewrite)."""
    if P is None:
        P = grid_states(prob)
    step_q = int(round(prob.step * QS))
    py, px = P[y], P[x]
    d2 = int(np.sum((px - py) ** 2))
    k1 = max(1, math.isqrt(max(d2 - 1, 0)) // step_q)
    while (k1 * step_q) ** 2 < d2:
        k1 += 1
    while k1 > 1 and ((k1 - 1) * step_q) ** 2 >= d2:
        k1 -= 1
    k = np.arange(k1 + 1, dtype=np.int64)[:, None]
    pts = k1 * py[None, :] + k * (px - py)[None, :]
    if np.any(pts < 0) or np.any(pts > k1 * QS):
        return False
    b = np.rint(prob.boxes.astype(np.float64) * QS).astype(np.int64)
    d = prob.pdim
    for lo, hi in zip(b[:, :d], b[:, d:]):
        inside = np.all((pts >= k1 * lo) & (pts <= k1 * hi), axis=1)
        if np.any(inside):
            return False
    return True


def segments_free(prob, ys, xs, P=None, chunk=4096) -> np.ndarray:
    """Vectorised lazy check of many straight edges ys[k] -> xs[k]."""
    if P is None:
        P = grid_states(prob)
    ys = np.asarray(ys, np.int64)
    xs = np.asarray(xs, np.int64)
    out = np.ones(len(ys), bool)
    step_q = int(round(prob.step * QS))
    b = np.rint(prob.boxes.astype(np.float64) * QS).astype(np.int64)
    d = prob.pdim
    for s0 in range(0, len(ys), chunk):
        py, px = P[ys[s0:s0 + chunk]], P[xs[s0:s0 + chunk]]
        dd = px - py
        d2 = np.sum(dd * dd, axis=1)
        k1 = np.maximum(1, np.ceil(np.sqrt(d2.astype(np.float64)) / step_q).astype(np.int64))
        k1 = np.where((k1 > 1) & (((k1 - 1) * step_q) ** 2 >= d2), k1 - 1, k1)
        k1 = np.where((k1 * step_q) ** 2 < d2, k1 + 1, k1)
        K = int(k1.max()) + 1
        k = np.arange(K, dtype=np.int64)[None, :, None]
        pts = k1[:, None, None] * py[:, None, :] + k * dd[:, None, :]
        valid = (np.arange(K)[None, :] <= k1[:, None])
        bad = np.any(((pts < 0) | (pts > k1[:, None, None] * QS)).any(axis=2) & valid, axis=1)
        for lo, hi in zip(b[:, :d], b[:, d:]):
            inside = np.all((pts >= k1[:, None, None] * lo) & (pts <= k1[:, None, None] * hi), axis=2)
            bad |= np.any(inside & valid, axis=1)
        out[s0:s0 + chunk] = ~bad
    return out


def scipy_dist(prob, r: float, check_collisions: bool = True, clear_only: bool = False):
    """Least cost from the root over the (collision-free) disk graph."""
    n = prob.n
    u, v, c = euclid_pairs(prob, r)
    P = grid_states(prob)
    keep = np.ones(len(u), bool)
    if clear_only:
        R2 = float(r) * float(r) * float(QS) * float(QS)
        b = np.rint(prob.boxes.astype(np.float64) * QS).astype(np.int64)
        d = prob.pdim
        ok = np.ones(n + 1, bool)
        for w in range(n + 1):
            gap = np.maximum(np.maximum(b[:, :d] - P[w], 0), P[w] - b[:, d:])
            if b.shape[0] and np.any(np.sum(gap * gap, axis=1).astype(np.float64) <= R2):
                ok[w] = False
            if np.any(P[w].astype(np.float64) ** 2 <= R2) or np.any((QS - P[w]).astype(np.float64) ** 2 <= R2):
                ok[w] = False
        keep &= ok[u] & ok[v]
    if check_collisions:
        idx = np.nonzero(keep)[0]
        keep[idx] = segments_free(prob, u[idx], v[idx], P)
    A = sp.csr_matrix((c[keep], (u[keep], v[keep])), shape=(n + 1, n + 1))
    return dijkstra(A, directed=True, indices=n)


def fmt_heap(prob, r: float):
    """FMT* with a binary heap: expand the least-cost open node (lowest index on
    ties) one at a time; lazy parent choice among open neighbours; stop when the
    expanded node lies in the goal ball."""
    n = prob.n
    P = grid_states(prob)
    R2 = float(r) * float(r) * float(QS) * float(QS)
    gq = np.rint(prob.goal_center.astype(np.float64) * QS).astype(np.int64)
    g2 = float(prob.goal_radius) * float(prob.goal_radius) * float(QS) * float(QS)

    def nbrs(u):
        d = P[:n] - P[u][None, :]
        d2 = np.sum(d * d, axis=1)
        ok = d2.astype(np.float64) < R2
        if u < n:
            ok[u] = False
        idx = np.nonzero(ok)[0]
        return idx, np.sqrt(d2[idx].astype(np.float64)) / QS

    nb = [nbrs(u) for u in range(n + 1)]
    state = np.zeros(n + 1, np.int8)  # 0 unvisited, 1 open, 2 closed
    cost = np.full(n + 1, np.inf)
    parent = np.full(n + 1, -1)
    root = n
    state[root] = 1
    cost[root] = 0.0
    heap = [(0.0, root)]
    while heap:
        cz, z = heapq.heappop(heap)
        if state[z] != 1 or cz != cost[z]:
            continue
        if float(np.sum((P[z][:prob.pdim] - gq) ** 2)) <= g2:
            path = [z]
            while parent[path[-1]] >= 0:
                path.append(int(parent[path[-1]]))
            return cost, parent, path[::-1]
        idx, _ = nb[z]
        new = []
        for x in idx:
            if state[x] != 0:
                continue
            best, by = np.inf, -1
            for y in range(n + 1):
                if state[y] != 1:
                    continue
                iy, cy = nb[y]
                pos = np.searchsorted(iy, x)
                if pos < len(iy) and iy[pos] == x:
                    val = cost[y] + cy[pos]
                    if val < best or (val == best and y < by):
                        best, by = val, y
            if by >= 0 and segment_free(prob, by, int(x), P):
                new.append((int(x), by, best))
        for x, y, c in new:
            state[x] = 1
            cost[x] = c
            parent[x] = y
            heapq.heappush(heap, (c, x))
        state[z] = 2
    return cost, parent, None
