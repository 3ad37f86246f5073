"""Algorithm 1 written out with Python sets, for tiny Euclidean instances.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``).  A second, independent
transcription of GMT* (Section III-A, Algorithm 1) used to pin the C oracle:
no shortcuts, every neighbour relation recomputed by brute force, the three
sets V_unexplored / V_open / V_closed kept literally, the threshold index i
advanced by one per pass (empty groups included).

Readings (shared with the C oracle because the paper fixes them, not code):
neighbours have cost strictly below r; the group is cost <= i*delta; the
parent is the least (cost-to-come + edge cost, node index) over open
neighbours as they stood when the iteration began; the lazy check tests
points y + k (x - y)/(K-1), K-1 the least k >= 1 with k*step >= |x - y|, on
the 2^-20 grid; the goal is a closed ball; lambda = 0 expands the least-cost
open nodes only (FMT*).
"""

from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

QS = 1 << 20


def _q(v: float) -> int:
    return int(round(float(v) * QS))


class Literal:
    def __init__(self, samples: Sequence[Sequence[float]], x_init: Sequence[float],
                 goal_center: Sequence[float], goal_radius: float,
                 boxes: Sequence[Sequence[float]], r: float, lam: float, step: float):
        self.dim = len(x_init)
        self.n = len(samples)
        self.pts: List[Tuple[int, ...]] = [tuple(_q(c) for c in s) for s in samples]
        self.pts.append(tuple(_q(c) for c in x_init))  # root = node n
        self.root = self.n
        d = self.dim
        self.boxes = [(tuple(_q(b[a]) for a in range(d)), tuple(_q(b[d + a]) for a in range(d)))
                      for b in boxes]
        self.R2 = float(r) * float(r) * float(QS) * float(QS)
        self.r = float(r)
        self.lam = float(lam)
        self.step_q = int(round(float(step) * QS))
        gc = tuple(_q(c) for c in goal_center)
        g2 = float(goal_radius) * float(goal_radius) * float(QS) * float(QS)
        self.goal = {v for v in range(self.n + 1)
                     if float(sum((self.pts[v][a] - gc[a]) ** 2 for a in range(d))) <= g2}

    def d2(self, u: int, v: int) -> int:
        return sum((self.pts[u][a] - self.pts[v][a]) ** 2 for a in range(self.dim))

    def c(self, u: int, v: int) -> Optional[float]:
        d2 = self.d2(u, v)
        if float(d2) < self.R2:
            return math.sqrt(float(d2)) / QS
        return None

    def free(self, y: int, x: int) -> bool:
        d2 = self.d2(y, x)
        k1 = 1
        while (k1 * self.step_q) ** 2 < d2:
            k1 += 1
        py, px = self.pts[y], self.pts[x]
        for k in range(k1 + 1):
            p = [k1 * py[a] + k * (px[a] - py[a]) for a in range(self.dim)]
            if any(c < 0 or c > k1 * QS for c in p):
                return False
            for lo, hi in self.boxes:
                if all(k1 * lo[a] <= p[a] <= k1 * hi[a] for a in range(self.dim)):
                    return False
        return True

    def run(self, max_iters: int = 100000) -> Dict:
        n, root = self.n, self.root
        nodes = range(n + 1)
        # root is never a target: it starts in the tree
        nbr_out = {u: {v for v in range(n) if v != u and self.c(u, v) is not None} for u in nodes}
        unexplored = set(range(n))
        open_ = {root}
        closed = set()
        cost: Dict[int, float] = {root: 0.0}
        parent: Dict[int, int] = {root: -1}
        added: Dict[int, int] = {root: -1}
        group: Dict[int, int] = {}
        delta = self.lam * self.r
        i = 0
        while True:
            if i >= max_iters:
                return dict(status=2, i=i, cost=cost, parent=parent, added=added, group=group)
            if self.lam > 0:
                G = {y for y in open_ if cost[y] <= i * delta}
            else:
                mn = min(cost[y] for y in open_)
                G = {y for y in open_ if cost[y] == mn}
            for g in G:
                group[g] = i
            X = {x for g in G for x in nbr_out[g] if x in unexplored}
            staged = {}
            for x in sorted(X):
                Y = [y for y in open_ if x in nbr_out[y]]
                ystar = min(Y, key=lambda y: (cost[y] + self.c(y, x), y))
                if self.free(ystar, x):
                    staged[x] = (ystar, cost[ystar] + self.c(ystar, x))
            for x, (y, cv) in staged.items():
                parent[x] = y
                cost[x] = cv
                added[x] = i
                unexplored.discard(x)
                open_.add(x)
            open_ -= G
            closed |= G
            hits = sorted(G & self.goal, key=lambda v: (cost[v], v))
            if hits:
                z = hits[0]
                path = []
                v = z
                while v != -1:
                    path.append(v)
                    v = parent[v]
                return dict(status=0, i=i, cost=cost, parent=parent, added=added, group=group,
                            z=z, path=path[::-1], path_cost=cost[z])
            if not open_:
                return dict(status=1, i=i, cost=cost, parent=parent, added=added, group=group)
            i += 1


def run_problem(prob, r: float, lam: Optional[float] = None) -> Dict:
    """Literal Algorithm 1 on a Euclidean ``Problem``-like object."""
    s = prob.samples
    samples = [tuple(float(s[a, v]) for a in range(s.shape[0])) for v in range(s.shape[1])]
    boxes = [tuple(float(c) for c in b) for b in prob.boxes]
    L = Literal(samples, [float(c) for c in prob.x_init], [float(c) for c in prob.goal_center],
                prob.goal_radius, boxes, r, prob.lam if lam is None else lam, prob.step)
    return L.run()
