"""Replanning in a changing world (Section V-C: a collapsing cave, modelled as
obstacle boxes added at a rate, with the planner rerun as often as it can).

Many independent scenarios share one resident roadmap.  Every tick (dt
seconds of world time) the loop

1. adds each scenario's boxes that are due -- a box that would contain the
   scenario's committed next node, or touch the goal ball, lands elsewhere
   (it is skipped and counted), so the robot is never inside an obstacle;
2. moves each robot along its plan at `speed` cost units per second; a robot
   that reaches a node flies on with the plan computed from that node, and
   waits there while there is none (so every edge it flies was checked
   against the boxes present when it was planned; a box that appears across
   the edge being flown is not seen until the next node);
3. replans every live scenario from its committed next node against its
   current boxes -- all scenarios in one batched launch.

The planner is passed in (the library's batched GMT* by default), so the
same loop runs on any planner with the same inputs and outputs.  Reported:
replans per second, per-tick planning latency, success (reaching the goal
ball before `t_max`) and the cost flown.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import gmt

PlanOut = Tuple[int, np.ndarray, float]  # status, path (root first), path cost
GRID = float(1 << 20)  # coordinate quantum 2^-20


@dataclass
class Scenario:
    """One robot: start state, goal ball, initial boxes, and the boxes the
    collapse adds (arrival time, box), in time order."""
    x_init: np.ndarray
    goal_center: np.ndarray
    goal_radius: float
    boxes: np.ndarray
    schedule: List[Tuple[float, np.ndarray]]
    lam: float = 0.5


@dataclass
class RobotState:
    cur: int = -1               # node reached last (-1: the start state)
    active: Optional[np.ndarray] = None  # plan being flown (node ids, root first)
    costs: Optional[np.ndarray] = None   # its edge costs
    ai: int = 0                 # edge being flown: active[ai] -> active[ai + 1]
    progress: float = 0.0       # cost flown along that edge
    flown: float = 0.0          # cost flown in all
    latest: Optional[tuple] = None  # newest plan: (root node, path, path cost, boxes it saw)
    seen: int = 0               # boxes the plan being flown was checked against
    reached: List[tuple] = field(default_factory=list)  # (node, boxes its plan saw)
    done: bool = False
    success: bool = False
    t_done: float = 0.0
    boxes: List[np.ndarray] = field(default_factory=list)
    next_box: int = 0
    skipped: int = 0

    @property
    def nxt(self) -> int:
        """Committed next node (-1: waiting at cur)."""
        return int(self.active[self.ai + 1]) if self.active is not None else -1


class EdgeCosts:
    """Edge costs c(u -> v) from an in-table (row v lists its in-neighbours u,
    ascending): a roadmap's export, or given arrays."""

    def __init__(self, roadmap: "gmt.Roadmap" = None, table: tuple = None):
        if roadmap is not None:
            self.row_ptr, self.col, self.cost, _ = roadmap.export()
        else:
            self.row_ptr, self.col, self.cost = table

    def __call__(self, u: int, v: int) -> float:
        b, e = int(self.row_ptr[v]), int(self.row_ptr[v + 1])
        k = b + int(np.searchsorted(self.col[b:e], u))
        if k >= e or int(self.col[k]) != u:
            raise KeyError("edge %d -> %d not in the table" % (u, v))
        return float(self.cost[k])


def library_planner(roadmap: "gmt.Roadmap", opts: "gmt.gmt_plan_opts", pdim: int):
    """Batched GMT* on the GPU: queries (x_init, goal centre, goal radius,
    boxes, lambda) -> (status, path, path cost)."""
    def plan(queries: Sequence[tuple]) -> List[PlanOut]:
        qs = [gmt.BatchQuery(roadmap, x, gmt.make_goal(gc, gr, pdim), bx, lam, opts.edge_step)
              for (x, gc, gr, bx, lam) in queries]
        return [(r.status, r.path, r.path_cost) for r in gmt.gmt_plan_batch(qs, opts)]
    return plan


class Replanner:
    def __init__(self, samples: np.ndarray, edge_cost: Callable[[int, int], float],
                 plan_batch: Callable[[Sequence[tuple]], List[PlanOut]], scenarios: Sequence[Scenario],
                 pdim: int = 3, dt: float = 0.01, speed: float = 1.0, t_max: float = 10.0):
        self.s = np.asarray(samples)
        self.n = self.s.shape[1]
        self.edge_cost = edge_cost
        self.plan_batch = plan_batch
        self.sc = list(scenarios)
        self.pdim = pdim
        self.dt, self.speed, self.t_max = float(dt), float(speed), float(t_max)
        self.robots = [RobotState(boxes=[np.asarray(b) for b in sc.boxes]) for sc in self.sc]
        self.tick_ms: List[float] = []
        self.replans = 0
        self.events: List[tuple] = []  # (tick, scenario, what, node) -- for determinism checks

    # -- helpers ------------------------------------------------------------
    def state_of(self, k: int, v: int) -> np.ndarray:
        return self.sc[k].x_init if v < 0 else self.s[:, v]

    def _in_goal(self, k: int, v: int) -> bool:
        """The library's goal test: squared grid distance against the FP32
        radius squared in FP64, times 2^40."""
        q = np.rint(self.state_of(k, v)[: self.pdim].astype(np.float64) * GRID).astype(np.int64)
        g = np.rint(np.asarray(self.sc[k].goal_center, np.float64)[: self.pdim] * GRID).astype(np.int64)
        rr = float(np.float32(self.sc[k].goal_radius))
        return float(np.sum((q - g) ** 2)) <= rr * rr * GRID * GRID

    def _box_allowed(self, k: int, box: np.ndarray) -> bool:
        pd = self.pdim
        lo, hi = box[:pd].astype(np.float64), box[pd:].astype(np.float64)
        anchor = self.robots[k].nxt if self.robots[k].nxt >= 0 else self.robots[k].cur
        p = self.state_of(k, anchor)[:pd].astype(np.float64)
        if np.all(p >= lo) and np.all(p <= hi):
            return False
        gc = np.asarray(self.sc[k].goal_center, np.float64)[:pd]
        gap = np.maximum(np.maximum(lo - gc, 0.0), gc - hi)
        return float(np.sum(gap * gap)) > float(self.sc[k].goal_radius) ** 2

    def _edge_costs(self, path: np.ndarray, cost: float) -> np.ndarray:
        """Edge costs of a plan: table lookups, the first edge being what the
        path cost leaves over."""
        c = np.array([self.edge_cost(int(a), int(b)) for a, b in zip(path[1:-1], path[2:])], np.float64)
        return np.concatenate([[cost - float(c.sum())], c])

    def _adopt(self, k: int) -> bool:
        """At node cur: fly the newest plan if it was computed from cur."""
        r = self.robots[k]
        if r.latest is None or r.latest[0] != r.cur or len(r.latest[1]) < 2:
            return False
        r.active, r.costs, r.ai, r.progress = r.latest[1], self._edge_costs(r.latest[1], r.latest[2]), 0, 0.0
        r.seen = r.latest[3]
        return True

    # -- the loop -------------------------------------------------------------
    def _replan(self, tick: int) -> None:
        live = [k for k, r in enumerate(self.robots) if not r.done]
        if not live:
            return
        qs, roots = [], []
        for k in live:
            r = self.robots[k]
            root = r.nxt if r.nxt >= 0 else r.cur
            roots.append(root)
            bx = np.ascontiguousarray(np.array(r.boxes, np.float32).reshape(-1, 2 * self.pdim))
            qs.append((self.state_of(k, root).astype(np.float32), self.sc[k].goal_center, self.sc[k].goal_radius,
                       bx, self.sc[k].lam))
        t0 = time.perf_counter()
        out = self.plan_batch(qs)
        self.tick_ms.append((time.perf_counter() - t0) * 1e3)
        self.replans += len(qs)
        for k, root, (st, path, cost) in zip(live, roots, out):
            r = self.robots[k]
            if st == gmt.GMT_OK:
                # the path is rooted at the replanning state: name it by its node
                p = np.array(path, np.int64)
                p[0] = root
                r.latest = (root, p, float(cost), len(r.boxes))
            else:
                r.latest = None
            self.events.append((tick, k, "plan", int(st)))

    def _advance(self, tick: int, t: float) -> None:
        for k, r in enumerate(self.robots):
            if r.done:
                continue
            sc = self.sc[k]
            while r.next_box < len(sc.schedule) and sc.schedule[r.next_box][0] <= t:
                box = np.asarray(sc.schedule[r.next_box][1], np.float32)
                if self._box_allowed(k, box):
                    r.boxes.append(box)
                else:
                    r.skipped += 1
                r.next_box += 1
            if r.active is None:
                self._adopt(k)  # waiting: a plan from this node may have appeared
            left = self.dt * self.speed
            while left > 0.0 and r.active is not None and not r.done:
                step = min(left, float(r.costs[r.ai]) - r.progress)
                r.progress += step
                r.flown += step
                left -= step
                if r.progress < float(r.costs[r.ai]):
                    break
                r.cur = int(r.active[r.ai + 1])
                r.reached.append((r.cur, r.seen))
                self.events.append((tick, k, "reach", r.cur))
                if self._in_goal(k, r.cur):
                    r.done, r.success, r.t_done = True, True, t
                    break
                if not self._adopt(k):
                    # no plan from this node yet (or none exists): wait here
                    # for the next replan rather than fly a stale plan on
                    r.active = None
            if not r.done and t >= self.t_max:
                r.done, r.t_done = True, t

    def run(self) -> dict:
        # plan from the start and fly it
        self._replan(0)
        for k, r in enumerate(self.robots):
            if self._in_goal(k, -1):
                r.done, r.success = True, True
            else:
                self._adopt(k)
        tick = 0
        wall0 = time.perf_counter()
        while any(not r.done for r in self.robots):
            tick += 1
            t = tick * self.dt
            self._advance(tick, t)
            self._replan(tick)
        wall = time.perf_counter() - wall0
        lat = np.array(self.tick_ms) if self.tick_ms else np.zeros(1)
        ok = [r for r in self.robots if r.success]
        return {
            "scenarios": len(self.sc),
            "ticks": tick,
            "replans": self.replans,
            "wall_s": round(wall, 3),
            "replans_per_s": round(self.replans / max(wall, 1e-9), 1),
            "ticks_per_s": round(tick / max(wall, 1e-9), 1),
            "plan_p50_ms": round(float(np.percentile(lat, 50)), 3),
            "plan_p99_ms": round(float(np.percentile(lat, 99)), 3),
            "success": len(ok),
            "mean_time_s": round(float(np.mean([r.t_done for r in ok])), 3) if ok else None,
            "mean_cost_flown": round(float(np.mean([r.flown for r in ok])), 4) if ok else None,
            "boxes_added": int(sum(len(r.boxes) - len(s.boxes) for r, s in zip(self.robots, self.sc))),
            "boxes_skipped": int(sum(r.skipped for r in self.robots)),
        }
