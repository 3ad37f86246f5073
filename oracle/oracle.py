"""ctypes front end of the FP64 serial GMT* oracle (``gmt_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the benchmark's CPU-baseline leg, never by the planning library.  It
imports nothing from the library package; problems arrive as plain arrays.

Node numbering: samples 0..n-1, the start x_init is node n (the root).
Status codes: 0 success, 1 no path (open set emptied, Algorithm 1 line 12a),
2 iteration cap reached.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gmt_oracle.c")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "liborc.so")
# a build of the same source to load instead (the sanitizer run of the pins)
LIB_OVERRIDE = os.environ.get("GMT_ORACLE_LIB")

EUCLID, DI, DUBINS = 0, 1, 2
OK, NO_PATH, TIMEOUT = 0, 1, 2
MG_GROUP, MG_ARGMIN, MG_GOAL, MG_ROOT, MG_COLLIDE = 0, 1, 2, 3, 4

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (OpenMP for the pair loops)."""
    os.makedirs(BUILD, exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def build_sanitized(path: str) -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts), for running the pins under them."""
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-shared", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", path, SRC, "-lm"])
    return path


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if LIB_OVERRIDE:
                L = C.CDLL(LIB_OVERRIDE)
            else:
                build()
                L = C.CDLL(LIB)
            P = C.c_void_p
            i32, f64 = C.c_int, C.c_double
            L.orc_free_volume.restype = f64
            L.orc_free_volume.argtypes = [i32, i32, P]
            L.orc_radius.restype = f64
            L.orc_radius.argtypes = [i32, f64, i32, f64]
            L.orc_di_cost.restype = None
            L.orc_di_cost.argtypes = [P, P, P, P]
            L.orc_di_point.restype = None
            L.orc_di_point.argtypes = [P, P, f64, f64, P]
            L.orc_set_turn_radius.restype = None
            L.orc_set_turn_radius.argtypes = [f64]
            L.orc_dubins_cost.restype = None
            L.orc_dubins_cost.argtypes = [P, P, P, P, P, P]
            L.orc_dubins_point.restype = None
            L.orc_dubins_point.argtypes = [P, P, i32, i32, P]
            L.orc_neighbors.restype = i32
            L.orc_neighbors.argtypes = [i32, i32, i32, P, f64, P, P, P, P, P]
            L.orc_transpose.restype = i32
            L.orc_transpose.argtypes = [i32, P, P, P, P]
            L.orc_edge_free.restype = i32
            L.orc_edge_free.argtypes = [i32, i32, i32, P, P, P, i32, f64, i32, i32, i32, f64, P]
            L.orc_plan.restype = i32
            L.orc_plan.argtypes = [i32, i32, i32, P, P, P, C.c_float, i32, P, i32, f64, f64, f64,
                                   i32, i32, P, P, P, P, P, P, P, P, P, P, P, i32, P, P, P, P]
            L.orc_trace_begin.restype = None
            L.orc_trace_begin.argtypes = [P, i32]
            L.orc_trace_end.restype = i32
            L.orc_trace_end.argtypes = []
            L.orc_dijkstra.restype = i32
            L.orc_dijkstra.argtypes = [i32, i32, i32, P, P, P, i32, f64, f64, i32, P, P, P, P,
                                       i32, P]
            _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def free_volume(pdim: int, boxes) -> float:
    b = _f32(boxes).reshape(-1, 2 * pdim)
    return float(lib().orc_free_volume(pdim, b.shape[0], _p(b)))


def radius(d: int, mu: float, n: int, factor: float = 1.1) -> float:
    return float(lib().orc_radius(d, float(mu), int(n), float(factor)))


def euclid_radius(prob) -> float:
    """Theorem 1 radius of a Euclidean problem (mu from its box world)."""
    return radius(prob.dim, free_volume(prob.pdim, prob.boxes), prob.n, prob.r_factor)


def problem_radius(prob) -> float:
    return euclid_radius(prob) if prob.kind == "euclid" else float(prob.r)


def set_turn_radius(rho: float) -> None:
    """Turning radius of the Dubins airplane cost (process-wide in the oracle)."""
    lib().orc_set_turn_radius(float(rho))


def dubins_cost(x0, x1, rho: float):
    """Dubins airplane cost x0 -> x1 (4-vectors x, y, z, heading in turns):
    (cost, planar length, word (+1 left, -1 right, 0 straight) x3, planar
    segment lengths x3)."""
    set_turn_radius(rho)
    a = np.ascontiguousarray(x0, np.float64)
    b = np.ascontiguousarray(x1, np.float64)
    c = np.zeros(1)
    pl = np.zeros(1)
    w = np.zeros(3, np.int32)
    sg = np.zeros(3)
    lib().orc_dubins_cost(_p(a), _p(b), _p(c), _p(pl), _p(w), _p(sg))
    return float(c[0]), float(pl[0]), w, sg


def dubins_point(x0, x1, k: int, K: int, rho: float) -> np.ndarray:
    """Point k of K on the optimal trajectory x0 -> x1 (position)."""
    set_turn_radius(rho)
    a = np.ascontiguousarray(x0, np.float64)
    b = np.ascontiguousarray(x1, np.float64)
    p = np.zeros(3)
    lib().orc_dubins_point(_p(a), _p(b), int(k), int(K), _p(p))
    return p


def di_cost(x0, x1):
    a = np.ascontiguousarray(x0, np.float64)
    b = np.ascontiguousarray(x1, np.float64)
    J = np.zeros(1)
    t = np.zeros(1)
    lib().orc_di_cost(_p(a), _p(b), _p(J), _p(t))
    return float(J[0]), float(t[0])


def di_point(x0, x1, tau: float, t: float) -> np.ndarray:
    a = np.ascontiguousarray(x0, np.float64)
    b = np.ascontiguousarray(x1, np.float64)
    p = np.zeros(3)
    lib().orc_di_point(_p(a), _p(b), float(tau), float(t), _p(p))
    return p


@dataclass
class Csr:
    """In-neighbour table: row x lists y with c(y -> x) < r, ascending y."""
    row_ptr: np.ndarray
    col: np.ndarray
    cost: np.ndarray
    tau: np.ndarray
    margin: float  # least |J - r|/r over solved DI pairs (inf for Euclidean)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def neighbors(samples, kind: int, r: float, turn_radius: Optional[float] = None) -> Csr:
    if kind == DUBINS:
        assert turn_radius is not None, "the Dubins cost needs its turning radius"
        set_turn_radius(turn_radius)
    s = _f32(samples)
    dim, n = s.shape
    rp = np.zeros(n + 1, np.int32)
    L = lib()
    mg = np.zeros(1)
    L.orc_neighbors(n, dim, kind, _p(s), float(r), _p(rp), None, None, None, _p(mg))
    E = int(rp[-1])
    col = np.zeros(max(E, 1), np.int32)
    cost = np.zeros(max(E, 1), np.float64)
    tau = np.zeros(max(E, 1), np.float64)
    L.orc_neighbors(n, dim, kind, _p(s), float(r), _p(rp), _p(col), _p(cost), _p(tau), _p(mg))
    return Csr(rp, col[:E], cost[:E], tau[:E], float(mg[0]))


def transpose(n: int, in_ptr: np.ndarray, in_col: np.ndarray):
    op = np.zeros(n + 1, np.int32)
    oc = np.zeros(max(len(in_col), 1), np.int32)
    ip = np.ascontiguousarray(in_ptr, np.int32)
    ic = np.ascontiguousarray(in_col, np.int32)
    lib().orc_transpose(n, _p(ip), _p(ic), _p(op), _p(oc))
    return op, oc[:len(in_col)]


def out_table(n: int, t: Csr):
    """Out-neighbour table with costs/arrival times (transpose of ``t``)."""
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(t.row_ptr))
    order = np.lexsort((src, t.col))
    col = src[order].astype(np.int32)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, t.col.astype(np.int64) + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return rp, col, np.ascontiguousarray(t.cost[order]), np.ascontiguousarray(t.tau[order])


@dataclass
class Plan:
    status: int
    parent: np.ndarray
    cost: np.ndarray
    group_iter: np.ndarray
    added_iter: np.ndarray
    path: np.ndarray
    path_cost: float
    iters: int
    margins: np.ndarray
    # per non-empty iteration: i, |open|, |G_i|, |C|, C in obstacles, lazy-check
    # failures, nodes added (plan(..., trace=True) only)
    trace: Optional[np.ndarray] = None


TRACE_FIELDS = ("iter", "open", "group", "candidates", "candidates_in_obstacles", "check_failures", "added")


def kind_of(prob) -> int:
    return {"di": DI, "dubins": DUBINS}.get(prob.kind, EUCLID)


def plan(prob, r: float, table: Optional[Csr] = None, lam: Optional[float] = None,
         max_iters: int = 0, trace: bool = False) -> Plan:
    """Run Algorithm 1 on ``prob`` with radius ``r`` (table built when absent).
    ``trace``: also return one record per iteration with a non-empty group
    (columns TRACE_FIELDS)."""
    kind = kind_of(prob)
    if kind == DUBINS:
        set_turn_radius(prob.turn_radius)
    s = _f32(prob.samples)
    dim, n = s.shape
    if table is None:
        table = neighbors(s, kind, r, prob.turn_radius)
    if kind == EUCLID:
        op, oc = table.row_ptr, table.col
    else:
        op, oc = transpose(n, table.row_ptr, table.col)
    N = n + 1
    parent = np.zeros(N, np.int32)
    cost = np.zeros(N, np.float64)
    gi = np.zeros(N, np.int32)
    ai = np.zeros(N, np.int32)
    path = np.zeros(N, np.int32)
    plen = np.zeros(1, np.int32)
    pcost = np.zeros(1, np.float64)
    iters = np.zeros(1, np.int32)
    mg = np.zeros(8, np.float64)
    xi = _f32(prob.x_init)
    gc = _f32(prob.goal_center)
    bx = _f32(prob.boxes).reshape(-1, 2 * prob.pdim)
    ip = np.ascontiguousarray(table.row_ptr, np.int32)
    ic = np.ascontiguousarray(table.col, np.int32)
    cc = np.ascontiguousarray(table.cost, np.float64)
    tt = np.ascontiguousarray(table.tau, np.float64)
    op = np.ascontiguousarray(op, np.int32)
    oc = np.ascontiguousarray(oc, np.int32)
    tr = np.zeros((N + 1, len(TRACE_FIELDS)), np.int32) if trace else None
    if trace:
        lib().orc_trace_begin(_p(tr), tr.shape[0])
    st = lib().orc_plan(n, dim, kind, _p(s), _p(xi), _p(gc), C.c_float(prob.goal_radius),
                        prob.pdim, _p(bx), bx.shape[0], float(r),
                        float(prob.lam if lam is None else lam), float(prob.step),
                        int(prob.traj_points), int(max_iters), _p(ip), _p(ic), _p(cc),
                        _p(tt) if kind == DI else None, _p(op), _p(oc), _p(parent), _p(cost),
                        _p(gi), _p(ai), _p(path), N, _p(plen), _p(pcost), _p(iters), _p(mg))
    if trace:
        k = lib().orc_trace_end()
        tr = tr[:min(k, tr.shape[0])].copy()
    if st < 0:
        raise ValueError("oracle rejected the problem (status %d)" % st)
    return Plan(int(st), parent, cost, gi, ai, path[:int(plen[0])].copy(), float(pcost[0]),
                int(iters[0]), mg, tr)


def dijkstra(prob, r: float, table: Optional[Csr] = None, only_clear: bool = False) -> np.ndarray:
    """Least cost from the root over the collision-free disk graph ([n+1])."""
    kind = kind_of(prob)
    if kind == DUBINS:
        set_turn_radius(prob.turn_radius)
    s = _f32(prob.samples)
    dim, n = s.shape
    if table is None:
        table = neighbors(s, kind, r, prob.turn_radius)
    if kind == EUCLID:
        op, oc, ocost, otau = table.row_ptr, table.col, table.cost, table.tau
    else:
        op, oc, ocost, otau = out_table(n, table)
    op = np.ascontiguousarray(op, np.int32)
    oc = np.ascontiguousarray(oc, np.int32)
    ocost = np.ascontiguousarray(ocost, np.float64)
    otau = np.ascontiguousarray(otau, np.float64)
    dist = np.zeros(n + 1, np.float64)
    xi = _f32(prob.x_init)
    bx = _f32(prob.boxes).reshape(-1, 2 * prob.pdim)
    lib().orc_dijkstra(n, dim, kind, _p(s), _p(xi), _p(bx), bx.shape[0], float(r),
                       float(prob.step), int(prob.traj_points), _p(op), _p(oc), _p(ocost),
                       _p(otau), int(bool(only_clear)), _p(dist))
    return dist


def edge_free(prob, y: int, x: int, tau: float = 0.0):
    """Lazy check of edge y -> x; returns (free, margin)."""
    if kind_of(prob) == DUBINS:
        set_turn_radius(prob.turn_radius)
    s = _f32(prob.samples)
    dim, n = s.shape
    xi = _f32(prob.x_init)
    bx = _f32(prob.boxes).reshape(-1, 2 * prob.pdim)
    mg = np.zeros(1)
    ok = lib().orc_edge_free(n, dim, kind_of(prob), _p(s), _p(xi), _p(bx), bx.shape[0],
                             float(prob.step), int(prob.traj_points), int(y), int(x), float(tau),
                             _p(mg))
    return bool(ok), float(mg[0])


def min_margin(p: Plan, kind: int) -> float:
    """Least relative decision margin of a plan (collision margin excluded)."""
    keys = [MG_GROUP, MG_ARGMIN, MG_GOAL] + ([MG_ROOT] if kind != EUCLID else [])
    return float(min(p.margins[k] for k in keys))


def decisive(p: Plan, kind: int, rel: float = 1e-6, collide_abs: float = 1e-5) -> bool:
    """True when every decision of the run is separated by at least ``rel``
    (relative) and, for the double integrator, every lazy check by at least
    ``collide_abs`` in position (and, for the Dubins airplane, every point
    count by as much in path length)."""
    if min_margin(p, kind) < rel:
        return False
    if kind != EUCLID and p.margins[MG_COLLIDE] < collide_abs:
        return False
    return True
