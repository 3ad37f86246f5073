"""ctypes binding of ``libgmt.so`` (declared in ``include/gmt.h``).

Argument marshalling only: every planning step runs in the library's HIP
kernels.  Functions carry the C names (``gmt_build_neighbors``, ``gmt_plan``,
``gmt_plan_batch``, ...).  Device buffers are torch tensors on the current
GPU; torch's caching allocator backs the library's device allocations
(``gmt_set_allocator``) and torch streams are passed as ``hipStream_t``.

Loading never compiles: ``lib()`` raises when the library has not been built
(``build_library()``, also run by ``__graft_entry__.build()``).
"""

from __future__ import annotations

import atexit
import ctypes as C
import os
import struct
import subprocess
import sys
import threading
import weakref
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD, "libgmt.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

GMT_OK, GMT_NO_PATH, GMT_ETIMEOUT = 0, 1, 2
GMT_EINVAL, GMT_ENOMEM, GMT_EDEVICE, GMT_EBUSY = -1, -2, -3, -4
GMT_COST_EUCLIDEAN, GMT_COST_DOUBLE_INTEGRATOR, GMT_COST_DUBINS_AIRPLANE = 0, 1, 2
STATUS_NAMES = {0: "GMT_OK", 1: "GMT_NO_PATH", 2: "GMT_ETIMEOUT", -1: "GMT_EINVAL",
                -2: "GMT_ENOMEM", -3: "GMT_EDEVICE", -4: "GMT_EBUSY"}

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# symbols the header declares (checked by the CPU tests)
EXPORTS = ["gmt_set_allocator", "gmt_build_neighbors", "gmt_build_neighbors_ex", "gmt_sample_halton", "gmt_roadmap_from_csr", "gmt_roadmap_info", "gmt_roadmap_bytes",
           "gmt_roadmap_save", "gmt_roadmap_load",
           "gmt_roadmap_export", "gmt_roadmap_free", "gmt_plan", "gmt_plan_noalloc", "gmt_plan_batch",
           "gmt_last_work", "gmt_last_trace", "gmt_last_build", "gmt_profile_enable", "gmt_profile_read",
           "gmt_engine_create", "gmt_engine_submit", "gmt_engine_poll", "gmt_engine_poll_any", "gmt_engine_cancel",
           "gmt_engine_set_budget", "gmt_engine_get_stats", "gmt_engine_destroy",
           "gmt_batch_prepare", "gmt_batch_run", "gmt_batch_free",
           "gmt_autotune", "gmt_autotune_build", "gmt_tune_lookup", "gmt_tune_store", "gmt_tune_clear", "gmt_tune_save",
           "gmt_tune_load", "gmt_shutdown", "gmt_last_error", "gmt_version", "gmt_steady_ns"]


def pdim_of(kind: int, dim: int) -> int:
    """Position dimensions (those boxes and the goal constrain): all of a
    Euclidean state, the first 3 of a double-integrator or Dubins state."""
    return dim if kind == GMT_COST_EUCLIDEAN else 3


class GmtError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s (%s): %s" % (what, STATUS_NAMES.get(status, status), last_error()))
        self.status = status


def sources() -> List[str]:
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
            if f.endswith((".hip", ".hpp"))] + [os.path.join(INCLUDE, f) for f in ("gmt.h", "gmt_sampler.h")]


def build_library(force: bool = True) -> str:
    """Compile libgmt.so for gfx950 with hipcc (in-tree, under ``_build/``)."""
    os.makedirs(BUILD, exist_ok=True)
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(p) for p in sources())
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    units = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")]
    cmd = ["hipcc"] + HIPCC_FLAGS + ["-o", tmp] + units
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


# ---------------------------------------------------------------------------
# structs
# ---------------------------------------------------------------------------
class gmt_allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)),
                ("ctx", C.c_void_p)]


class gmt_cost_params(C.Structure):
    _fields_ = [("turn_radius", C.c_double), ("row_slots", C.c_int32), ("build_tile", C.c_int32)]


class gmt_goal(C.Structure):
    _fields_ = [("center", C.c_float * 6), ("radius", C.c_float), ("ndims", C.c_int32)]


class gmt_plan_opts(C.Structure):
    _fields_ = [("edge_step", C.c_double), ("traj_points", C.c_int32), ("max_iters", C.c_int32),
                ("team_wgs", C.c_int32), ("lanes", C.c_int32), ("threads", C.c_int32),
                ("trace", C.c_int32)]


class gmt_trace_rec(C.Structure):
    _fields_ = [("iter", C.c_int32), ("open", C.c_int32), ("group", C.c_int32), ("goal_in_group", C.c_int32),
                ("candidates", C.c_int32), ("check_failures", C.c_int32), ("added", C.c_int32),
                ("reserved", C.c_int32), ("select_ns", C.c_int64), ("frontier_ns", C.c_int64),
                ("connect_ns", C.c_int64), ("check_ns", C.c_int64)]


# numpy view of gmt_trace_rec
TRACE_DTYPE = np.dtype([(k, np.int32 if t is C.c_int32 else np.int64) for k, t in gmt_trace_rec._fields_])


class gmt_problem(C.Structure):
    _fields_ = [("roadmap", C.c_void_p), ("x_init", C.POINTER(C.c_float)), ("goal", gmt_goal),
                ("boxes", C.POINTER(C.c_float)), ("m", C.c_int32), ("lambda_", C.c_double),
                ("edge_step", C.c_double)]


class gmt_work(C.Structure):
    _fields_ = [("out_edges", C.c_int64), ("in_edges", C.c_int64), ("candidates", C.c_int64),
                ("commits", C.c_int64), ("open_entries", C.c_int64), ("iterations", C.c_int64),
                ("setup_ns", C.c_int64), ("select_ns", C.c_int64), ("frontier_ns", C.c_int64),
                ("connect_ns", C.c_int64), ("check_ns", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class gmt_build_info(C.Structure):
    _fields_ = [("edges", C.c_int64), ("pairs_tested", C.c_int64), ("pairs_solved", C.c_int64),
                ("kernel_ms", C.c_double), ("segments", C.c_int32), ("tile", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gmt_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("path_len", C.c_int32),
                ("path_cap", C.c_int32), ("path_cost", C.c_double),
                ("path", C.POINTER(C.c_int32)), ("d_parent", C.c_void_p), ("d_cost", C.c_void_p),
                ("d_group_iter", C.c_void_p), ("d_added_iter", C.c_void_p), ("work", gmt_work),
                ("submit_ns", C.c_int64), ("done_ns", C.c_int64)]


class gmt_batch_opts(C.Structure):
    _fields_ = [("plan", gmt_plan_opts), ("workgroups", C.c_int32)]


class gmt_engine_opts(C.Structure):
    _fields_ = [("budget_bytes", C.c_size_t), ("slots", C.c_int32), ("max_batch", C.c_int32),
                ("queue_cap", C.c_int32), ("workgroups", C.c_int32), ("plan", gmt_plan_opts),
                ("batch_only", C.c_int32)]


class gmt_engine_stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "completed", "cancelled", "rejected", "batches",
                                         "queued", "inflight_bytes", "peak_inflight_bytes",
                                         "peak_inflight_requests", "lone_launches", "early_completions")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lock = threading.Lock()
_lib = None
_alloc_keep = None
# open handles (roadmaps, prepared batches, engines, samplers), closed at exit
_live = weakref.WeakSet()


def _track(obj) -> None:
    _live.add(obj)


def _at_exit() -> None:
    """Close every handle still open while torch (whose allocator backs the
    library's device memory) is alive, then release the library's pools
    (gmt_shutdown).  Finalizers that run later do nothing."""
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass
    if _lib is not None:
        _lib.gmt_shutdown()


class gmt_tune_shape(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("n", C.c_int32), ("m", C.c_int32),
                ("batch", C.c_int32)]


class gmt_build_tune(C.Structure):
    _fields_ = [("tile", C.c_int32), ("candidates", C.c_int32), ("rejected", C.c_int32), ("pad", C.c_int32),
                ("ms", C.c_double), ("default_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


GMT_BUILD_TILES = 4


class gmt_tune_choice(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("team_wgs", C.c_int32), ("workgroups", C.c_int32),
                ("threads", C.c_int32), ("ms", C.c_double), ("default_ms", C.c_double),
                ("candidates", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libgmt.so is not built (%s); run __graft_entry__.build() or "
                                   "paper_1705_02403_amd.gmt.build_library()" % LIB_PATH)
            L = C.CDLL(LIB_PATH)
            P, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
            L.gmt_set_allocator.argtypes = [C.POINTER(gmt_allocator)]
            L.gmt_build_neighbors.argtypes = [P, i32, i32, i32, f64, P, C.POINTER(P)]
            L.gmt_build_neighbors_ex.argtypes = [P, i32, i32, i32, f64, C.POINTER(gmt_cost_params), P, C.POINTER(P)]
            L.gmt_roadmap_save.argtypes = [P, C.c_char_p, P]
            L.gmt_roadmap_load.argtypes = [C.c_char_p, P, C.POINTER(P)]
            L.gmt_sample_halton.argtypes = [i32, i32, i32, i64, P, i32, P, C.POINTER(i64), P]
            L.gmt_roadmap_from_csr.argtypes = [P, i32, i32, i32, f64, P, P, P, P, P, C.POINTER(P)]
            L.gmt_roadmap_info.argtypes = [P, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                           C.POINTER(i64)]
            L.gmt_roadmap_bytes.argtypes = [P, C.POINTER(C.c_int64)]
            L.gmt_roadmap_export.argtypes = [P, P, P, P, P, P]
            L.gmt_roadmap_free.argtypes = [P]
            L.gmt_plan.argtypes = [P, P, C.POINTER(gmt_goal), P, i32, f64, C.POINTER(gmt_plan_opts),
                                   P, P, P, P, P, i32, C.POINTER(i32), C.POINTER(f64),
                                   C.POINTER(i32), P]
            L.gmt_plan_noalloc.argtypes = L.gmt_plan.argtypes
            L.gmt_plan_batch.argtypes = [C.POINTER(gmt_problem), i32, C.POINTER(gmt_batch_opts),
                                         C.POINTER(gmt_result), P]
            L.gmt_last_work.argtypes = [C.POINTER(gmt_work)]
            L.gmt_last_trace.argtypes = [i32, P, i32, C.POINTER(i32)]
            L.gmt_last_build.argtypes = [C.POINTER(gmt_build_info)]
            L.gmt_profile_enable.argtypes = [i32]
            L.gmt_profile_read.argtypes = [C.POINTER(f64), C.POINTER(i64)]
            L.gmt_engine_create.argtypes = [C.POINTER(gmt_engine_opts), C.POINTER(P)]
            L.gmt_engine_submit.argtypes = [P, C.POINTER(gmt_problem), i32, C.POINTER(i64)]
            L.gmt_engine_poll.argtypes = [P, i64, i32, C.POINTER(gmt_result), P, i32]
            L.gmt_engine_poll_any.argtypes = [P, i32, C.POINTER(i64), C.POINTER(gmt_result), P, i32]
            L.gmt_engine_cancel.argtypes = [P, i64]
            L.gmt_engine_set_budget.argtypes = [P, C.c_size_t]
            L.gmt_engine_get_stats.argtypes = [P, C.POINTER(gmt_engine_stats)]
            L.gmt_engine_destroy.argtypes = [P]
            L.gmt_batch_prepare.argtypes = [C.POINTER(gmt_problem), i32, C.POINTER(gmt_batch_opts), C.POINTER(P),
                                            P]
            L.gmt_batch_run.argtypes = [P, C.POINTER(gmt_result), P]
            L.gmt_batch_free.argtypes = [P]
            L.gmt_autotune.argtypes = [C.POINTER(gmt_problem), i32, i32, C.POINTER(gmt_plan_opts), i32,
                                       C.POINTER(gmt_tune_choice), P]
            L.gmt_tune_lookup.argtypes = [C.POINTER(gmt_tune_shape), C.POINTER(gmt_tune_choice)]
            L.gmt_autotune_build.argtypes = [P, i32, i32, f64, i32, C.POINTER(gmt_build_tune), P]
            L.gmt_tune_store.argtypes = [C.POINTER(gmt_tune_shape), C.POINTER(gmt_tune_choice)]
            L.gmt_tune_clear.argtypes = []
            L.gmt_tune_save.argtypes = [C.c_char_p]
            L.gmt_tune_load.argtypes = [C.c_char_p]
            L.gmt_shutdown.argtypes = []
            L.gmt_last_error.restype = C.c_char_p
            L.gmt_version.restype = C.c_char_p
            L.gmt_steady_ns.restype = i64
            for name in EXPORTS:
                if name not in ("gmt_last_error", "gmt_version", "gmt_steady_ns"):
                    getattr(L, name).restype = i32
            _lib = L
            atexit.register(_at_exit)
    return _lib


def last_error() -> str:
    try:
        return lib().gmt_last_error().decode()
    except Exception:  # pragma: no cover - library absent
        return ""


def gmt_version() -> str:
    return lib().gmt_version().decode()


def gmt_last_work() -> dict:
    w = gmt_work()
    _check(lib().gmt_last_work(C.byref(w)), "gmt_last_work")
    return w.as_dict()


def gmt_last_trace(query: int = 0) -> np.ndarray:
    """Per-iteration records (TRACE_DTYPE) of query ``query`` of the last
    traced gmt_plan / gmt_plan_batch call on this thread."""
    n = C.c_int32()
    _check(lib().gmt_last_trace(int(query), None, 0, C.byref(n)), "gmt_last_trace")
    out = np.zeros(int(n.value), TRACE_DTYPE)
    if len(out):
        _check(lib().gmt_last_trace(int(query), out.ctypes.data, len(out), C.byref(n)), "gmt_last_trace")
    return out


def gmt_last_build() -> dict:
    """Record of the last gmt_build_neighbors on this thread (kernel_ms is
    measured only while profiling is enabled)."""
    b = gmt_build_info()
    _check(lib().gmt_last_build(C.byref(b)), "gmt_last_build")
    return b.as_dict()


def gmt_profile_enable(enable: bool = True) -> None:
    _check(lib().gmt_profile_enable(int(bool(enable))), "gmt_profile_enable")


def gmt_profile_read():
    """(kernel milliseconds, launches) since the last read."""
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().gmt_profile_read(C.byref(ms), C.byref(n)), "gmt_profile_read")
    return float(ms.value), int(n.value)


def _check(st: int, what: str, ok=(GMT_OK,)) -> int:
    if st not in ok:
        raise GmtError(st, what)
    return st


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _host_f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def use_torch_allocator() -> None:
    """Route the library's device allocations through torch's caching allocator.

    The callbacks are created once and kept for the life of the process: every
    device buffer remembers the allocator that produced it and calls its free
    callback later, so the callbacks must outlive all buffers."""
    global _alloc_keep
    import torch

    if _alloc_keep is None:
        @C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
        def _alloc(nbytes, ctx, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0) or None)
            except Exception:
                return None

        @C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
        def _free(ptr, ctx, stream):
            torch.cuda.caching_allocator_delete(int(ptr))

        _alloc_keep = (gmt_allocator(_alloc, _free, None), _alloc, _free)
    _check(lib().gmt_set_allocator(C.byref(_alloc_keep[0])), "gmt_set_allocator")


# ---------------------------------------------------------------------------
# roadmaps
# ---------------------------------------------------------------------------
class Roadmap:
    """Owns a ``gmt_roadmap_t`` handle."""

    def __init__(self, handle: int, n: int, dim: int, kind: int, r: float):
        self.handle = C.c_void_p(handle)
        self.n, self.dim, self.kind, self.r = n, dim, kind, r
        _track(self)

    @property
    def nnz(self) -> int:
        n, d, k = C.c_int32(), C.c_int32(), C.c_int32()
        e = C.c_int64()
        _check(lib().gmt_roadmap_info(self.handle, C.byref(n), C.byref(d), C.byref(k), C.byref(e)),
               "gmt_roadmap_info")
        return int(e.value)

    @property
    def device_bytes(self) -> int:
        """Device memory the roadmap holds."""
        b = C.c_int64()
        _check(lib().gmt_roadmap_bytes(self.handle, C.byref(b)), "gmt_roadmap_bytes")
        return int(b.value)

    def export(self, stream=None):
        """(row_ptr, col, cost, tau) of the in-neighbour table as numpy arrays."""
        E = self.nnz
        rp = np.zeros(self.n + 1, np.int32)
        col = np.zeros(max(E, 1), np.int32)
        cost = np.zeros(max(E, 1), np.float64)
        tau = np.zeros(max(E, 1), np.float64) if self.kind == GMT_COST_DOUBLE_INTEGRATOR else None
        _check(lib().gmt_roadmap_export(self.handle, rp.ctypes.data, col.ctypes.data,
                                        cost.ctypes.data, None if tau is None else tau.ctypes.data,
                                        _stream(stream)), "gmt_roadmap_export")
        return rp, col[:E], cost[:E], (None if tau is None else tau[:E])

    def save(self, path: str, stream=None) -> None:
        """Checkpoint the roadmap to `path` (gmt_roadmap_save)."""
        _check(lib().gmt_roadmap_save(self.handle, os.fsencode(path), _stream(stream)), "gmt_roadmap_save")

    def free(self) -> None:
        if self.handle:
            lib().gmt_roadmap_free(self.handle)
            self.handle = C.c_void_p(None)

    close = free

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            if sys.is_finalizing():
                return  # closed by the exit handler, or left to the process exit
            self.free()
        except Exception:
            pass


def gmt_build_neighbors(samples, kind: int, r_n: float, stream=None, turn_radius=None,
                        row_slots=None, build_tile=None) -> Roadmap:
    """samples: CUDA float32 tensor [dim][n] (SoA) on the 2^-20 grid;
    turn_radius: the Dubins airplane's; row_slots: scratch entries per row of
    the asymmetric kinds' build; build_tile: the Euclidean build's tile shape
    (1..GMT_BUILD_TILES) (all three through gmt_build_neighbors_ex)."""
    import torch
    assert samples.is_cuda and samples.dtype == torch.float32 and samples.dim() == 2
    s = samples.contiguous()
    dim, n = int(s.shape[0]), int(s.shape[1])
    h = C.c_void_p()
    if turn_radius is None and row_slots is None and build_tile is None:
        _check(lib().gmt_build_neighbors(s.data_ptr(), n, dim, int(kind), float(r_n), _stream(stream),
                                         C.byref(h)), "gmt_build_neighbors")
    else:
        prm = gmt_cost_params(float(turn_radius or 0.0), int(row_slots or 0), int(build_tile or 0))
        _check(lib().gmt_build_neighbors_ex(s.data_ptr(), n, dim, int(kind), float(r_n), C.byref(prm),
                                            _stream(stream), C.byref(h)), "gmt_build_neighbors_ex")
    return Roadmap(h.value, n, dim, int(kind), float(r_n))


def gmt_roadmap_load(path: str, stream=None) -> Roadmap:
    """A roadmap checkpointed with Roadmap.save (gmt_roadmap_load)."""
    h = C.c_void_p()
    _check(lib().gmt_roadmap_load(os.fsencode(path), _stream(stream), C.byref(h)), "gmt_roadmap_load")
    n, dim, kind, nnz = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib().gmt_roadmap_info(h, C.byref(n), C.byref(dim), C.byref(kind), C.byref(nnz)), "gmt_roadmap_info")
    with open(path, "rb") as f:  # the radius from the file's header (magic, 6 int32, int64, r)
        r = struct.unpack_from("<8s6iqd", f.read(48))[8]
    return Roadmap(h.value, int(n.value), int(dim.value), int(kind.value), float(r))


def gmt_sample_halton(n: int, dim: int, kind: int, first: int = 1, boxes=None, out=None, stream=None):
    """Halton sample set on the device: returns (CUDA float32 [dim][n], next
    index).  `boxes` host [m][2*pdim]; `out` an optional [dim][n] tensor."""
    import torch
    pd = pdim_of(kind, dim)
    bx = _host_f32(boxes if boxes is not None else np.zeros((0, 2 * pd), np.float32)).reshape(-1)
    m = int(bx.size // (2 * pd)) if bx.size else 0
    if out is None:
        out = torch.empty((dim, max(n, 0)), dtype=torch.float32, device=torch.device("cuda", torch.cuda.current_device()))
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= dim * max(n, 0)
    nxt = C.c_int64()
    _check(lib().gmt_sample_halton(int(n), int(dim), int(kind), int(first), bx.ctypes.data if m else None, m,
                                   out.data_ptr() if n > 0 else None, C.byref(nxt), _stream(stream)),
           "gmt_sample_halton")
    return out, int(nxt.value)


def gmt_roadmap_from_csr(samples, kind: int, r_n: float, row_ptr, col, cost, tau=None,
                         stream=None) -> Roadmap:
    """Host arrays: samples [dim][n] float32, CSR int32/int32/float64 (+ tau float64)."""
    s = _host_f32(samples)
    dim, n = s.shape
    rp = np.ascontiguousarray(row_ptr, np.int32)
    cl = np.ascontiguousarray(col, np.int32)
    cs = np.ascontiguousarray(cost, np.float64)
    tt = None if tau is None else np.ascontiguousarray(tau, np.float64)
    h = C.c_void_p()
    _check(lib().gmt_roadmap_from_csr(s.ctypes.data, n, dim, int(kind), float(r_n), rp.ctypes.data,
                                      cl.ctypes.data if len(cl) else None,
                                      cs.ctypes.data if len(cs) else None,
                                      None if tt is None or not len(tt) else tt.ctypes.data,
                                      _stream(stream), C.byref(h)), "gmt_roadmap_from_csr")
    return Roadmap(h.value, n, dim, int(kind), float(r_n))


# ---------------------------------------------------------------------------
# planning
# ---------------------------------------------------------------------------
@dataclass
class PlanResult:
    status: int
    path: np.ndarray
    path_cost: float
    iters: int
    parent: object = None      # torch tensors when requested
    cost: object = None
    group_iter: object = None
    added_iter: object = None
    work: Optional[dict] = None
    trace: Optional[np.ndarray] = None  # per-iteration records when opts.trace > 0


def make_goal(center: Sequence[float], radius: float, ndims: int) -> gmt_goal:
    g = gmt_goal()
    for a, c in enumerate(center):
        g.center[a] = float(c)
    g.radius = float(radius)
    g.ndims = int(ndims)
    return g


def make_opts(edge_step: float = 0.0, traj_points: int = 16, max_iters: int = 0,
              team_wgs: int = 0, lanes: int = 0, threads: int = 0, trace: int = 0) -> gmt_plan_opts:
    return gmt_plan_opts(float(edge_step), int(traj_points), int(max_iters), int(team_wgs),
                         int(lanes), int(threads), int(trace))


def gmt_plan(rm: Roadmap, x_init, goal: gmt_goal, boxes, lam: float, opts: gmt_plan_opts,
             outputs: bool = True, stream=None, path_cap: int = 4096) -> PlanResult:
    """One query; returns the path and (optionally) the tree as device tensors."""
    import torch
    xi = _host_f32(x_init)
    bx = _host_f32(boxes).reshape(-1)
    pd = pdim_of(rm.kind, rm.dim)
    m = int(bx.size // (2 * pd)) if bx.size else 0
    N = rm.n + 1
    dev = torch.device("cuda", torch.cuda.current_device())
    par = cst = gi = ai = None
    if outputs:
        par = torch.empty(N, dtype=torch.int32, device=dev)
        cst = torch.empty(N, dtype=torch.float64, device=dev)
        gi = torch.empty(N, dtype=torch.int32, device=dev)
        ai = torch.empty(N, dtype=torch.int32, device=dev)
    path = np.zeros(path_cap, np.int32)
    plen = C.c_int32()
    pcost = C.c_double()
    iters = C.c_int32()
    st = lib().gmt_plan(rm.handle, xi.ctypes.data, C.byref(goal), bx.ctypes.data if m else None, m,
                        float(lam), C.byref(opts), _ptr(par), _ptr(cst), _ptr(gi), _ptr(ai),
                        path.ctypes.data, path_cap, C.byref(plen), C.byref(pcost), C.byref(iters),
                        _stream(stream))
    _check(st, "gmt_plan", ok=(GMT_OK, GMT_NO_PATH, GMT_ETIMEOUT))
    L = int(plen.value) if st == GMT_OK else 0
    return PlanResult(int(st), path[:min(L, path_cap)].copy(), float(pcost.value), int(iters.value),
                      par, cst, gi, ai, gmt_last_work(), gmt_last_trace(0) if opts.trace > 0 else None)


def gmt_plan_noalloc(rm: Roadmap, x_init, goal: gmt_goal, boxes, lam: float, opts: gmt_plan_opts,
                     parent, cost, group_iter, added_iter, stream=None, path_cap: int = 4096) -> PlanResult:
    """One query solved without device allocation: the caller supplies the four
    device tree arrays (n+1 entries: int32, float64, int32, int32); the
    library's static device array holds the workspace."""
    N = rm.n + 1
    for t, dt in ((parent, "torch.int32"), (cost, "torch.float64"), (group_iter, "torch.int32"),
                  (added_iter, "torch.int32")):
        if t is None or str(t.dtype) != dt or t.numel() < N or not t.is_cuda or not t.is_contiguous():
            raise ValueError("gmt_plan_noalloc needs contiguous device arrays of n+1 entries (%s)" % dt)
    xi = _host_f32(x_init)
    bx = _host_f32(boxes).reshape(-1)
    pd = pdim_of(rm.kind, rm.dim)
    m = int(bx.size // (2 * pd)) if bx.size else 0
    path = np.zeros(path_cap, np.int32)
    plen = C.c_int32()
    pcost = C.c_double()
    iters = C.c_int32()
    st = lib().gmt_plan_noalloc(rm.handle, xi.ctypes.data, C.byref(goal), bx.ctypes.data if m else None, m,
                                float(lam), C.byref(opts), _ptr(parent), _ptr(cost), _ptr(group_iter),
                                _ptr(added_iter), path.ctypes.data, path_cap, C.byref(plen), C.byref(pcost),
                                C.byref(iters), _stream(stream))
    _check(st, "gmt_plan_noalloc", ok=(GMT_OK, GMT_NO_PATH, GMT_ETIMEOUT))
    L = int(plen.value) if st == GMT_OK else 0
    return PlanResult(int(st), path[:min(L, path_cap)].copy(), float(pcost.value), int(iters.value),
                      parent, cost, group_iter, added_iter, gmt_last_work())


@dataclass
class BatchQuery:
    roadmap: Roadmap
    x_init: np.ndarray
    goal: gmt_goal
    boxes: np.ndarray
    lam: float
    edge_step: float = 0.0  # > 0: this query's Euclidean edge step


class PreparedBatch:
    """Queries marshalled once into ABI structs; ``run()`` solves them with one
    ``gmt_plan_batch`` call and can be repeated without re-marshalling."""

    def __init__(self, queries: Sequence[BatchQuery], opts: gmt_plan_opts, workgroups: int = 0,
                 outputs: bool = False, path_cap: int = 1024):
        import torch
        k = len(queries)
        self.k = k
        self.probs = (gmt_problem * k)()
        self.res = (gmt_result * k)()
        self.keep = []
        self.paths = []
        self.outs = []
        dev = torch.device("cuda", torch.cuda.current_device())
        for j, q in enumerate(queries):
            xi = _host_f32(q.x_init)
            bx = _host_f32(q.boxes).reshape(-1)
            pd = pdim_of(q.roadmap.kind, q.roadmap.dim)
            m = int(bx.size // (2 * pd)) if bx.size else 0
            path = np.zeros(path_cap, np.int32)
            self.keep += [xi, bx]
            self.paths.append(path)
            self.probs[j].roadmap = q.roadmap.handle
            self.probs[j].x_init = xi.ctypes.data_as(C.POINTER(C.c_float))
            self.probs[j].goal = q.goal
            self.probs[j].boxes = bx.ctypes.data_as(C.POINTER(C.c_float)) if m else None
            self.probs[j].m = m
            self.probs[j].lambda_ = float(q.lam)
            self.probs[j].edge_step = float(q.edge_step)
            self.res[j].path = path.ctypes.data_as(C.POINTER(C.c_int32))
            self.res[j].path_cap = path_cap
            o = [None] * 4
            if outputs:
                N = q.roadmap.n + 1
                o = [torch.empty(N, dtype=torch.int32, device=dev),
                     torch.empty(N, dtype=torch.float64, device=dev),
                     torch.empty(N, dtype=torch.int32, device=dev),
                     torch.empty(N, dtype=torch.int32, device=dev)]
                self.res[j].d_parent, self.res[j].d_cost = o[0].data_ptr(), o[1].data_ptr()
                self.res[j].d_group_iter, self.res[j].d_added_iter = o[2].data_ptr(), o[3].data_ptr()
            self.outs.append(o)
        self.bo = gmt_batch_opts(opts, int(workgroups))
        self.path_cap = path_cap

    def run(self, stream=None) -> None:
        _check(lib().gmt_plan_batch(self.probs, self.k, C.byref(self.bo), self.res, _stream(stream)),
               "gmt_plan_batch")
        # records live in thread-local library state until the next call
        self.traces = [gmt_last_trace(j) for j in range(self.k)] if self.bo.plan.trace > 0 else None

    def statuses(self) -> np.ndarray:
        return np.array([self.res[j].status for j in range(self.k)], np.int32)

    def results(self) -> List[PlanResult]:
        out = []
        traces = getattr(self, "traces", None)
        for j in range(self.k):
            r = self.res[j]
            L = int(r.path_len) if r.status == GMT_OK else 0
            out.append(PlanResult(int(r.status), self.paths[j][:min(L, self.path_cap)].copy(),
                                  float(r.path_cost), int(r.iters), *self.outs[j],
                                  work=r.work.as_dict(), trace=traces[j] if traces else None))
        return out


class GraphBatch(PreparedBatch):
    """Queries staged once by the library (gmt_batch_prepare) with their launch
    captured as a HIP graph; ``run()`` replays it (gmt_batch_run)."""

    def __init__(self, queries: Sequence[BatchQuery], opts: gmt_plan_opts, workgroups: int = 0,
                 path_cap: int = 1024, team_wgs: int = 0, stream=None):
        super().__init__(queries, opts, workgroups, False, path_cap)
        if team_wgs:
            self.bo.plan.team_wgs = int(team_wgs)
        h = C.c_void_p()
        _check(lib().gmt_batch_prepare(self.probs, self.k, C.byref(self.bo), C.byref(h), _stream(stream)),
               "gmt_batch_prepare")
        self.handle = h
        _track(self)

    def run(self, stream=None) -> None:
        _check(lib().gmt_batch_run(self.handle, self.res, _stream(stream)), "gmt_batch_run")

    def close(self) -> None:
        if self.handle:
            lib().gmt_batch_free(self.handle)
            self.handle = C.c_void_p(None)

    def __del__(self):  # pragma: no cover
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass


def gmt_plan_batch(queries: Sequence[BatchQuery], opts: gmt_plan_opts, workgroups: int = 0,
                   outputs: bool = False, stream=None, path_cap: int = 1024) -> List[PlanResult]:
    """Solve queries in one persistent launch; returns a list of PlanResult."""
    pb = PreparedBatch(queries, opts, workgroups, outputs, path_cap)
    pb.run(stream)
    return pb.results()


# ---------------------------------------------------------------------------
# autotuner
# ---------------------------------------------------------------------------
def gmt_autotune(queries: Sequence[BatchQuery], opts: gmt_plan_opts, single: bool = False,
                 reps: int = 3, stream=None) -> dict:
    """Time every launch configuration on ``queries`` and cache the fastest
    for their shape bucket (see gmt_autotune in the header)."""
    pb = PreparedBatch(queries, opts)
    out = gmt_tune_choice()
    _check(lib().gmt_autotune(pb.probs, pb.k, int(bool(single)), C.byref(opts), int(reps), C.byref(out),
                              _stream(stream)), "gmt_autotune")
    return out.as_dict()


def gmt_autotune_build(samples, r_n: float, reps: int = 3, stream=None) -> dict:
    """Time every Euclidean build tile shape on ``samples`` (CUDA float32
    [dim][n]) and cache the fastest whose table equals the default shape's
    (see gmt_autotune_build in the header)."""
    import torch
    assert samples.is_cuda and samples.dtype == torch.float32 and samples.dim() == 2
    s = samples.contiguous()
    out = gmt_build_tune()
    _check(lib().gmt_autotune_build(s.data_ptr(), int(s.shape[1]), int(s.shape[0]), float(r_n), int(reps),
                                    C.byref(out), _stream(stream)), "gmt_autotune_build")
    return out.as_dict()


def tune_shape(kind: int, dim: int, n: int, m: int, batch: int) -> gmt_tune_shape:
    return gmt_tune_shape(int(kind), int(dim), int(n), int(m), int(batch))


def gmt_tune_lookup(shape: gmt_tune_shape) -> dict:
    out = gmt_tune_choice()
    _check(lib().gmt_tune_lookup(C.byref(shape), C.byref(out)), "gmt_tune_lookup")
    return out.as_dict()


def gmt_tune_store(shape: gmt_tune_shape, lanes: int, team_wgs: int, workgroups: int = 0,
                   threads: int = 256) -> None:
    c = gmt_tune_choice(int(lanes), int(team_wgs), int(workgroups), int(threads), 0.0, 0.0, 0)
    _check(lib().gmt_tune_store(C.byref(shape), C.byref(c)), "gmt_tune_store")


def gmt_tune_clear() -> None:
    _check(lib().gmt_tune_clear(), "gmt_tune_clear")


def gmt_tune_save(path: str) -> None:
    _check(lib().gmt_tune_save(os.fsencode(path)), "gmt_tune_save")


def gmt_tune_load(path: str) -> None:
    _check(lib().gmt_tune_load(os.fsencode(path)), "gmt_tune_load")


# ---------------------------------------------------------------------------
# replanning engine
# ---------------------------------------------------------------------------
def gmt_steady_ns() -> int:
    return int(lib().gmt_steady_ns())


class Engine:
    """Continuous-batching engine (``gmt_engine_*``)."""

    def __init__(self, budget_bytes: int, opts: gmt_plan_opts, slots: int = 4, max_batch: int = 256,
                 queue_cap: int = 0, workgroups: int = 0, batch_only: bool = False):
        eo = gmt_engine_opts(int(budget_bytes), int(slots), int(max_batch), int(queue_cap),
                             int(workgroups), opts, int(bool(batch_only)))
        h = C.c_void_p()
        _check(lib().gmt_engine_create(C.byref(eo), C.byref(h)), "gmt_engine_create")
        self.handle = h
        _track(self)

    def submit(self, q: BatchQuery, path_cap: int = 512) -> int:
        xi = _host_f32(q.x_init)
        bx = _host_f32(q.boxes).reshape(-1)
        pd = pdim_of(q.roadmap.kind, q.roadmap.dim)
        m = int(bx.size // (2 * pd)) if bx.size else 0
        p = gmt_problem()
        p.roadmap = q.roadmap.handle
        p.x_init = xi.ctypes.data_as(C.POINTER(C.c_float))
        p.goal = q.goal
        p.boxes = bx.ctypes.data_as(C.POINTER(C.c_float)) if m else None
        p.m = m
        p.lambda_ = float(q.lam)
        p.edge_step = float(q.edge_step)
        t = C.c_int64()
        _check(lib().gmt_engine_submit(self.handle, C.byref(p), int(path_cap), C.byref(t)),
               "gmt_engine_submit")
        return int(t.value)

    def poll(self, ticket: int, wait_us: int = 0, path_cap: int = 512):
        """PlanResult (with submit_ns/done_ns in .work) or None if not done."""
        r = gmt_result()
        path = np.zeros(path_cap, np.int32)
        st = lib().gmt_engine_poll(self.handle, int(ticket), int(wait_us), C.byref(r), path.ctypes.data,
                                   path_cap)
        if st == GMT_EBUSY:
            return None
        _check(st, "gmt_engine_poll")
        L = int(r.path_len) if r.status == GMT_OK else 0
        w = r.work.as_dict()
        w["submit_ns"], w["done_ns"] = int(r.submit_ns), int(r.done_ns)
        return PlanResult(int(r.status), path[:min(L, path_cap)].copy(), float(r.path_cost),
                          int(r.iters), work=w)

    def poll_any(self, wait_us: int = 0, path_cap: int = 512):
        """(ticket, PlanResult) of the next finished request, or None."""
        r = gmt_result()
        t = C.c_int64()
        path = np.zeros(path_cap, np.int32)
        st = lib().gmt_engine_poll_any(self.handle, int(wait_us), C.byref(t), C.byref(r), path.ctypes.data,
                                       path_cap)
        if st == GMT_EBUSY:
            return None
        _check(st, "gmt_engine_poll_any")
        L = int(r.path_len) if r.status == GMT_OK else 0
        w = r.work.as_dict()
        w["submit_ns"], w["done_ns"] = int(r.submit_ns), int(r.done_ns)
        return int(t.value), PlanResult(int(r.status), path[:min(L, path_cap)].copy(), float(r.path_cost),
                                        int(r.iters), work=w)

    def cancel(self, ticket: int) -> bool:
        return lib().gmt_engine_cancel(self.handle, int(ticket)) == GMT_OK

    def set_budget(self, budget_bytes: int) -> None:
        _check(lib().gmt_engine_set_budget(self.handle, int(budget_bytes)), "gmt_engine_set_budget")

    def stats(self) -> dict:
        s = gmt_engine_stats()
        _check(lib().gmt_engine_get_stats(self.handle, C.byref(s)), "gmt_engine_get_stats")
        return s.as_dict()

    def close(self) -> None:
        if self.handle:
            lib().gmt_engine_destroy(self.handle)
            self.handle = C.c_void_p(None)

    def __del__(self):  # pragma: no cover
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass
