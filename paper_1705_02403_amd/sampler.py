"""Binding of include/gmt_sampler.h (ctypes, argument marshalling only) and
the learned sampler's host-side workflow: condition features, training data
from plain GMT* paths, training loop, and the 50/50 learned/uniform sample
set of a query.  Every numeric step of training and inference runs in the
library's kernels."""

from __future__ import annotations

import ctypes as C
import sys
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import gmt
from . import inputs as I

EXPORTS = ["gmt_gemm_bf16", "gmt_sampler_create", "gmt_sampler_get_params", "gmt_sampler_get_grads",
           "gmt_sampler_set_data", "gmt_sampler_train_step", "gmt_sampler_decode", "gmt_sampler_finish",
           "gmt_sampler_generate", "gmt_sampler_destroy"]

IN, HIDDEN, OUT, COND, BOX_SLOTS = 416, 256, 16, 396, 64
NET_PARAMS = HIDDEN * IN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + OUT * HIDDEN + OUT
PARAMS = 2 * NET_PARAMS


class gmt_train_opts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("adam_eps", C.c_float),
                ("recon_weight", C.c_float), ("kl_weight", C.c_float)]


def train_opts(lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8, recon_weight=1.0, kl_weight=1.0):
    return gmt_train_opts(lr, beta1, beta2, adam_eps, recon_weight, kl_weight)


_bound = False


def lib():
    global _bound
    L = gmt.lib()
    if not _bound:
        P, i32, f = C.c_void_p, C.c_int32, C.c_float
        L.gmt_gemm_bf16.argtypes = [i32, i32, i32, i32, i32, P, i32, P, i32, P, i32, P, P, i32, P]
        L.gmt_sampler_create.argtypes = [P, C.POINTER(P)]
        L.gmt_sampler_get_params.argtypes = [P, P]
        L.gmt_sampler_get_grads.argtypes = [P, P]
        L.gmt_sampler_set_data.argtypes = [P, P, i32, P, P, i32]
        L.gmt_sampler_train_step.argtypes = [P, P, P, i32, C.POINTER(gmt_train_opts), P, P]
        L.gmt_sampler_decode.argtypes = [P, P, P, i32, P, P]
        L.gmt_sampler_finish.argtypes = [P, i32, i32, P, i32, P, i32, P, i32, C.POINTER(i32), P]
        L.gmt_sampler_generate.argtypes = [P, P, P, i32, P, i32, P, i32, P, i32, C.POINTER(i32), P]
        L.gmt_sampler_destroy.argtypes = [P]
        for name in EXPORTS:
            getattr(L, name).restype = i32
        _bound = True
    return L


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _dev(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# BF16 GEMM
# ---------------------------------------------------------------------------
def gemm_bf16(A, B, trans_a: bool = False, trans_b: bool = False, bias=None, relu: bool = False,
              out_f32: bool = True, out_bf16: bool = False, stream=None):
    """op(A) op(B) (+ bias) (ReLU) of 2-D BF16 CUDA tensors (row-major, any
    leading dimension); returns (C fp32 or None, C bf16 or None)."""
    import torch
    assert A.dtype == torch.bfloat16 and B.dtype == torch.bfloat16 and A.stride(1) == 1 and B.stride(1) == 1
    M, K = (A.shape[1], A.shape[0]) if trans_a else (A.shape[0], A.shape[1])
    K2, N = (B.shape[1], B.shape[0]) if trans_b else (B.shape[0], B.shape[1])
    assert K == K2, "inner dimensions differ"
    dev = A.device
    Cf = torch.empty((M, N), dtype=torch.float32, device=dev) if out_f32 else None
    Cb = torch.empty((M, N), dtype=torch.bfloat16, device=dev) if out_bf16 else None
    st = lib().gmt_gemm_bf16(int(trans_a), int(trans_b), M, N, K, _dev(A), A.stride(0), _dev(B), B.stride(0),
                             _dev(bias), int(relu), _dev(Cf), _dev(Cb), N, gmt._stream(stream))
    gmt._check(st, "gmt_gemm_bf16")
    return Cf, Cb


# ---------------------------------------------------------------------------
# the sampler object
# ---------------------------------------------------------------------------
class Sampler:
    def __init__(self, params: np.ndarray):
        p = _f32(params)
        assert p.shape == (PARAMS,)
        h = C.c_void_p()
        gmt._check(lib().gmt_sampler_create(p.ctypes.data, C.byref(h)), "gmt_sampler_create")
        self.handle = h
        gmt._track(self)
        self.W = 0

    def params(self) -> np.ndarray:
        out = np.empty(PARAMS, np.float32)
        gmt._check(lib().gmt_sampler_get_params(self.handle, out.ctypes.data), "gmt_sampler_get_params")
        return out

    def grads(self) -> np.ndarray:
        out = np.empty(PARAMS, np.float32)
        gmt._check(lib().gmt_sampler_get_grads(self.handle, out.ctypes.data), "gmt_sampler_get_grads")
        return out

    def set_data(self, cond: np.ndarray, targets: np.ndarray, owner: np.ndarray) -> None:
        c, t = _f32(cond), _f32(targets)
        o = np.ascontiguousarray(owner, dtype=np.int32)
        gmt._check(lib().gmt_sampler_set_data(self.handle, c.ctypes.data, c.shape[0], t.ctypes.data,
                                              o.ctypes.data, t.shape[0]), "gmt_sampler_set_data")
        self.W = t.shape[0]

    def train_step(self, rows: np.ndarray, eps, opts: gmt_train_opts, loss=None, stream=None) -> None:
        """rows: host int32 [B]; eps: CUDA float32 [B][6]; loss: CUDA float32 [2] or None."""
        r = np.ascontiguousarray(rows, dtype=np.int32)
        assert eps.is_contiguous() and tuple(eps.shape) == (r.size, 6)
        gmt._check(lib().gmt_sampler_train_step(self.handle, r.ctypes.data, _dev(eps), r.size, C.byref(opts),
                                                _dev(loss), gmt._stream(stream)), "gmt_sampler_train_step")

    def decode(self, cond: np.ndarray, eps, stream=None):
        import torch
        c = _f32(cond)
        raw = torch.empty((eps.shape[0], 6), dtype=torch.float32, device=eps.device)
        gmt._check(lib().gmt_sampler_decode(self.handle, c.ctypes.data, _dev(eps), eps.shape[0], _dev(raw),
                                            gmt._stream(stream)), "gmt_sampler_decode")
        return raw

    def generate(self, cond: np.ndarray, eps, boxes: np.ndarray, fallback, out, stream=None) -> int:
        """Learned samples into ``out`` (a CUDA float32 view [6][count] with row
        stride ld); ``fallback`` CUDA [6][count]; returns the rejected count."""
        c, bx = _f32(cond), _f32(boxes).reshape(-1)
        count = eps.shape[0]
        rej = C.c_int32()
        gmt._check(lib().gmt_sampler_generate(self.handle, c.ctypes.data, _dev(eps), count,
                                              bx.ctypes.data if bx.size else None, bx.size // 6, _dev(fallback),
                                              fallback.stride(0), _dev(out), out.stride(0), C.byref(rej),
                                              gmt._stream(stream)), "gmt_sampler_generate")
        return int(rej.value)

    def close(self) -> None:
        if self.handle:
            lib().gmt_sampler_destroy(self.handle)
            self.handle = C.c_void_p(None)

    def __del__(self):  # pragma: no cover
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass


def finish(raw, boxes: np.ndarray, fallback, stream=None):
    """gmt_sampler_finish on CUDA tensors raw [count][6] and fallback
    [6][count]; returns (states [6][count] CUDA, rejected)."""
    import torch
    bx = _f32(boxes).reshape(-1)
    count = raw.shape[0]
    out = torch.empty((6, count), dtype=torch.float32, device=raw.device)
    rej = C.c_int32()
    gmt._check(lib().gmt_sampler_finish(_dev(raw), raw.stride(0), count, bx.ctypes.data if bx.size else None,
                                        bx.size // 6, _dev(fallback), fallback.stride(0), _dev(out), count,
                                        C.byref(rej), gmt._stream(stream)), "gmt_sampler_finish")
    return out, int(rej.value)


# ---------------------------------------------------------------------------
# features and training data
# ---------------------------------------------------------------------------
def condition(prob) -> np.ndarray:
    """Condition features of a double-integrator query (396 floats): x_init,
    goal centre and radius, then up to 64 boxes (lo xyz, hi xyz)."""
    c = np.zeros(COND, np.float32)
    c[0:6] = prob.x_init
    c[6:9] = prob.goal_center[:3]
    c[9] = prob.goal_radius
    m = prob.boxes.shape[0]
    if m > BOX_SLOTS:
        raise ValueError("the sampler conditions on at most %d boxes (query has %d)" % (BOX_SLOTS, m))
    if m:
        c[12:12 + 6 * m] = prob.boxes.reshape(-1)
    return c


def to_unconstrained(states: np.ndarray) -> np.ndarray:
    """States [k][6] (position in [0,1]^3, velocity in the unit ball) ->
    training targets: logit of the position, v / sqrt(1 - |v|^2) of the
    velocity (inverse of the output map), clipped away from the boundary."""
    s = np.asarray(states, dtype=np.float64)
    p = np.clip(s[:, 0:3], 1e-4, 1.0 - 1e-4)
    v = s[:, 3:6]
    nv = np.linalg.norm(v, axis=1, keepdims=True)
    v = np.where(nv > 0.999, v * (0.999 / np.maximum(nv, 1e-300)), v)
    nv2 = np.sum(v * v, axis=1, keepdims=True)
    out = np.concatenate([np.log(p / (1.0 - p)), v / np.sqrt(1.0 - nv2)], axis=1)
    return out.astype(np.float32)


@dataclass
class TrainingSet:
    cond: np.ndarray      # [P][396]
    targets: np.ndarray   # [W][6] unconstrained
    owner: np.ndarray     # [W]
    solved: int
    problems: int


def path_dataset(problems: Sequence, roadmaps: dict, samples: dict, opts, batch: int = 1024) -> TrainingSet:
    """Solve ``problems`` with plain GMT* (gmt_plan_batch on resident
    roadmaps keyed by sample_seed) and keep every path node after the root
    as a training waypoint of its problem."""
    conds, targ, owner = [], [], []
    solved = 0
    for k0 in range(0, len(problems), batch):
        chunk = problems[k0:k0 + batch]
        qs = [gmt.BatchQuery(roadmaps[p.sample_seed], p.x_init, gmt.make_goal(p.goal_center, p.goal_radius, 3),
                             p.boxes, p.lam) for p in chunk]
        out = gmt.gmt_plan_batch(qs, opts, path_cap=256)
        for p, o in zip(chunk, out):
            if o.status != gmt.GMT_OK or len(o.path) < 2:
                continue
            solved += 1
            nodes = np.asarray(o.path[1:], dtype=np.int64)
            st = samples[p.sample_seed][:, nodes].T
            j = len(conds)
            conds.append(condition(p))
            targ.append(to_unconstrained(st))
            owner.append(np.full(len(nodes), j, np.int32))
    if not conds:
        raise RuntimeError("no solved problem to train on")
    return TrainingSet(np.stack(conds), np.concatenate(targ), np.concatenate(owner), solved, len(problems))


def train(sampler: Sampler, data: TrainingSet, steps: int, batch: int = 1024, seed: int = 0,
          opts: Optional[gmt_train_opts] = None, log_every: int = 0) -> List[tuple]:
    """Train on the resident set: uniform row draws and normal noise from
    seeded generators; returns (step, recon, kl) at the logged steps."""
    import torch
    sampler.set_data(data.cond, data.targets, data.owner)
    opts = opts or train_opts()
    rng = np.random.default_rng(50_000_017 + seed)
    dev = torch.device("cuda", torch.cuda.current_device())
    loss = torch.zeros(2, dtype=torch.float32, device=dev)
    hist = []
    for step in range(steps):
        rows = rng.integers(0, data.targets.shape[0], size=batch, dtype=np.int64).astype(np.int32)
        eps = torch.from_numpy(I.normal_draws(seed * 1_000_003 + step, batch)).to(dev)
        sampler.train_step(rows, eps, opts, loss)
        if log_every and (step % log_every == 0 or step == steps - 1):
            r, k = loss.tolist()
            hist.append((step, r, k))
    return hist


def mixed_samples(sampler: Sampler, prob, n: int, seed: int, learned: bool = True, uniform=None,
                  fallback=None, eps=None):
    """Sample set of one query as a CUDA SoA [6][n] tensor: the first n - n/2
    uniform (with a goal sample), the rest from the network (rejected ones
    replaced by uniform fallback draws) -- or all uniform when ``learned`` is
    false.  ``uniform`` [6][n - n/2], ``fallback`` [6][n/2] and ``eps``
    [n/2][6] may be supplied as resident CUDA tensors (they do not depend on
    the query); otherwise they are drawn from ``seed``.  Returns
    (samples, rejected)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    n_l = n // 2 if learned else 0
    n_u = n - n_l
    out = torch.empty((6, n), dtype=torch.float32, device=dev)
    if uniform is None:
        uniform = torch.from_numpy(I.di_samples(1_000 + seed, n_u)).to(dev)
    out[:, :n_u] = uniform
    rej = 0
    if n_l:
        if fallback is None:
            fallback = torch.from_numpy(I.di_samples(2_000_000 + seed, n_l)).to(dev)
        if eps is None:
            eps = torch.from_numpy(I.normal_draws(3_000_000 + seed, n_l)).to(dev)
        rej = sampler.generate(condition(prob), eps, prob.boxes, fallback, out[:, n_u:])
    return out, rej
