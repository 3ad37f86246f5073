"""CPU checks of the boundary: the library loads and exports every symbol the
header declares; host-side helpers agree with the oracle.  No GPU calls."""

import ctypes
import os
import re
import struct

import numpy as np
import pytest

from paper_1705_02403_amd import gmt, inputs, radius, sampler
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="gmt.h"):
    src = open(os.path.join(ROOT, "include", name)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmt_[a-z0-9_]+)\s*\(", src)))


def test_header_lists_the_bound_symbols():
    assert header_functions() == sorted(gmt.EXPORTS)
    assert header_functions("gmt_sampler.h") == sorted(sampler.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(gmt.LIB_PATH):
        gmt.build_library()
    L = ctypes.CDLL(gmt.LIB_PATH)
    for name in header_functions() + header_functions("gmt_sampler.h"):
        assert hasattr(L, name), name
    assert "gfx950" in gmt.gmt_version()


def test_invalid_arguments_rejected_without_gpu():
    """Validation happens on the host before any device work."""
    L = gmt.lib()
    h = ctypes.c_void_p()
    assert L.gmt_build_neighbors(None, 10, 2, 0, 0.1, None, ctypes.byref(h)) == gmt.GMT_EINVAL
    assert L.gmt_plan(None, None, None, None, 0, 0.5, None, None, None, None, None, None, 0,
                      None, None, None, None) == gmt.GMT_EINVAL
    assert "null" in gmt.last_error()
    assert L.gmt_plan_noalloc(None, None, None, None, 0, 0.5, None, None, None, None, None, None, 0,
                              None, None, None, None) == gmt.GMT_EINVAL
    S = sampler.lib()
    assert S.gmt_gemm_bf16(0, 1, 64, 64, 12, None, 16, None, 16, None, 0, None, None, 64, None) == gmt.GMT_EINVAL
    assert S.gmt_sampler_create(None, ctypes.byref(h)) == gmt.GMT_EINVAL
    assert S.gmt_sampler_finish(None, 6, 0, None, 0, None, 0, None, 0, None, None) == gmt.GMT_EINVAL
    bt = gmt.gmt_build_tune()
    assert L.gmt_autotune_build(None, 100, 3, 0.1, 1, ctypes.byref(bt), None) == gmt.GMT_EINVAL
    n = ctypes.c_int32(-1)
    assert L.gmt_last_trace(0, None, 0, ctypes.byref(n)) == gmt.GMT_EINVAL  # no traced call yet
    assert L.gmt_last_trace(0, None, 0, None) == gmt.GMT_EINVAL
    bad = gmt.gmt_allocator()
    assert L.gmt_set_allocator(ctypes.byref(bad)) == gmt.GMT_EINVAL
    assert L.gmt_set_allocator(None) == gmt.GMT_OK


def test_malformed_roadmap_files_rejected_without_gpu(tmp_path):
    """A roadmap file's header is checked against the file's length before
    anything is allocated: a field larger than the file, sizes that do not add
    up, a wrong magic and a missing file are all errors, with no device work."""
    L = gmt.lib()
    h = ctypes.c_void_p()
    fmt = "<8s6iqdd10Q"
    body = b"\0" * 64

    def write(magic, sizes, tail):
        p = str(tmp_path / "x.gmtr")
        open(p, "wb").write(struct.pack(fmt, magic, 1, 4, 2, 0, 0, 0, 0, 0.1, 0.0, *sizes) + tail)
        return p.encode()

    huge = [1 << 62] + [0] * 9
    assert L.gmt_roadmap_load(write(b"GMTRMAP1", huge, body), None, ctypes.byref(h)) == gmt.GMT_EINVAL
    assert not h.value and "roadmap" in gmt.last_error()
    wrong_sum = [32, 20] + [0] * 8  # 52 bytes declared, 64 present
    assert L.gmt_roadmap_load(write(b"GMTRMAP1", wrong_sum, body), None, ctypes.byref(h)) == gmt.GMT_EINVAL
    two = [(1 << 64) - 32, 96] + [0] * 8  # wraps to 64 when added: still refused
    assert L.gmt_roadmap_load(write(b"GMTRMAP1", two, body), None, ctypes.byref(h)) == gmt.GMT_EINVAL
    assert L.gmt_roadmap_load(write(b"NOTAROAD", [64] + [0] * 9, body), None, ctypes.byref(h)) == gmt.GMT_EINVAL
    assert L.gmt_roadmap_load(str(tmp_path / "none").encode(), None, ctypes.byref(h)) == gmt.GMT_EINVAL


def test_product_radius_matches_oracle():
    for f, s in [(inputs.problem_2d, 0), (inputs.problem_2d, 3), (inputs.problem_3d, 1)]:
        p = f(s)
        mu_o = O.free_volume(p.pdim, p.boxes)
        mu_p = radius.free_volume(p.pdim, p.boxes)
        assert abs(mu_o - mu_p) <= 1e-12
        assert abs(radius.problem_radius(p) - O.euclid_radius(p)) <= 1e-14 * O.euclid_radius(p)


def test_inputs_in_the_library_range():
    p = inputs.problem_di(0, n=512)
    assert inputs.on_grid(p.samples) and np.all(np.abs(p.samples) <= 1.0)
