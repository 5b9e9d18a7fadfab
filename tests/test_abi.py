"""The C ABI library: it loads, exports every symbol include/tide.h
declares, and rejects bad arguments on the host before any launch (CPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2605_20150_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(tide_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert declared_functions() == set(L.SIGNATURES)


def test_workspace_size_queries_are_host_only():
    lib = L.load()
    assert lib.tide_preprocess_ws_bytes(1 << 20) > 0
    a = lib.tide_bin_sort_ws_bytes(4, 1 << 20, 120, 68, 1 << 22)
    b = lib.tide_bin_sort_ws_bytes(4, 1 << 20, 120, 68, 1 << 23)
    assert b > a > 0
    assert lib.tide_loss_ws_bytes(4, 1080, 1920, L.TIDE_F32) > 3 * 4 * 3 * 1080 * 1920


def test_null_arguments_rejected_before_launch():
    lib = L.load()
    cam = L.camera_array([type("Cam", (), dict(R=[1, 0, 0, 0, 1, 0, 0, 0, 1], t=[0, 0, 3], fx=64, fy=64, cx=32,
                                                cy=32, width=64, height=64, z_near=0.2, z_far=1e4))()])
    assert lib.tide_preprocess(None, cam, 1, None, None, 0, None) == L.TIDE_EINVAL
    assert b"null" in lib.tide_last_error()
    pool = L.tide_pool()
    assert lib.tide_preprocess(C.byref(pool), cam, 1, None, None, 0, None) == L.TIDE_EINVAL
    assert lib.tide_loss(None, None, 1, 8, 8, 0, None, None, None, 0, None) == L.TIDE_EINVAL
    cfg = L.tide_adam_cfg()
    assert lib.tide_adam_sparse(None, None, None, 0, C.byref(cfg), None, None, 0, None, 0, None) == L.TIDE_EINVAL
    assert lib.tide_render_bwd_adam(None, cam, 1, None, None, None, None, None, C.byref(cfg), None, None, 0, None,
                                    0, None) == L.TIDE_EINVAL
    assert lib.tide_render_bwd_adam(C.byref(pool), cam, 1, None, None, None, None, None, None, None, None, 0, None,
                                    0, None) == L.TIDE_EINVAL


def test_noalloc_preprocess_rejects_a_size_beyond_its_scratch_on_the_host():
    """tide_preprocess_noalloc refuses n_pidx above its static scratch before
    any device call (host buffers stand in for the device pointers, which
    the size check never touches)."""
    lib = L.load()
    host = (C.c_double * 64)()
    p = C.cast(host, C.c_void_p).value
    pool = L.tide_pool()
    pool.params = pool.exp_avg = pool.exp_avg_sq = pool.step = p
    pool.slot_block = pool.slot_rows = pool.order = p
    pool.block_rows, pool.n_order, pool.n_slots, pool.dtype = 65536, 2047, 2047, L.TIDE_F32
    proj = L.tide_proj()
    proj.rec = proj.depth = proj.rect = proj.tiles_touched = proj.active = proj.act_idx = proj.n_active = p
    proj.n_pidx, proj.n_cams, proj.dtype = 65536 * 2047, 1, L.TIDE_F32
    assert proj.n_pidx > L.TIDE_PREPROCESS_NOALLOC_MAX_PIDX
    cam = L.camera_array([type("Cam", (), dict(R=[1, 0, 0, 0, 1, 0, 0, 0, 1], t=[0, 0, 3], fx=64, fy=64, cx=32,
                                                cy=32, width=64, height=64, z_near=0.2, z_far=1e4))()])
    assert lib.tide_preprocess_noalloc(C.byref(pool), cam, 1, C.byref(proj), None) == L.TIDE_ECAPACITY
    assert b"exceeds the maximum" in lib.tide_last_error()
    assert lib.tide_preprocess_noalloc(None, cam, 1, C.byref(proj), None) == L.TIDE_EINVAL
