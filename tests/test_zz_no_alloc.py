"""The allocation-free preprocess (tide_preprocess_noalloc) against
tide_preprocess, through the C ABI on the GPU.  (Records, depths and
rectangles are compared where the pair is kept, the only entries either call
defines.)

Two calls in a row on one device share the static scratch: the first on the
aerial 1920x1080 shape (4 views, blocks of 65 536, 80 scan blocks), the second
on a smaller input (2 views, blocks of 4096); both must give the projection
records, rectangles, tile counts, active flags, compact indices and active
count bit for bit equal to the workspace entry point's on the same inputs.
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from paper_2605_20150_amd import _lib as L
from paper_2605_20150_amd import synth
from paper_2605_20150_amd.raster import Pool, Proj, Rasterizer, _stream

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def fresh_proj(V, N, dtype):
    dev = "cuda"
    fill = lambda shape, dt: torch.full(shape, -7, dtype=dt, device=dev)
    return Proj(rec=fill((V * N * 12,), dtype), depth=fill((V * N,), torch.float32),
                rect=fill((2 * V * N,), torch.int32), tiles_touched=fill((V * N,), torch.int32),
                active=fill((N,), torch.int32), act_idx=fill((N,), torch.int32),
                n_active=fill((1,), torch.int32), n_cams=V, n_pidx=N,
                dtype=L.TIDE_F32 if dtype == torch.float32 else L.TIDE_F64)


def noalloc(pool, cams, proj):
    lib = L.load()
    pc, jc = pool.c(), proj.c()
    L.check(lib.tide_preprocess_noalloc(C.byref(pc), L.camera_array(cams), len(cams), C.byref(jc),
                                        C.c_void_p(_stream())))
    return proj


def fields(p):
    return {k: getattr(p, k).cpu().numpy() for k in
            ("rec", "depth", "rect", "tiles_touched", "active", "act_idx", "n_active")}


def compare(pool, cams, dtype):
    V, N = len(cams), pool.n_pidx
    ref = Rasterizer("cuda").preprocess(pool, cams)
    got = noalloc(pool, cams, fresh_proj(V, N, dtype))
    torch.cuda.synchronize()
    a, b = fields(ref), fields(got)
    for k in ("tiles_touched", "active", "act_idx", "n_active"):
        assert np.array_equal(a[k], b[k]), f"{k} differs"
    # records, depths and rectangles are defined where the pair is kept
    kept = a["tiles_touched"].reshape(V, N) > 0
    assert kept.any()
    rec_a, rec_b = a["rec"].reshape(V, N, 12), b["rec"].reshape(V, N, 12)
    assert np.array_equal(rec_a[kept].view(np.uint8), rec_b[kept].view(np.uint8)), "rec differs"
    assert np.array_equal(a["depth"].reshape(V, N)[kept].view(np.uint32),
                          b["depth"].reshape(V, N)[kept].view(np.uint32)), "depth differs"
    assert np.array_equal(a["rect"].reshape(V, N, 2)[kept], b["rect"].reshape(V, N, 2)[kept]), "rect differs"
    return int(a["n_active"][0])


def test_noalloc_preprocess_equals_the_workspace_entry_point_on_two_calls():
    assert torch.cuda.is_available(), "the gpu tests need an MI355X"
    say("noalloc: call 1, aerial 300k Gaussians, 4 x 1920x1080, blocks of 65536")
    theta, cams = synth.aerial_workload(n_blobs=60, per_blob=5000, n_views=400)
    pool = Pool.from_dense(torch.tensor(theta, device="cuda"), 65536)
    n1 = compare(pool, cams[:4], torch.float32)
    say(f"noalloc: call 1 equal ({pool.n_pidx} pidx, {n1} active)")
    assert n1 > 0

    say("noalloc: call 2, dense 3000 Gaussians, 2 views, blocks of 4096")
    th2 = synth.dense_scene(3000, 21, extent=1.0, logscale_mu=-2.6, logscale_sigma=0.6)
    cams2 = [synth.look_at((0.4, -0.3, -3.2), (0, 0, 0), (0, -1, 0), 150, 110, 120.0),
             synth.look_at((-0.6, 0.2, -2.9), (0.1, 0, 0), (0, -1, 0), 150, 110, 110.0)]
    pool2 = Pool.from_dense(torch.tensor(th2, device="cuda"), 4096)
    n2 = compare(pool2, cams2, torch.float32)
    say(f"noalloc: call 2 equal ({pool2.n_pidx} pidx, {n2} active)")
    assert 0 < n2 <= 3000

    say("noalloc: call 3, the same small input in FP64")
    pool3 = Pool.from_dense(torch.tensor(th2, dtype=torch.float64, device="cuda"), 4096)
    n3 = compare(pool3, cams2, torch.float64)
    assert n3 == n2


def test_noalloc_preprocess_rejects_sizes_beyond_its_scratch():
    lib = L.load()
    buf = torch.zeros(64, dtype=torch.float32, device="cuda")
    p = buf.data_ptr()
    pool = L.tide_pool()
    pool.params = pool.exp_avg = pool.exp_avg_sq = pool.step = p
    pool.slot_block = pool.slot_rows = pool.order = p
    pool.block_rows, pool.n_order, pool.n_slots, pool.dtype = 65536, 2047, 2047, L.TIDE_F32
    proj = L.tide_proj()
    proj.rec = proj.depth = proj.rect = proj.tiles_touched = proj.active = proj.act_idx = proj.n_active = p
    proj.n_pidx, proj.n_cams, proj.dtype = 65536 * 2047, 1, L.TIDE_F32
    assert proj.n_pidx > L.TIDE_PREPROCESS_NOALLOC_MAX_PIDX
    cams = L.camera_array([synth.tiny_camera()])
    code = lib.tide_preprocess_noalloc(C.byref(pool), cams, 1, C.byref(proj), C.c_void_p(_stream()))
    assert code == L.TIDE_ECAPACITY
    assert b"exceeds the maximum" in lib.tide_last_error()
