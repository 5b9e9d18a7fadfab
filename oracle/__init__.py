"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it and shares no code
with it.  This module is ctypes glue: it marshals numpy arrays into the C++
oracle (``raster_oracle.cpp``, ``tier_oracle.cpp``, ``mlp_oracle.cpp``) and
holds none of the arithmetic itself.  ``ordering.py`` (the training-view
order) and ``logstore.py`` (the log-structured block store and a reader of
its persisted Index) are the oracles written in Python.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["raster_oracle.cpp", "tier_oracle.cpp", "mlp_oracle.cpp"]


# IEEE double arithmetic exactly as written: no fast-math, and no fused
# multiply-adds contracted by the compiler (so that a build for the host's
# own instruction set gives the same bits as the portable one)
_FLAGS = ["-std=c++17", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off"]


def build(force: bool = True, so: str = _SO, native: bool = False) -> str:
    """Compile the oracle with g++ (OpenMP).  The portable build (-O2) is the
    one the tests load; ``native`` gives -O3 -march=native for timing it on
    the machine that builds it."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    if force or not os.path.exists(so):
        tmp = so + ".tmp"
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        subprocess.check_call(["g++"] + opt + _FLAGS + ["-o", tmp] + srcs)
        os.replace(tmp, so)
    return so


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        _lib = C.CDLL(_SO)
        _declare(_lib)
    return _lib


def use(so: str):
    """Load the oracle from another build of the same sources (a native
    build for timing); later calls go to it."""
    global _lib
    _lib = C.CDLL(so)
    _declare(_lib)
    return _lib


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's loops (0 keeps the current count);
    returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)
_u8 = C.POINTER(C.c_uint8)
_u32 = C.POINTER(C.c_uint32)
_f32 = C.POINTER(C.c_float)


def _declare(L):
    L.orc_sh_basis.argtypes = [_d, _d]
    L.orc_sh_basis_grad.argtypes = [_d, _d]
    L.orc_project.argtypes = [_d, C.c_int64, _d, C.c_int, _d, _i32, _d]
    L.orc_tile_rect.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _i32]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = C.c_int
    L.orc_tile_rects.argtypes = [_d, _d, _i32, C.c_int64, C.c_int, C.c_int, _i32]
    L.orc_bin.argtypes = [_d, _d, _d, _i32, _i32, C.c_int64, _d, C.c_int, _i64, C.c_int64, _i64]
    L.orc_bin.restype = C.c_int64
    L.orc_composite.argtypes = [_i64, _i64, _d, C.c_int64, _d, C.c_int, _d, _d, _d, _i32, _i64, _d, _d]
    L.orc_render.argtypes = [_d, C.c_int64, _d, C.c_int, _d, _d, _d, _i32, _i64, _d, _d, _i32]
    L.orc_loss.argtypes = [_d, _d, C.c_int, C.c_int, C.c_int, _d, _d]
    L.orc_backward.argtypes = [_d, C.c_int64, _d, C.c_int, _d, _d, _d, _d]
    L.orc_adam.argtypes = [_d, _d, _d, _i64, _d, _u8, C.c_int64, _d, C.c_double, C.c_double,
                           C.c_double]
    if hasattr(L, "orc_cull_blocks"):
        _declare_tier(L)
    if hasattr(L, "orc_mlp_forward"):
        _declare_mlp(L)


def _declare_tier(L):
    L.orc_kappa.argtypes = [_d, C.c_int]
    L.orc_kappa.restype = C.c_double
    L.orc_block_spheres.argtypes = [_d, C.c_int64, C.c_int64, C.c_double, _d]
    L.orc_morton_order.argtypes = [_d, C.c_int64, C.c_int64, _i64]
    L.orc_cull_blocks.argtypes = [_d, C.c_int64, _d, C.c_int, _u8]
    L.orc_alg1.argtypes = [_i32, C.c_int, _i32, C.c_int, _i32, _i32, C.c_int, _d, C.c_int64, C.c_double,
                           C.c_double, C.c_int, _i32, _i32]
    L.orc_alg1.restype = C.c_int


def _declare_mlp(L):
    _pd = C.POINTER(_d)
    L.orc_bf16_round.argtypes = [_d, C.c_int64, _d]
    L.orc_mlp_forward.argtypes = [_d, C.c_int, _i32, C.c_int, _pd, _pd, _d]
    L.orc_mlp_loss_backward.argtypes = [_d, C.c_int, _i32, C.c_int, _pd, _pd, _u8, _u8, C.c_int, _d, _pd, _pd]
    L.orc_mlp_adam.argtypes = [_d, _d, _d, _d, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double,
                               C.c_double]


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# rasterizer
# --------------------------------------------------------------------------

def sh_basis(d) -> np.ndarray:
    d = _f64(d)
    Y = np.zeros(16)
    lib().orc_sh_basis(_p(d, _d), _p(Y, _d))
    return Y


def sh_basis_grad(d) -> np.ndarray:
    d = _f64(d)
    g = np.zeros((16, 3))
    lib().orc_sh_basis_grad(_p(d, _d), _p(g, _d))
    return g


def project(theta, cams):
    """Per (camera, Gaussian) projection.  Returns dict of arrays [V, N, ...]."""
    th = _f64(theta)
    cm = _f64(cams)
    V, N = cm.shape[0], th.shape[0]
    pf = np.zeros((V, N, 16))
    pi = np.zeros((V, N, 7), dtype=np.int32)
    mg = np.zeros((V, N))
    lib().orc_project(_p(th, _d), N, _p(cm, _d), V, _p(pf, _d), _p(pi, _i32), _p(mg, _d))
    return dict(u=pf[..., 0], v=pf[..., 1], depth=pf[..., 2], conic=pf[..., 3:6], opacity=pf[..., 6],
                rgb=pf[..., 7:10], cov2d=pf[..., 10:13], rr=pf[..., 13], perr=pf[..., 14], derr=pf[..., 15],
                keep=pi[..., 0].astype(bool),
                radius=pi[..., 1], rect=pi[..., 2:6], tiles_touched=pi[..., 6], margin=mg)


def tile_rect(u, v, r, Tx, Ty):
    out = np.zeros(4, dtype=np.int32)
    lib().orc_tile_rect(float(u), float(v), int(r), int(Tx), int(Ty), _p(out, _i32))
    return out


def tile_rects(u, v, r, Tx, Ty):
    """O4's rectangle (x0, y0, x1, y1) for each of the n triples (u, v, r);
    int32 [n, 4], empty rectangles as zeros."""
    u, v = _f64(u).ravel(), _f64(v).ravel()
    r = np.ascontiguousarray(r, dtype=np.int32).ravel()
    out = np.zeros((u.size, 4), dtype=np.int32)
    lib().orc_tile_rects(_p(u, _d), _p(v, _d), _p(r, _i32), u.size, int(Tx), int(Ty), _p(out, _i32))
    return out


def n_tiles(cams) -> np.ndarray:
    cm = np.asarray(cams)
    W, H = cm[:, 16].astype(int), cm[:, 17].astype(int)
    return ((W + 15) // 16) * ((H + 15) // 16)


def bin_sort(u, v, depth, radius, keep, cams):
    """O6 binning + (tile, depth, gid) sort for all cameras.
    Returns (gid list int64[M], ranges int64[sum T, 2])."""
    u, v, depth = _f64(u), _f64(v), _f64(depth)
    radius = np.ascontiguousarray(radius, dtype=np.int32)
    keep = np.ascontiguousarray(keep, dtype=np.int32)
    cm = _f64(cams)
    V, N = u.shape
    T = int(n_tiles(cm).sum())
    ranges = np.zeros((T, 2), dtype=np.int64)
    L = lib()
    m = L.orc_bin(_p(u, _d), _p(v, _d), _p(depth, _d), _p(radius, _i32), _p(keep, _i32), N,
                  _p(cm, _d), V, None, 0, _p(ranges, _i64))
    gid = np.zeros(max(m, 1), dtype=np.int64)
    L.orc_bin(_p(u, _d), _p(v, _d), _p(depth, _d), _p(radius, _i32), _p(keep, _i32), N,
              _p(cm, _d), V, _p(gid, _i64), m, _p(ranges, _i64))
    return gid[:m], ranges


def composite(gid, ranges, rec, cams, bg=(0.0, 0.0, 0.0), depth=None, perr=None, derr=None):
    """O7 over given lists.  rec[V, N, 9] = u, v, A, B, C, opacity, r, g, b.
    depth / perr / derr [V, N] only feed the near-tie margins; by default
    the inputs are taken as exact (position uncertainty = rounding of u, v
    in single precision, depth ties impossible)."""
    cm = _f64(cams)
    rec = _f64(rec)
    V, N = rec.shape[0], rec.shape[1]
    unc = np.zeros((V, N, 3))
    unc[..., 0] = 0.0 if depth is None else depth
    unc[..., 1] = (np.abs(rec[..., 0]) + np.abs(rec[..., 1]) + 1.0) * 2.0 ** -22 if perr is None else perr
    unc[..., 2] = 0.0 if derr is None else derr
    W, H = int(cm[0, 16]), int(cm[0, 17])
    gid = np.ascontiguousarray(gid, dtype=np.int64)
    ranges = np.ascontiguousarray(ranges, dtype=np.int64)
    bgv = _f64(bg)
    img = np.zeros((V, 3, H, W))
    tf = np.zeros((V, H, W))
    last = np.zeros((V, H, W), dtype=np.int32)
    vis = np.zeros((V, H, W), dtype=np.int64)
    mg = np.zeros((V, H, W))
    lib().orc_composite(_p(gid, _i64), _p(ranges, _i64), _p(rec, _d), N, _p(cm, _d), V, _p(bgv, _d),
                        _p(img, _d), _p(tf, _d), _p(last, _i32), _p(vis, _i64), _p(mg, _d), _p(unc, _d))
    return dict(image=img, t_final=tf, last=last, visits=vis, pix_margin=mg)


def render(theta, cams, bg=(0.0, 0.0, 0.0)):
    """Full FP64 forward.  Returns image [V,3,H,W], t_final, last, visits
    (per pixel), keep [V,N], and pair / pixel near-tie ratios (margin over
    its first-order single-precision uncertainty; below 1 is a near tie)."""
    th = _f64(theta)
    cm = _f64(cams)
    V, N = cm.shape[0], th.shape[0]
    W, H = int(cm[0, 16]), int(cm[0, 17])
    bgv = _f64(bg)
    img = np.zeros((V, 3, H, W))
    tf = np.zeros((V, H, W))
    last = np.zeros((V, H, W), dtype=np.int32)
    vis = np.zeros((V, H, W), dtype=np.int64)
    pm = np.zeros((V, N))
    xm = np.zeros((V, H, W))
    keep = np.zeros((V, N), dtype=np.int32)
    lib().orc_render(_p(th, _d), N, _p(cm, _d), V, _p(bgv, _d), _p(img, _d), _p(tf, _d),
                     _p(last, _i32), _p(vis, _i64), _p(pm, _d), _p(xm, _d), _p(keep, _i32))
    return dict(image=img, t_final=tf, last=last, visits=vis, pair_margin=pm, pix_margin=xm,
                keep=keep.astype(bool))


def loss(image, target):
    """0.8 L1 + 0.2 (1 - SSIM), mean over views.  Returns (loss, dL/dimage)."""
    img = _f64(image)
    tg = _f64(target)
    V, _, H, W = img.shape
    g = np.zeros_like(img)
    out = C.c_double(0.0)
    lib().orc_loss(_p(img, _d), _p(tg, _d), V, H, W, C.byref(out), _p(g, _d))
    return out.value, g


def backward(theta, cams, dimg, bg=(0.0, 0.0, 0.0), want_2d=False):
    """dL/dtheta [N, 59] for upstream image gradient ``dimg`` [V,3,H,W]."""
    th = _f64(theta)
    cm = _f64(cams)
    gi = _f64(dimg)
    V, N = cm.shape[0], th.shape[0]
    bgv = _f64(bg)
    grad = np.zeros((N, 59))
    g2 = np.zeros((V, N, 9)) if want_2d else None
    lib().orc_backward(_p(th, _d), N, _p(cm, _d), V, _p(bgv, _d), _p(gi, _d), _p(grad, _d),
                       _p(g2, _d) if want_2d else None)
    return (grad, g2) if want_2d else grad


# per-column learning rates of the resident training recipe
LR59 = np.array([1.6e-4] * 3 + [5e-3] * 3 + [1e-3] * 4 + [5e-2] + [2.5e-3] * 48)


def adam(theta, m, v, step, grad, active, lr=LR59, b1=0.9, b2=0.999, eps=1e-15):
    """Masked Adam step; returns updated copies (theta, m, v, step)."""
    th = _f64(theta).copy()
    m = _f64(m).copy()
    v = _f64(v).copy()
    st = np.ascontiguousarray(step, dtype=np.int64).copy()
    g = _f64(grad)
    act = np.ascontiguousarray(active, dtype=np.uint8)
    lr = _f64(lr)
    lib().orc_adam(_p(th, _d), _p(m, _d), _p(v, _d), _p(st, _i64), _p(g, _d), _p(act, _u8),
                   th.shape[0], _p(lr, _d), b1, b2, eps)
    return th, m, v, st


# --------------------------------------------------------------------------
# block tier (Level-1 culling, Alg. 1)
# --------------------------------------------------------------------------

def kappa(cams) -> float:
    cm = _f64(cams)
    return lib().orc_kappa(_p(cm, _d), cm.shape[0])


def block_spheres(theta, block_rows, kap):
    th = _f64(theta)
    K = (th.shape[0] + block_rows - 1) // block_rows
    sp = np.zeros((K, 4))
    lib().orc_block_spheres(_p(th, _d), th.shape[0], block_rows, float(kap), _p(sp, _d))
    return sp


def cull_blocks(spheres, cams):
    """vis[c, k]: block k survives camera c's six-plane sphere test."""
    sp = _f64(spheres)
    cm = _f64(cams)
    vis = np.zeros((cm.shape[0], sp.shape[0]), dtype=np.uint8)
    lib().orc_cull_blocks(_p(sp, _d), sp.shape[0], _p(cm, _d), cm.shape[0], _p(vis, _u8))
    return vis.astype(bool)


def alg1(R, Kcur, Knext_per_cam, age, lam, gamma, C):
    """One step of Alg. 1.  Returns (R_next sorted, S_plus, S_minus, age', pick order)."""
    R = np.ascontiguousarray(sorted(set(int(x) for x in R)), dtype=np.int32)
    Kc = np.ascontiguousarray(sorted(set(int(x) for x in Kcur)), dtype=np.int32)
    lists = [sorted(set(int(x) for x in k)) for k in Knext_per_cam]
    flat = np.ascontiguousarray([x for l in lists for x in l] or [0], dtype=np.int32)
    counts = np.ascontiguousarray([len(l) for l in lists] or [0], dtype=np.int32)
    ag = _f64(age).copy()
    outR = np.zeros(max(C, 1), dtype=np.int32)
    rank = np.zeros(max(C, 1), dtype=np.int32)
    n = lib().orc_alg1(_p(R, _i32), len(R), _p(Kc, _i32), len(Kc), _p(flat, _i32), _p(counts, _i32), len(lists),
                       _p(ag, _d), len(ag), float(lam), float(gamma), int(C), _p(outR, _i32), _p(rank, _i32))
    Rn = outR[:n].copy()
    sR, sN = set(R.tolist()), set(Rn.tolist())
    return Rn, sorted(sN - sR), sorted(sR - sN), ag, rank[:n].copy()


# --------------------------------------------------------------------------
# prefetch predictor MLP
# --------------------------------------------------------------------------

def bf16_round(x):
    a = _f64(x)
    out = np.empty_like(a)
    lib().orc_bf16_round(_p(a, _d), a.size, _p(out, _d))
    return out


def _ptrs(arrs):
    arr = (C.POINTER(C.c_double) * len(arrs))()
    for i, a in enumerate(arrs):
        arr[i] = a.ctypes.data_as(C.POINTER(C.c_double))
    return arr


def mlp_forward(x, Ws, bs):
    """Ws[l]: [out, in] (already rounded as desired), bs[l]: [out]."""
    x = _f64(x)
    Ws = [_f64(w) for w in Ws]
    bs = [_f64(b) for b in bs]
    dims = np.ascontiguousarray([Ws[0].shape[1]] + [w.shape[0] for w in Ws], dtype=np.int32)
    out = np.zeros((x.shape[0], dims[-1]))
    lib().orc_mlp_forward(_p(x, _d), x.shape[0], _p(dims, _i32), len(Ws), _ptrs(Ws), _ptrs(bs), _p(out, _d))
    return out


def mlp_loss_backward(x, Ws, bs, labels, valid):
    """Mean BCE-with-logits over (sample, valid output) and its gradients."""
    x = _f64(x)
    Ws = [_f64(w) for w in Ws]
    bs = [_f64(b) for b in bs]
    dims = np.ascontiguousarray([Ws[0].shape[1]] + [w.shape[0] for w in Ws], dtype=np.int32)
    lab = np.ascontiguousarray(labels, dtype=np.uint8)
    val = np.ascontiguousarray(valid, dtype=np.uint8)
    dW = [np.zeros_like(w) for w in Ws]
    db = [np.zeros_like(b) for b in bs]
    out = C.c_double(0.0)
    lib().orc_mlp_loss_backward(_p(x, _d), x.shape[0], _p(dims, _i32), len(Ws), _ptrs(Ws), _ptrs(bs), _p(lab, _u8),
                                _p(val, _u8), 0, C.byref(out), _ptrs(dW), _ptrs(db))
    return out.value, dW, db


def mlp_adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step at step number t (1-based); returns new (p, m, v)."""
    p, g, m, v = (_f64(a).copy() for a in (p, g, m, v))
    lib().orc_mlp_adam(_p(p, _d), _p(g, _d), _p(m, _d), _p(v, _d), p.size, int(t), lr, b1, b2, eps)
    return p, m, v


def morton_order(xyz):
    """Stable Morton order of the rows of xyz [n, 3] (2^21 cells per axis)."""
    x = _f64(xyz)
    perm = np.zeros(x.shape[0], dtype=np.int64)
    lib().orc_morton_order(_p(x, _d), x.shape[0], x.shape[1], _p(perm, _i64))
    return perm
