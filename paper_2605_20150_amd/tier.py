"""Driver of the out-of-core block tier (libtide.so's tide_residency).

Argument marshalling only: the log store, host cache, I/O threads, Level-1
culling, Alg. 1 and the transfers all run in the library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .raster import D, Pool


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Tier:
    def __init__(self, directory: str, n_rows: int, pool: Pool, capacity: int, host_cache_blocks: int,
                 io_threads: int = 4, lam: float = 0.75, gamma: float = 0.9, kappa: float = 1.32,
                 host_pool: bool = False, odirect: bool = False, no_tide: bool = False, no_overlap: bool = False,
                 cold_restart: bool = False, bounded: bool = False):
        """no_tide / no_overlap: the paper's ablations (full retransmission of
        K_{t+1}; transfers serialised with compute).  cold_restart / bounded:
        its default optimizer placement (moments only while resident) and a
        binding budget (render R_t and K_t's intersection)."""
        self.lib = L.load()
        self.pool = pool
        self.B = pool.block_rows
        self.N = int(n_rows)
        self.K = (self.N + self.B - 1) // self.B
        dev = pool.params.device
        self.spheres = torch.zeros((self.K, 4), dtype=torch.float32, device=dev)
        self.dirty = torch.zeros((self.K,), dtype=torch.uint8, device=dev)
        self.cpool = pool.c()          # persistent struct: the tier writes n_order into it
        cfg = L.tide_store_cfg()
        self._dir = directory.encode()
        cfg.dir = self._dir
        cfg.n_rows = self.N
        cfg.block_rows = self.B
        cfg.capacity = int(capacity)
        cfg.host_cache_blocks = int(host_cache_blocks)
        cfg.io_threads = int(io_threads)
        cfg.flags = ((L.TIDE_TIER_HOST_POOL if host_pool else 0) | (L.TIDE_TIER_ODIRECT if odirect else 0) |
                     (L.TIDE_TIER_NO_TIDE if no_tide else 0) | (L.TIDE_TIER_NO_OVERLAP if no_overlap else 0) |
                     (L.TIDE_TIER_COLD_RESTART if cold_restart else 0) | (L.TIDE_TIER_BOUNDED if bounded else 0))
        self.bounded = bool(bounded)
        cfg.lambda_, cfg.gamma, cfg.kappa = float(lam), float(gamma), float(kappa)
        self.cfg = cfg
        h = C.c_void_p()
        L.check(self.lib.tide_residency_create(C.byref(cfg), C.byref(self.cpool),
                                               C.c_void_p(self.spheres.data_ptr()),
                                               C.c_void_p(self.dirty.data_ptr()), C.byref(h)))
        self.h = h
        self.rec_bytes = int(self.lib.tide_block_record_bytes(self.B))

    # ------------------------------------------------------------ layout
    def put_block(self, k: int, params_cols: np.ndarray):
        """params_cols: f32 [59][rows of block k] (column-major block)."""
        a = np.ascontiguousarray(params_cols, dtype=np.float32)
        L.check(self.lib.tide_store_put_block(self.h, int(k), C.c_void_p(a.ctypes.data)))

    def finalize(self):
        L.check(self.lib.tide_store_finalize(self.h))

    def open(self):
        L.check(self.lib.tide_store_open(self.h))

    # -------------------------------------------------------- per iteration
    def cull(self, cams) -> list[np.ndarray]:
        arr = L.camera_array(cams)
        cap = self.K * len(cams)
        ids = np.zeros(max(cap, 1), dtype=np.int32)
        counts = np.zeros(len(cams), dtype=np.int32)
        L.check(self.lib.tide_cull_blocks(self.h, arr, len(cams), _ptr(ids), _ptr(counts), cap))
        out, o = [], 0
        for c in counts:
            out.append(ids[o:o + c].copy())
            o += c
        return out

    def ensure_resident(self, K, stream=None) -> float:
        k = _i32(sorted(set(int(x) for x in K)) or [0])
        n = len(set(int(x) for x in K))
        stall = C.c_double(0.0)
        L.check(self.lib.tide_ensure_resident(self.h, _ptr(k), n, C.c_void_p(stream or 0), C.byref(stall)))
        self.pool.n_order = int(self.cpool.n_order)
        return stall.value

    def stream_delta(self, knext_per_cam, side_stream=None):
        lists = [sorted(set(int(x) for x in k)) for k in knext_per_cam]
        flat = _i32([x for l in lists for x in l] or [0])
        counts = _i32([len(l) for l in lists])
        cap = self.K
        plus = np.zeros(cap, dtype=np.int32)
        minus = np.zeros(cap, dtype=np.int32)
        npl, nmi = C.c_int32(0), C.c_int32(0)
        L.check(self.lib.tide_stream_delta(self.h, _ptr(flat), _ptr(counts), len(lists), C.c_void_p(side_stream or 0),
                                           _ptr(plus), C.byref(npl), _ptr(minus), C.byref(nmi), cap))
        return plus[:npl.value].copy(), minus[:nmi.value].copy()

    def end_iteration(self, stream=None):
        L.check(self.lib.tide_residency_end_iteration(self.h, C.c_void_p(stream or 0)))

    def sync_bounds(self):
        L.check(self.lib.tide_residency_sync_bounds(self.h))

    def prefetch(self, blocks, horizon: int = 1):
        b = _i32(list(blocks) or [0])
        L.check(self.lib.tide_prefetch_hint(self.h, _ptr(b), len(list(blocks)), int(horizon)))

    def checkpoint(self):
        L.check(self.lib.tide_checkpoint(self.h))

    def compact(self):
        """Merge the patch segments into a new base segment (checkpoint first)."""
        L.check(self.lib.tide_store_compact(self.h))

    def layout_build(self, table_path: str, tmp_dir: str, run_rows: int):
        """Out-of-core Morton layout of a new store from an f32 [N][59] table
        file; the store is finalized on return."""
        L.check(self.lib.tide_layout_build(self.h, table_path.encode(), tmp_dir.encode(), int(run_rows)))

    # ------------------------------------------------------------ inspection
    def read_block(self, k: int) -> dict:
        buf = np.zeros(self.rec_bytes, dtype=np.uint8)
        L.check(self.lib.tide_read_block(self.h, int(k), C.c_void_p(buf.ctypes.data)))
        n = D * self.B
        f = buf.view(np.float32)
        return dict(params=f[:n].reshape(D, self.B).copy(), exp_avg=f[n:2 * n].reshape(D, self.B).copy(),
                    exp_avg_sq=f[2 * n:3 * n].reshape(D, self.B).copy(), step=buf[12 * n:].view(np.uint32).copy())

    def stats(self) -> dict:
        s = L.tide_tier_stats()
        L.check(self.lib.tide_tier_get_stats(self.h, C.byref(s)))
        return s.as_dict()

    def host_spheres(self) -> np.ndarray:
        out = np.zeros((self.K, 4), dtype=np.float32)
        L.check(self.lib.tide_tier_spheres(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), self.K))
        return out

    def resident(self) -> list[int]:
        """R as the tier's host tables hold it (ascending block ids)."""
        out = np.zeros(max(1, self.K), dtype=np.int32)
        n = C.c_int32(0)
        L.check(self.lib.tide_tier_resident(self.h, _ptr(out), self.K, C.byref(n)))
        return out[:n.value].tolist()

    def resident_slots(self) -> dict:
        """block -> slot, read from the pool's slot table."""
        sb = self.pool.slot_block.cpu().numpy()
        return {int(b): s for s, b in enumerate(sb) if b >= 0}

    def close(self):
        if self.h:
            self.lib.tide_residency_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
