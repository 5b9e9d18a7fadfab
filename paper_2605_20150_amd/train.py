"""Training loops over the C ABI: all-resident, and out-of-core through the
block tier (Sec. 3.2 stages 1-4 with Alg. 1).  Each iteration is one batch of
views: forward, loss, adjoint, masked Adam, all in libtide.so."""
from __future__ import annotations

import hashlib
import time

import numpy as np
import torch

from .raster import LR59, Pool, Rasterizer, adam_cfg
from .tier import Tier


def image_digest(img: torch.Tensor) -> str:
    return hashlib.sha1(img.contiguous().cpu().numpy().tobytes()).hexdigest()


def step(rast: Rasterizer, pool: Pool, cams, target, cfg, grad, spheres=None, dirty=None):
    proj, bins, fr = rast.forward(pool, cams)
    loss, dimg = rast.loss(fr.image, target)
    g = rast.backward(pool, cams, proj, bins, fr, dimg, grad=grad)
    rast.adam(pool, proj, g, cfg, spheres, dirty)
    return fr, loss


class ResidentTrainer:
    """Every block resident (block k in slot k)."""

    def __init__(self, theta: np.ndarray, block_rows: int, device="cuda", kappa=1.32):
        self.rast = Rasterizer(device)
        self.pool = Pool.from_dense(torch.tensor(theta, device=device), block_rows)
        self.cfg = adam_cfg(LR59, kappa=kappa)
        self.grad = torch.empty((59, self.pool.n_pidx), dtype=torch.float32, device=device)
        self.N = theta.shape[0]

    def iterate(self, cams, target):
        return step(self.rast, self.pool, cams, target, self.cfg, self.grad)

    def params(self) -> np.ndarray:
        return self.pool.dense(self.N).cpu().numpy()


class OutOfCoreTrainer:
    """Blocks live in the tier's SSD store; GPU slots hold the resident set.

    Per iteration t: sync bounds -> K_t (Level-1 culling) -> ensure resident
    -> compute -> end iteration -> K_{t+1} -> Alg. 1 delta (transfers on a
    side stream, overlapping the compute that is still running)."""

    def __init__(self, theta, block_rows: int, directory: str, capacity: int, spare_slots: int,
                 host_cache_blocks: int, device="cuda", kappa=1.32, io_threads=4, predictor=None,
                 n_rows: int | None = None, odirect: bool = False, no_tide: bool = False,
                 no_overlap: bool = False, cold_restart: bool = False, bounded: bool = False):
        """theta: the [N][59] table to lay out in a new store, or None to
        reopen the store already in ``directory`` (n_rows rows, from its
        persisted Index)."""
        self.rast = Rasterizer(device)
        self.N = theta.shape[0] if theta is not None else int(n_rows)
        self.B = block_rows
        self.pool = Pool.empty(capacity + spare_slots, block_rows, device)
        self.tier = Tier(directory, self.N, self.pool, capacity, host_cache_blocks, io_threads=io_threads,
                         kappa=kappa, odirect=odirect, no_tide=no_tide, no_overlap=no_overlap,
                         cold_restart=cold_restart, bounded=bounded)
        if theta is not None:
            for k in range(self.tier.K):
                rows = theta[k * block_rows:(k + 1) * block_rows]
                self.tier.put_block(k, np.ascontiguousarray(rows.T))
            self.tier.finalize()
        else:
            self.tier.open()
        self.cfg = adam_cfg(LR59, kappa=kappa)
        self.grad = torch.empty((59, self.pool.n_slots * block_rows), dtype=torch.float32, device=device)
        self.side = torch.cuda.Stream(device=device)
        self.predictor = predictor
        self.stall = 0.0
        self.k_sets = []        # K_t per iteration
        self.r_sets = []        # R_t per iteration (after ensure_resident)

    def iterate(self, cams, target, next_cams=None):
        t = self.tier
        cs = torch.cuda.current_stream().cuda_stream
        t.sync_bounds()
        per_cam = t.cull(cams)
        K = sorted(set(int(x) for s in per_cam for x in s))
        self.k_sets.append(K)
        if t.bounded and not self.r_sets:
            # under a binding budget the first batch comes in by a delta from the empty set
            t.stream_delta(per_cam, self.side.cuda_stream)
        self.stall += t.ensure_resident(K, cs)
        self.r_sets.append(t.resident())
        hinting = self.predictor is not None and next_cams is not None
        if hinting:
            self.predictor.launch(list(cams) + list(next_cams))   # its own stream: overlaps the compute
        fr, loss = step(self.rast, self.pool, cams, target, self.cfg, self.grad, t.spheres, t.dirty)
        t.end_iteration(cs)
        if next_cams is not None:
            t.stream_delta(t.cull(next_cams), self.side.cuda_stream)
            if hinting:
                self.predictor.hint(t)
        return fr, loss

    def params(self) -> np.ndarray:
        torch.cuda.synchronize()
        t = self.tier
        t.sync_bounds()
        out = np.zeros((self.N, 59), dtype=np.float32)
        for k in range(t.K):
            r = t.read_block(k)
            rows = min(self.B, self.N - k * self.B)
            out[k * self.B:k * self.B + rows] = r["params"][:, :rows].T
        return out


def view_order(cams, cluster_size: int = 16, dir_weight: float = 10.0) -> np.ndarray:
    """Clustered travelling-salesperson order of the training views (Sec. 3.5,
    App. A), from the library: a permutation of range(len(cams))."""
    import ctypes as C
    from . import _lib as L
    n = len(cams)
    perm = np.zeros(max(1, n), dtype=np.int32)
    arr = L.camera_array(cams) if n else None
    L.check(L.load().tide_view_order(arr, n, int(cluster_size), float(dir_weight),
                                     perm.ctypes.data_as(C.POINTER(C.c_int32))))
    return perm[:n].copy()
