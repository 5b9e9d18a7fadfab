"""Out-of-core training over a synthetic street city, with and without the
learned prefetch hints.

1. Layout build (Sec. 3.3): the city's centres are put in the library's
   Morton order and cut into blocks; every block's attributes come from a
   stream keyed by (seed, block), so the scene is generated one block at a
   time; the library writes each record to the base segment and computes the
   block spheres.
2. Predictor: dry-run street walks (culling only, no rendering) give
   (8-pose history, exact block sets of the 4 following batches) pairs; the
   MLP is trained on the GPU kernels and its threshold set for 99 % recall
   on held-out pairs.
3. The same held-out walk is trained twice from the same base store (each
   run reopens the persisted Index, so both start from identical state):
   exact-culling-only streaming (Alg. 1) and Alg. 1 plus the predictor's
   SSD-to-host prefetch hints.  Stall, iteration rate and I/O volumes are
   measured per run, and the rendered images are compared per iteration.

Argument marshalling and orchestration only; every step runs in libtide.so.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np
import torch

from . import predictor as P
from . import synth
from .raster import Pool
from .tier import Tier
from .train import OutOfCoreTrainer


def build_store(directory: str, n_blocks: int, B: int, seed: int, extent: float, kappa: float = 1.32,
                layout: str = "morton", log=print):
    """Lays out a city of n_blocks * B Gaussians in a new store; returns
    (N, City, host spheres f32 [K][4], seconds).  layout "random" is the
    ablation without spatial locality (Sec. 4.4): the same centres in a
    seeded random order."""
    if layout not in ("morton", "random"):
        raise ValueError(f"unknown layout {layout!r}")
    t0 = time.perf_counter()
    N = n_blocks * B
    mu, city = synth.city_means(N, seed, extent)
    mu32 = mu.astype(np.float32)
    del mu
    if layout == "morton":
        perm = P.morton_order(mu32)
    else:
        perm = np.random.Generator(np.random.PCG64(seed + 7)).permutation(N).astype(np.int64)
    log(f"layout: {N} centres generated and put in {layout} order in {time.perf_counter() - t0:.1f} s")
    pool = Pool.empty(1, B, "cpu")
    tier = Tier(directory, N, pool, 1, 4, io_threads=1, kappa=kappa, host_pool=True, odirect=True)
    for k in range(n_blocks):
        rows = perm[k * B:(k + 1) * B]
        blk = synth.block_attributes(seed, k, len(rows))
        blk[:, 0:3] = mu32[rows]
        tier.put_block(k, np.ascontiguousarray(blk.T))
        if k % 100 == 99:
            log(f"layout: {k + 1}/{n_blocks} blocks written, {time.perf_counter() - t0:.1f} s")
    tier.finalize()
    spheres = tier.host_spheres()
    tier.close()
    return N, city, spheres, time.perf_counter() - t0


def write_table(path: str, n_blocks: int, B: int, seed: int, extent: float, log=print):
    """Writes the city's n_blocks * B Gaussians in generation order (no
    layout) as an f32 [N][59] table file, B rows at a time; returns
    (N, City, seconds).  The input of the out-of-core layout build."""
    t0 = time.perf_counter()
    N = n_blocks * B
    mu, city = synth.city_means(N, seed, extent)
    with open(path, "wb") as f:
        for k in range(n_blocks):
            blk = synth.block_attributes(seed, k, B)
            blk[:, 0:3] = mu[k * B:(k + 1) * B]
            f.write(np.ascontiguousarray(blk, dtype=np.float32).tobytes())
            if k % 100 == 99:
                log(f"table: {k + 1}/{n_blocks} chunks written, {time.perf_counter() - t0:.1f} s")
    return N, city, time.perf_counter() - t0


def walk_batches(city, seed: int, n_iters: int, z_far: float, width: int, height: int):
    cams = synth.street_walk(city, 4 * n_iters, seed, width=width, height=height, z_far=z_far)
    return [cams[4 * t:4 * t + 4] for t in range(n_iters)]


def train_predictor(spheres, city, z_far: float, seeds, n_iters: int, epochs: int = 20, log=print):
    K = spheres.shape[0]
    words = P.DEFAULT_DIMS[-1] // (32 * P.HORIZON)
    if K > 32 * words:
        raise ValueError(f"{K} blocks exceed the predictor's {32 * words} outputs per horizon")
    t0 = time.perf_counter()
    Xs, Ys = [], []
    for s in seeds:
        X, Y = P.log_pairs(spheres, walk_batches(city, s, n_iters, z_far, 1600, 900), words)
        Xs.append(X)
        Ys.append(Y)
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    t1 = time.perf_counter()
    base = float(np.unpackbits(Y.view(np.uint8)).sum()) / (Y.shape[0] * P.HORIZON * K)
    mlp = P.MLP(P.DEFAULT_DIMS, seed=3, out_bias=math.log(base / (1.0 - base)))
    out = P.train(mlp, X, Y, P.valid_mask(K, words), epochs=epochs, batch=256, lr=1e-3, seed=4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = dict(pairs=int(X.shape[0]), log_s=round(t1 - t0, 2), train_s=round(t2 - t1, 2), base_rate=base,
                steps=int(len(out["losses"])), loss_first=float(out["losses"][:10].mean()),
                loss_last=float(out["losses"][-10:].mean()), val_recall=out["val_recall"],
                val_precision=out["val_precision"], threshold_logit=out["threshold_logit"])
    log(f"predictor: {info}")
    return P.Predictor(mlp, out["threshold_logit"], K, words), info


def targets_for(batches, seed: int, height: int, width: int, device="cuda"):
    """Per-view smooth value noise (a 9 x 16 grid of seeded values, bilinearly
    upsampled), identical for every run."""
    out = []
    for t, b in enumerate(batches):
        g = torch.Generator().manual_seed(seed * 100003 + t)
        low = torch.rand((len(b), 3, 9, 16), generator=g)
        out.append(torch.nn.functional.interpolate(low, size=(height, width), mode="bilinear",
                                                   align_corners=False).to(device).contiguous())
    return out


def churn_stats(r_sets, k_sets) -> dict:
    """Residency churn of a run (the paper's churn table, App. B), from R_t
    and K_t per iteration:
      eviction rate      mean over t of |R_t minus R_{t+1}| / |R_t|;
      re-admission rate  mean over t of the blocks of R_{t+1} minus R_t that
                         had been resident before, over |R_{t+1}|;
      cold-restarted updates / updates   an update is a block rendered at t
                         (in K_t and R_t); it is cold-restarted when it is the
                         first update of a residency interval other than the
                         block's first;
      mean resident streak   mean length of the maximal runs of consecutive
                         iterations a block stays resident (runs cut by the
                         walk's end included)."""
    T = len(r_sets)
    Rs = [set(r) for r in r_sets]
    ev, re = [], []
    seen = set(Rs[0]) if T else set()
    for t in range(T - 1):
        if Rs[t]:
            ev.append(len(Rs[t] - Rs[t + 1]) / len(Rs[t]))
        new = Rs[t + 1] - Rs[t]
        if Rs[t + 1]:
            re.append(len(new & seen) / len(Rs[t + 1]))
        seen |= Rs[t + 1]
    updates = cold = 0
    interval_updated = {}       # block -> updated in its current interval
    intervals = {}              # block -> residency intervals begun so far
    streaks, open_run = [], {}
    for t in range(T):
        for k in Rs[t]:
            if t == 0 or k not in Rs[t - 1]:
                intervals[k] = intervals.get(k, 0) + 1
                interval_updated[k] = False
                open_run[k] = 0
            open_run[k] += 1
        if t > 0:
            for k in Rs[t - 1] - Rs[t]:
                streaks.append(open_run.pop(k))
        for k in set(k_sets[t]) & Rs[t]:
            updates += 1
            if not interval_updated[k]:
                interval_updated[k] = True
                cold += intervals[k] > 1
    streaks.extend(open_run.values())
    return dict(eviction_rate=round(float(np.mean(ev)) if ev else 0.0, 4),
                readmission_rate=round(float(np.mean(re)) if re else 0.0, 4),
                cold_restarted_update_ratio=round(cold / max(1, updates), 4),
                mean_resident_streak=round(float(np.mean(streaks)) if streaks else 0.0, 2),
                block_updates=updates)


def run(directory: str, N: int, B: int, batches, targets, capacity: int, spare: int, host_cache: int,
        predictor=None, io_threads: int = 8, no_tide: bool = False, no_overlap: bool = False,
        cold_restart: bool = False, bounded: bool = False, log=print):
    """One training run over the walk from the persisted base store
    (no_tide / no_overlap: the tier's ablation switches; cold_restart /
    bounded: the paper's default optimizer placement and a binding budget)."""
    tr = OutOfCoreTrainer(None, B, directory, capacity, spare, host_cache, n_rows=N, odirect=True,
                          io_threads=io_threads, predictor=predictor, no_tide=no_tide, no_overlap=no_overlap,
                          cold_restart=cold_restart, bounded=bounded)
    T = len(batches) - 1
    weights = None
    digests, losses, stalls, kset = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(T):
        s0 = tr.stall
        fr, loss = tr.iterate(batches[t], targets[t], batches[t + 1])
        if weights is None:
            g = torch.Generator(device=fr.image.device).manual_seed(12345)
            weights = torch.randint(1, 1 << 30, (fr.image.numel(),), generator=g, device=fr.image.device,
                                    dtype=torch.int64)
        digests.append((fr.image.reshape(-1).view(torch.int32).to(torch.int64) * weights).sum())
        losses.append(loss)
        stalls.append(tr.stall - s0)
        kset.append(len(tr.k_sets[-1]))
        if t % 25 == 24:
            log(f"  iteration {t + 1}/{T}: stall so far {sum(stalls):.2f} s, |K_t| {kset[-1]}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = tr.tier.stats()
    tr.tier.close()
    steady = stalls[1:]
    res = dict(iterations=T, wall_s=round(wall, 3), iters_per_s=round(T / wall, 3),
               stall_s_per_iter=round(float(np.mean(steady)), 5), stall_s_cold_start=round(stalls[0], 3),
               stall_s_total=round(float(np.sum(stalls)), 3), k_t_min=int(min(kset)), k_t_max=int(max(kset)),
               k_t_mean=round(float(np.mean(kset)), 1),
               ssd_read_GB=round(st["ssd_read_bytes"] / 1e9, 3), ssd_write_GB=round(st["ssd_write_bytes"] / 1e9, 3),
               h2d_GB=round(st["h2d_bytes"] / 1e9, 3), d2h_GB=round(st["d2h_bytes"] / 1e9, 3),
               pcie_GB_per_iter=round((st["h2d_bytes"] + st["d2h_bytes"]) / 1e9 / T, 4),
               blocks_in=st["blocks_in"], blocks_out=st["blocks_out"], readmissions=st["readmissions"],
               sync_fetches=st["sync_fetches"], host_hits=st["host_hits"], host_misses=st["host_misses"],
               host_hit_rate=round(st["host_hits"] / max(1, st["host_hits"] + st["host_misses"]), 4),
               prefetch_issued=st["prefetch_issued"], prefetch_used=st["prefetch_used"],
               skipped_blocks=st["skipped"],
               rendered_fraction=round(1.0 - st["skipped"] / max(1, sum(len(k) for k in tr.k_sets)), 4),
               churn=churn_stats(tr.r_sets, tr.k_sets))
    return res, [int(d.item()) for d in digests], [float(l) for l in losses]


def free_bytes(path: str) -> int:
    import shutil
    os.makedirs(path, exist_ok=True)
    return shutil.disk_usage(path).free
