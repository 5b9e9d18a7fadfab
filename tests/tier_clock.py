"""Simulated-clock model of the streaming tier (test infrastructure).

Replays a walk's exact block sets through Alg. 1 (the oracle's) and a
deterministic timing model of the tier, so that the stall a prefetch policy
saves can be measured without SSD or PCIe noise.  The model follows the
library's schedule:

  iteration t   wait until every block of K_t is on the GPU (the stall),
                then compute for c0 + c1 |K_t|;
                at the start of compute, prefetch hints (if any) queue
                speculative SSD reads into the host cache;
                Alg. 1 picks S+ for t+1: a block in the host cache (or
                already being read) goes host -> GPU when it is there, a
                block that is not is read from the SSD first (demand read);
                evicted blocks S- land in the host cache.

The SSD serves demand reads before speculative ones (one non-preemptive
server, each class FIFO), the host-to-device link is one FIFO server.  The
host cache is an LRU of H blocks; an entry whose read is still in flight is
never evicted.  As in the library, a hint never takes an entry filled by a
prefetch of the last 4 iterations that is still unused, at most
``spec_cap`` speculative reads are outstanding, and the rest of a hint list
is dropped."""
from __future__ import annotations

from collections import OrderedDict
from dataclasses import dataclass, field

import numpy as np

import oracle


@dataclass
class ClockConfig:
    capacity: int            # GPU block slots C
    host_blocks: int         # host cache H
    ssd_ms: float            # SSD read time of one block
    h2d_ms: float            # host-to-device time of one block
    c0_ms: float             # compute time per iteration: c0 + c1 |K_t|
    c1_ms: float
    lam: float = 0.75
    gamma: float = 0.9
    spec_cap: int | None = None   # outstanding speculative reads (None: unbounded)
    prefetch_ttl: int = 4


@dataclass
class ClockResult:
    stall_ms: list = field(default_factory=list)
    demand_reads: int = 0
    prefetch_reads: int = 0
    prefetch_used: int = 0
    render_sets: list = field(default_factory=list)

    @property
    def total_stall_ms(self) -> float:
        return float(sum(self.stall_ms))


class _Ssd:
    def __init__(self, ms):
        self.ms = ms
        self.free = 0.0
        self.low = []           # queued speculative reads: (arrival, block)

    def advance(self, until, host):
        while self.low:
            arr, k = self.low[0]
            start = max(self.free, arr)
            if start >= until:
                break
            self.low.pop(0)
            self.free = start + self.ms
            host[k] = self.free

    def demand(self, t):
        start = max(self.free, t)
        self.free = start + self.ms
        return self.free


def simulate(per_cam_sets, cfg: ClockConfig, hints=None) -> ClockResult:
    """per_cam_sets[t] = list of per-camera block-id lists of batch t.
    hints[t] = block ids to prefetch at iteration t (or None)."""
    n_blocks = 1 + max(int(k) for cams in per_cam_sets for s in cams for k in s)
    res = ClockResult()
    ssd = _Ssd(cfg.ssd_ms)
    host = OrderedDict()        # block -> time its host copy is ready (may be in the future)
    spec = {}                   # host entries filled by a prefetch and not yet used -> iteration
    pcie = 0.0
    gpu_ready = {}
    R = []
    age = np.full(n_blocks, 1e9)
    now = 0.0

    def host_insert(k, ready, t, it=None):
        """it: the iteration of a speculative insert (protects recent unused prefetches)."""
        if it is not None:
            victim = next((b for b, r in host.items() if r <= t and not
                           (b in spec and it - spec[b] <= cfg.prefetch_ttl)), None)
            if len(host) >= cfg.host_blocks and victim is None:
                return False
        host[k] = ready
        host.move_to_end(k)
        while len(host) > cfg.host_blocks:
            victim = next((b for b, r in host.items() if r <= t and b != k and not
                           (it is not None and b in spec and it - spec[b] <= cfg.prefetch_ttl)), None)
            if victim is None:
                return False
            del host[victim]
            spec.pop(victim, None)
        return True

    def to_gpu(k, t):
        nonlocal pcie
        ssd.advance(t, host)
        if k in host:
            ready = host[k]
            host.move_to_end(k)
            if k in spec:
                del spec[k]
                res.prefetch_used += 1
            # a queued speculative read of k becomes a demand read
            for i, (_, b) in enumerate(ssd.low):
                if b == k:
                    ssd.low.pop(i)
                    ready = ssd.demand(t)
                    host[k] = ready
                    break
        else:
            ready = ssd.demand(t)
            res.demand_reads += 1
            host_insert(k, ready, t)
        start = max(pcie, ready, t)
        pcie = start + cfg.h2d_ms
        gpu_ready[k] = pcie

    T = len(per_cam_sets)
    for t in range(T):
        Kt = sorted(set(int(k) for s in per_cam_sets[t] for k in s))
        res.render_sets.append(Kt)
        Rset = set(R)
        for k in Kt:                              # sync fetch (cold start only when Alg. 1 keeps up)
            if k not in Rset:
                to_gpu(k, now)
        if not R:
            R = Kt
        wait = max([gpu_ready.get(k, now) for k in Kt] + [now])
        stall = wait - now
        res.stall_ms.append(stall)
        now = wait
        end = now + cfg.c0_ms + cfg.c1_ms * len(Kt)
        if hints is not None and hints[t] is not None:
            ssd.advance(now, host)
            Rset = set(R)
            outstanding = sum(1 for b in spec if host.get(b, 0.0) > now)
            for k in hints[t]:
                k = int(k)
                if cfg.spec_cap is not None and outstanding >= cfg.spec_cap:
                    break
                if k in Rset or k in host:
                    continue
                if not host_insert(k, float("inf"), now, it=t):
                    break
                ssd.low.append((now, k))
                spec[k] = t
                res.prefetch_reads += 1
                outstanding += 1
        if t + 1 < T:
            Rn, Sp, Sm, age, _ = oracle.alg1(R, Kt, per_cam_sets[t + 1], age, cfg.lam, cfg.gamma, cfg.capacity)
            for k in Sm:
                gpu_ready.pop(k, None)
                host_insert(k, now, now)
            for k in Sp:
                to_gpu(k, now)
            R = Rn.tolist()
        now = end
    return res


# ------------------------------------------------------------- dry-run inputs

def dry_city(seed: int, extent: float, blocks_per_km2: float = 954.0, samples: int = 64, kappa: float = 1.32):
    """Block spheres of a synthetic city with the block density of the
    1B-Gaussian street city (15 259 blocks over 16 km^2), each block's
    sphere computed from a sample of ``samples`` of its Gaussians: the
    library's Morton layout order, then its block-sphere routine."""
    from paper_2605_20150_amd import predictor as P
    from paper_2605_20150_amd import synth
    K = max(1, int(round(blocks_per_km2 * (extent / 1000.0) ** 2)))
    th, city = synth.city_scene(K * samples, seed, extent=extent)
    th = th[P.morton_order(th)]
    return P.block_spheres(th, samples, kappa), city


def walk_sets(spheres, city, seed: int, n_iters: int, z_far: float, poses_per_batch: int = 4):
    """Camera batches of a street walk and, per batch, the per-camera Level-1
    block lists (from the library's culler)."""
    from paper_2605_20150_amd import predictor as P
    from paper_2605_20150_amd import synth
    cams = synth.street_walk(city, n_iters * poses_per_batch, seed, z_far=z_far)
    batches = [cams[poses_per_batch * t:poses_per_batch * (t + 1)] for t in range(n_iters)]
    K = spheres.shape[0]
    words = (K + 31) // 32
    sets = [[P.bits_to_ids(P.cull_bits(spheres, [c], words), K).tolist() for c in b] for b in batches]
    return batches, sets
