"""The simulated-clock tier model (CPU): a hand-timed case, and that
prefetching the true future blocks removes stall without changing what is
rendered, while no hints reproduce exact-only streaming."""
import numpy as np

from tier_clock import ClockConfig, dry_city, simulate, walk_sets


def test_hand_timed_case():
    cfg = ClockConfig(capacity=4, host_blocks=4, ssd_ms=10.0, h2d_ms=1.0, c0_ms=5.0, c1_ms=0.0)
    sets = [[[0]], [[0, 1]], [[1, 2]]]
    r = simulate(sets, cfg)
    # t0: cold fetch of 0: SSD [0,10], H2D [10,11] -> stall 11; compute [11,16]
    #     Alg. 1 admits 1 at 11: SSD [11,21], H2D [21,22]
    # t1: stall 22-16 = 6; compute [22,27]; Alg. 1 admits 2 at 22: SSD [22,32], H2D [32,33]
    # t2: stall 33-27 = 6
    assert r.stall_ms == [11.0, 6.0, 6.0]
    assert r.demand_reads == 3
    # a hint for block 2 at t0 (start of compute, 11) reads it while the SSD is idle after 21
    r2 = simulate(sets, cfg, hints=[[2], None, None])
    # SSD: demand 1 [11,21], then the speculative 2 [21,31]; at t1 (22) Alg. 1 finds 2 in flight:
    # H2D at 31 -> [31,32]; t2 starts at 27: stall 5
    assert r2.stall_ms == [11.0, 6.0, 5.0]
    assert r2.prefetch_reads == 1 and r2.prefetch_used == 1


def test_future_blocks_prefetch_cuts_stall():
    sp, city = dry_city(80, 800.0)
    batches, sets = walk_sets(sp, city, 81, 160, z_far=250.0)
    sizes = [len(set(k for s in b for k in s)) for b in sets]
    cfg = ClockConfig(capacity=2 * max(sizes) + 8, host_blocks=4 * max(sizes), ssd_ms=8.0, h2d_ms=1.0,
                      c0_ms=40.0, c1_ms=0.0)
    base = simulate(sets, cfg)
    none = simulate(sets, cfg, hints=[None] * len(sets))
    assert none.stall_ms == base.stall_ms
    future = [sorted(set(k for h in range(2, 6) if t + h < len(sets) for s in sets[t + h] for k in s))
              for t in range(len(sets))]
    perfect = simulate(sets, cfg, hints=future)
    assert perfect.render_sets == base.render_sets
    assert perfect.total_stall_ms < 0.8 * base.total_stall_ms
    assert perfect.prefetch_used > 0
