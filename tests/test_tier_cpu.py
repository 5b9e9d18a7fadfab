"""The block tier on the CPU: the library's host-memory backend stands in for
the GPU pool (same slot API, copies are memcpy), real segment files stand in
for the SSD.  Checks the log store, the host cache and write-back, Alg. 1
against the oracle, Level-1 culling against the oracle, and crash
consistency of the persisted Index."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2605_20150_amd import synth
from paper_2605_20150_amd.raster import D, Pool
from paper_2605_20150_amd.tier import Tier

B = 256


def scene(n=2500, seed=40):
    th = synth.dense_scene(n, seed, extent=3.0, logscale_mu=-3.0)
    cell = np.floor((th[:, :3] + 3.0) / 1.0).astype(int)
    return th[np.lexsort((cell[:, 2], cell[:, 1], cell[:, 0]))]


def build(tmp_path, th, n_slots=6, capacity=6, cache=4, name="store", odirect=False, rows=B, **flags):
    pool = Pool.empty(n_slots, rows, "cpu")
    t = Tier(str(tmp_path / name), th.shape[0], pool, capacity, cache, io_threads=2, host_pool=True, kappa=1.32,
             odirect=odirect, **flags)
    for k in range(t.K):
        r = th[k * rows:(k + 1) * rows]
        t.put_block(k, r.T)
    t.finalize()
    return t, pool


def test_store_roundtrip_and_spheres(tmp_path):
    th = scene()
    t, pool = build(tmp_path, th)
    assert t.K == 10
    for k in range(t.K):
        r = t.read_block(k)
        rows = th[k * B:(k + 1) * B]
        assert np.array_equal(r["params"][:, :len(rows)], rows.T)
        assert not r["exp_avg"].any() and not r["exp_avg_sq"].any() and not r["step"].any()
    ref = oracle.block_spheres(th.astype(np.float64), B, 1.32)
    sp = t.host_spheres()
    assert np.allclose(sp[:, :3], ref[:, :3], rtol=1e-6, atol=1e-6)
    assert (sp[:, 3] >= ref[:, 3]).all() and np.allclose(sp[:, 3], ref[:, 3], rtol=1e-5)
    t.close()


def test_cull_matches_oracle(tmp_path):
    th = scene()
    t, _ = build(tmp_path, th)
    rng = np.random.default_rng(41)
    sp = t.host_spheres().astype(np.float64)
    for _ in range(50):
        eye = rng.normal(0, 4, size=3)
        cam = synth.look_at(eye, rng.normal(0, 1, size=3), rng.normal(size=3), 96, 64, rng.uniform(40, 120),
                            z_far=rng.uniform(2, 10))
        got = t.cull([cam])[0]
        ref = np.where(oracle.cull_blocks(sp, synth.cams_array([cam]))[0])[0]
        assert got.tolist() == ref.tolist()
    t.close()


def walk_sets(rng, K, steps, J=2, width=3):
    """Per-camera block sets that drift along the block ids."""
    pos = 0
    out = []
    for _ in range(steps):
        pos = (pos + int(rng.integers(0, 2))) % K
        out.append([sorted({(pos + j + int(d)) % K for d in rng.integers(0, width, size=2)}) for j in range(J)])
    return out


def test_alg1_decisions_match_oracle(tmp_path):
    th = scene()
    t, pool = build(tmp_path, th, n_slots=6, capacity=6, cache=6)
    rng = np.random.default_rng(42)
    sets = walk_sets(rng, t.K, 40)
    age = np.full(t.K, 1e9)
    R = []
    Kt = sorted(set(x for s in sets[0] for x in s))
    t.ensure_resident(Kt)          # cold start: these blocks are fetched synchronously
    cold = len(Kt)
    R = sorted(t.resident_slots())
    for i in range(1, len(sets)):
        Rn, sp_ref, sm_ref, age, _ = oracle.alg1(R, Kt, sets[i], age, 0.75, 0.9, 6)
        t.end_iteration()
        sp, sm = t.stream_delta(sets[i])
        t.sync_bounds()
        assert sp.tolist() == sp_ref and sm.tolist() == sm_ref, i
        Kt = sorted(set(x for s in sets[i] for x in s))
        stall = t.ensure_resident(Kt)
        assert stall >= 0
        R = sorted(t.resident_slots())
        assert R == Rn.tolist()
        assert set(Kt) <= set(R)
    st = t.stats()
    assert st["sync_fetches"] == cold and st["blocks_in"] > 0
    t.close()


def test_stream_delta_rejects_a_small_output_without_changing_state(tmp_path):
    """An output array too small for S+ or S- (the other one null) is an
    argument error, whichever of the two is given, and the rejected call
    leaves the tier as it was: the next call's S+ and S- still follow Alg. 1
    from the state before the rejection."""
    import ctypes as C

    from paper_2605_20150_amd import _lib as L
    th = scene()
    t, pool = build(tmp_path, th, n_slots=6, capacity=6, cache=6)
    rng = np.random.default_rng(44)
    sets = walk_sets(rng, t.K, 30)
    age = np.full(t.K, 1e9)
    Kt = sorted(set(x for s in sets[0] for x in s))
    t.ensure_resident(Kt)
    R = sorted(t.resident_slots())
    tried = {"plus": 0, "minus": 0}
    for i in range(1, len(sets)):
        Rn, sp_ref, sm_ref, age, _ = oracle.alg1(R, Kt, sets[i], age, 0.75, 0.9, 6)
        t.end_iteration()
        lists = [sorted(set(int(x) for x in k)) for k in sets[i]]
        flat = np.ascontiguousarray([x for l in lists for x in l] or [0], dtype=np.int32)
        counts = np.ascontiguousarray([len(l) for l in lists], dtype=np.int32)
        buf = np.zeros(t.K, dtype=np.int32)
        npl, nmi = C.c_int32(-7), C.c_int32(-7)
        pi32 = C.POINTER(C.c_int32)
        fp, cp, bp = (a.ctypes.data_as(pi32) for a in (flat, counts, buf))
        for which, need in (("plus", len(sp_ref)), ("minus", len(sm_ref))):
            if need == 0:
                continue
            args = (bp, None) if which == "plus" else (None, bp)
            rc = t.lib.tide_stream_delta(t.h, fp, cp, len(lists), None, args[0], C.byref(npl), args[1],
                                         C.byref(nmi), need - 1)
            assert rc == L.TIDE_EINVAL, (i, which, rc)
            assert npl.value == -7 and nmi.value == -7 and not buf.any()
            tried[which] += 1
        sp, sm = t.stream_delta(sets[i])
        t.sync_bounds()
        assert sp.tolist() == sp_ref and sm.tolist() == sm_ref, i
        Kt = sorted(set(x for s in sets[i] for x in s))
        t.ensure_resident(Kt)
        R = sorted(t.resident_slots())
        assert R == Rn.tolist()
    assert tried["plus"] > 0 and tried["minus"] > 0
    t.close()


def test_residency_moves_data_and_writes_back(tmp_path, odirect=False):
    """Blocks updated while resident are written back through the host cache
    (dirty) to patch segments; a tiny host cache forces flushes; a reopened
    store reads the newest versions."""
    th = scene()
    t, pool = build(tmp_path, th, n_slots=4, capacity=4, cache=4, odirect=odirect)
    rng = np.random.default_rng(43)
    truth = {k: t.read_block(k) for k in range(t.K)}
    for it in range(30):
        Kt = sorted(rng.choice(t.K, 2, replace=False).tolist())
        t.ensure_resident(Kt)
        slots = t.resident_slots()
        for k in Kt:
            s = slots[k]
            for name in ("params", "exp_avg", "exp_avg_sq"):
                assert np.array_equal(getattr(pool, name)[s].numpy(), truth[k][name]), (it, k, name)
            # "train" the block: change parameters, moments and steps, mark dirty
            pool.params[s] += 0.5
            pool.exp_avg[s] += 1.0
            pool.exp_avg_sq[s] += 2.0
            pool.step[s] += 1
            t.dirty[k] = 1
            truth[k] = dict(params=pool.params[s].numpy().copy(), exp_avg=pool.exp_avg[s].numpy().copy(),
                            exp_avg_sq=pool.exp_avg_sq[s].numpy().copy(),
                            step=pool.step[s].numpy().view(np.uint32).copy())
        t.end_iteration()
        nxt = sorted(rng.choice(t.K, 2, replace=False).tolist())
        t.stream_delta([nxt])
        t.sync_bounds()
    for k in range(t.K):
        r = t.read_block(k)
        for name in ("params", "exp_avg", "exp_avg_sq", "step"):
            assert np.array_equal(r[name], truth[k][name]), (k, name)
    st = t.stats()
    assert st["ssd_write_bytes"] > 0 and st["blocks_out"] > 0 and st["readmissions"] > 0
    t.checkpoint()
    t.close()
    pool2 = Pool.empty(4, B, "cpu")
    t2 = Tier(str(tmp_path / "store"), th.shape[0], pool2, 4, 4, host_pool=True, odirect=odirect)
    t2.open()
    for k in range(t2.K):
        r = t2.read_block(k)
        for name in ("params", "exp_avg", "exp_avg_sq", "step"):
            assert np.array_equal(r[name], truth[k][name]), (k, name)
    t2.close()


def test_crash_mid_append_keeps_the_persisted_versions(tmp_path):
    th = scene()
    t, pool = build(tmp_path, th, n_slots=4, capacity=4, cache=4)
    t.ensure_resident([0, 1])
    slots = t.resident_slots()
    for k in (0, 1):
        pool.params[slots[k]] += 1.0
        t.dirty[k] = 1
    t.end_iteration()
    t.sync_bounds()
    t.checkpoint()
    saved = {k: t.read_block(k)["params"].copy() for k in (0, 1)}
    # more updates after the checkpoint, flushed to a patch segment
    for k in (0, 1):
        pool.params[slots[k]] += 5.0
        t.dirty[k] = 1
    t.end_iteration()
    t.stream_delta([[5, 6]])
    t.sync_bounds()
    t.ensure_resident([5, 6])
    for k in (7, 8, 9, 2):          # pressure the 4-block host cache: dirty entries get flushed
        t.stream_delta([[k]])
        t.ensure_resident([k])
    newest = t.read_block(0)["params"]
    assert np.allclose(newest, saved[0] + 5.0)        # read-after-write
    t.close()                                          # "crash": no checkpoint
    d = tmp_path / "store"
    patches = sorted(p for p in os.listdir(d) if p.startswith("patch_"))
    last = d / patches[-1]
    size = os.path.getsize(last)
    if size:
        with open(last, "r+b") as f:                   # a torn append
            f.truncate(size - t.rec_bytes // 2)
    pool2 = Pool.empty(4, B, "cpu")
    t2 = Tier(str(d), th.shape[0], pool2, 4, 4, host_pool=True)
    t2.open()
    for k in (0, 1):
        assert np.array_equal(t2.read_block(k)["params"], saved[k])
    t2.close()


def test_prefetch_feeds_the_host_cache(tmp_path):
    th = scene()
    t, pool = build(tmp_path, th, n_slots=4, capacity=4, cache=6)
    t.ensure_resident([0])
    t.prefetch([3, 4], horizon=2)
    t.end_iteration()
    t.stream_delta([[3, 4]])
    t.sync_bounds()
    t.ensure_resident([3, 4])
    st = t.stats()
    assert st["prefetch_issued"] == 2 and st["prefetch_used"] == 2
    t.close()


def test_direct_io_write_back_and_reopen(tmp_path):
    """The same data path with O_DIRECT segment files (block_rows a multiple
    of 512): updates written back through the host cache survive a reopen."""
    th = scene(n=3000)
    R = 512
    t, pool = build(tmp_path, th, n_slots=3, capacity=3, cache=4, odirect=True, rows=R)
    assert t.K == 6
    truth = {k: t.read_block(k)["params"].copy() for k in range(t.K)}
    rng = np.random.default_rng(44)
    for it in range(12):
        Kt = sorted(rng.choice(t.K, 2, replace=False).tolist())
        t.ensure_resident(Kt)
        slots = t.resident_slots()
        for k in Kt:
            assert np.array_equal(pool.params[slots[k]].numpy(), truth[k])
            pool.params[slots[k]] += 0.25
            t.dirty[k] = 1
            truth[k] = pool.params[slots[k]].numpy().copy()
        t.end_iteration()
        t.stream_delta([sorted(rng.choice(t.K, 2, replace=False).tolist())])
        t.sync_bounds()
    t.checkpoint()
    t.close()
    pool2 = Pool.empty(3, R, "cpu")
    t2 = Tier(str(tmp_path / "store"), th.shape[0], pool2, 3, 4, host_pool=True, odirect=True)
    t2.open()
    for k in range(t2.K):
        assert np.array_equal(t2.read_block(k)["params"], truth[k]), k
    t2.close()


def _trained_walk(tmp_path, name, **flags):
    """A drifting two-camera walk in which every rendered block is updated:
    per delta S+ and S-, the resident set after each ensure, the final
    blocks and the counters."""
    th = scene()
    t, pool = build(tmp_path, th, n_slots=6, capacity=6, cache=4, name=name, **flags)
    sets = walk_sets(np.random.default_rng(45), t.K, 30)
    deltas, resident = [], []
    for i, cams in enumerate(sets):
        Kt = sorted(set(x for c in cams for x in c))
        t.ensure_resident(Kt)
        resident.append(sorted(t.resident_slots()))
        slots = t.resident_slots()
        for k in Kt:
            pool.params[slots[k]] += 0.125 * (k + 1)
            pool.step[slots[k]] += 1
            t.dirty[k] = 1
        t.end_iteration()
        if i + 1 < len(sets):
            sp, sm = t.stream_delta(sets[i + 1])
            deltas.append((sp.tolist(), sm.tolist()))
        t.sync_bounds()
    blocks = [t.read_block(k) for k in range(t.K)]
    st = t.stats()
    t.close()
    return sets, deltas, resident, blocks, st


@pytest.mark.parametrize("flag", ["no_tide", "no_overlap"])
def test_ablation_switches_change_the_schedule_not_the_data(tmp_path, flag):
    """Sec. 4.4's ablations.  Without differential streaming every block of
    K_{t+1} moves again (S+ = K_{t+1}, S- = R_t, R_{t+1} = K_{t+1}) and the
    host-to-device traffic grows; without overlap the decisions are the full
    method's.  Either way every block ends with the same bytes."""
    sets, d_full, r_full, b_full, s_full = _trained_walk(tmp_path, "full")
    _, d_abl, r_abl, b_abl, s_abl = _trained_walk(tmp_path, flag, **{flag: True})
    for k, (a, b) in enumerate(zip(b_full, b_abl)):
        for name in ("params", "exp_avg", "exp_avg_sq", "step"):
            assert np.array_equal(a[name], b[name]), (flag, k, name)
    if flag == "no_overlap":
        assert d_abl == d_full and r_abl == r_full
        assert s_abl["h2d_bytes"] == s_full["h2d_bytes"]
    else:
        for i, (sp, sm) in enumerate(d_abl):
            nxt = sorted(set(x for c in sets[i + 1] for x in c))
            assert sorted(sp) == nxt and sorted(sm) == r_abl[i], i
            assert r_abl[i + 1] == nxt, i
        assert s_abl["h2d_bytes"] > s_full["h2d_bytes"]
        assert s_abl["blocks_in"] == sum(len(sp) for sp, _ in d_abl)


def test_host_cache_pinned_by_the_iteration_in_flight_is_an_error(tmp_path):
    """Blocks of the iteration in flight that leave the GPU stay pinned in the
    host cache until the next sync_bounds.  When they fill it, the delta
    reports the cache as too small instead of waiting forever."""
    th = scene()
    t, pool = build(tmp_path, th, n_slots=6, capacity=6, cache=4, no_tide=True)
    Kt = [0, 1, 2, 3, 4]
    t.ensure_resident(Kt)
    t.end_iteration()
    with pytest.raises(RuntimeError, match="too small"):
        t.stream_delta([[5, 6, 7, 8, 9]])
    t.close()


def test_cold_restart_moves_parameters_only_and_zeroes_the_moments(tmp_path):
    """Sec. 3.5's default placement: a block that leaves and comes back keeps
    its trained parameters and restarts m, v and its steps from zero; only
    parameters cross PCIe."""
    th = scene()
    t, pool = build(tmp_path, th, n_slots=4, capacity=4, cache=6, cold_restart=True)
    pbytes = 59 * B * 4
    t.ensure_resident([0, 1])
    s = t.resident_slots()
    for k in (0, 1):
        pool.params[s[k]] += 0.5
        pool.exp_avg[s[k]] += 1.0
        pool.exp_avg_sq[s[k]] += 2.0
        pool.step[s[k]] += 3
        t.dirty[k] = 1
    trained = {k: pool.params[s[k]].numpy().copy() for k in (0, 1)}
    t.end_iteration()
    t.stream_delta([[2, 3, 4, 5]])          # 0 and 1 leave
    t.sync_bounds()
    t.ensure_resident([2, 3, 4, 5])
    assert 0 not in t.resident() and 1 not in t.resident()
    t.end_iteration()
    t.stream_delta([[0, 1]])                # and come back
    t.sync_bounds()
    t.ensure_resident([0, 1])
    s = t.resident_slots()
    for k in (0, 1):
        assert np.array_equal(pool.params[s[k]].numpy(), trained[k])
        assert not pool.exp_avg[s[k]].any() and not pool.exp_avg_sq[s[k]].any() and not pool.step[s[k]].any()
    st = t.stats()
    assert st["h2d_bytes"] == pbytes * (st["blocks_in"] + st["sync_fetches"])
    assert st["d2h_bytes"] % pbytes == 0 and st["d2h_bytes"] > 0
    t.close()


def test_bounded_budget_follows_alg1_and_renders_the_resident_part(tmp_path):
    """A budget C below |K_{t+1}|: the camera-balanced Top-C decisions match
    the oracle, the render order holds K_t's resident blocks only, nothing is
    fetched outside the deltas, and the skipped blocks are counted."""
    th = scene()
    C_ = 5
    t, pool = build(tmp_path, th, n_slots=C_, capacity=C_, cache=8, bounded=True)
    rng = np.random.default_rng(46)
    sets = []
    for i in range(25):
        sets.append([sorted(set(((i // 2 + j * 3 + rng.integers(0, 5, size=3)) % t.K).tolist())) for j in range(2)])
    age = np.full(t.K, 1e9)
    R, Kprev = [], []
    skipped = 0
    for i, cams in enumerate(sets):
        Kt = sorted(set(x for c in cams for x in c))
        Rn, sp_ref, sm_ref, age, _ = oracle.alg1(R, Kprev, cams, age, 0.75, 0.9, C_)
        if i == 0:
            sp, sm = t.stream_delta(cams)
        assert sorted(sp.tolist()) == sp_ref and sorted(sm.tolist()) == sm_ref, i
        t.ensure_resident(Kt)
        R = t.resident()
        assert R == Rn.tolist() and len(R) <= C_, i
        rendered = [k for k in Kt if k in set(R)]
        order = pool.order[:pool.n_order].numpy().tolist()
        slots = t.resident_slots()
        assert order == [slots[k] for k in rendered], i
        skipped += len(Kt) - len(rendered)
        t.end_iteration()
        if i + 1 < len(sets):
            sp, sm = t.stream_delta(sets[i + 1])
        t.sync_bounds()
        Kprev = [k for k in Kt if k in set(R)]
    st = t.stats()
    assert st["sync_fetches"] == 0 and st["skipped"] == skipped and skipped > 0
    t.close()


def test_churn_statistics_on_a_hand_counted_walk():
    """Block 1 leaves at t = 2 and comes back at t = 3: eviction rates
    0, 1/2, 0; re-admission rates 0, 0, 1/2; seven block updates of which the
    first after the return is cold-restarted; streaks 4 (block 0), 2 and 1
    (block 1)."""
    from paper_2605_20150_amd.city import churn_stats
    r = [[0, 1], [0, 1], [0], [0, 1]]
    c = churn_stats(r, r)
    assert c["eviction_rate"] == round(0.5 / 3, 4) and c["readmission_rate"] == round(0.5 / 3, 4)
    assert c["block_updates"] == 7 and c["cold_restarted_update_ratio"] == round(1 / 7, 4)
    assert c["mean_resident_streak"] == round(7 / 3, 2)
    # a block resident but outside K_t is not updated; first admissions are not restarts
    c = churn_stats([[0, 1], [0, 2]], [[0], [0, 2]])
    assert c["block_updates"] == 3 and c["cold_restarted_update_ratio"] == 0.0


def _table(tmp_path, n=3001, seed=47):
    th = synth.dense_scene(n, seed, extent=3.0, logscale_mu=-3.0).astype(np.float32)
    th[100:110, :3] = th[5, :3]             # equal centres: ties keep row order
    path = tmp_path / "table.f32"
    th.tofile(path)
    return th, str(path)


@pytest.mark.parametrize("run_rows", [3001, 700, 64])
def test_out_of_core_layout_equals_the_oracle_morton_blocks(tmp_path, run_rows):
    """Sec. 3.3's layout from a table file through sorted runs on disk and a
    k-way merge: every block holds the rows of the oracle's stable Morton
    order (one run, several, many; a ragged last block), the spheres are the
    oracle's, the run files are gone and the store reopens."""
    th, path = _table(tmp_path)
    N = th.shape[0]
    t = Tier(str(tmp_path / "store"), N, Pool.empty(4, B, "cpu"), 4, 4, host_pool=True, kappa=1.32)
    t.layout_build(path, str(tmp_path), run_rows)
    ref = th[oracle.morton_order(th[:, :3])]
    assert t.K == 12
    for k in range(t.K):
        rows = ref[k * B:(k + 1) * B]
        assert np.array_equal(t.read_block(k)["params"][:, :len(rows)], rows.T), k
    sp = oracle.block_spheres(ref.astype(np.float64), B, 1.32)
    got = t.host_spheres()
    assert np.allclose(got[:, :3], sp[:, :3], rtol=1e-6, atol=1e-6) and (got[:, 3] >= sp[:, 3]).all()
    assert not [p for p in os.listdir(tmp_path) if p.startswith("tide_run_")]
    t.close()
    t2 = Tier(str(tmp_path / "store"), N, Pool.empty(4, B, "cpu"), 4, 4, host_pool=True)
    t2.open()
    assert np.array_equal(t2.read_block(11)["params"][:, :N - 11 * B], ref[11 * B:].T)
    t2.close()


def test_out_of_core_layout_rejects_bad_inputs(tmp_path):
    th, path = _table(tmp_path)
    t = Tier(str(tmp_path / "s1"), th.shape[0] + 1, Pool.empty(4, B, "cpu"), 4, 4, host_pool=True)
    with pytest.raises(RuntimeError, match="expected"):
        t.layout_build(path, str(tmp_path), 700)       # file holds one row fewer than N
    t.close()
    t = Tier(str(tmp_path / "s2"), th.shape[0], Pool.empty(4, B, "cpu"), 4, 4, host_pool=True)
    with pytest.raises(RuntimeError, match="runs"):
        t.layout_build(path, str(tmp_path), 5)         # 601 runs: more than 512 open files
    t.close()


def test_compaction_merges_the_patches_and_keeps_the_newest_versions(tmp_path):
    """Sec. 3.4's optional compaction: after write-backs spread blocks over
    patch segments, compaction leaves one base segment holding every block's
    newest version; training continues (new patches) and a reopened store
    reads the newest versions."""
    th = scene()
    t, pool = build(tmp_path, th, n_slots=4, capacity=4, cache=4)
    rng = np.random.default_rng(48)
    truth = {k: t.read_block(k)["params"].copy() for k in range(t.K)}

    def train(iters):
        for _ in range(iters):
            Kt = sorted(rng.choice(t.K, 2, replace=False).tolist())
            t.ensure_resident(Kt)
            slots = t.resident_slots()
            for k in Kt:
                assert np.array_equal(pool.params[slots[k]].numpy(), truth[k])
                pool.params[slots[k]] += 0.25
                t.dirty[k] = 1
                truth[k] = pool.params[slots[k]].numpy().copy()
            t.end_iteration()
            t.stream_delta([sorted(rng.choice(t.K, 2, replace=False).tolist())])
            t.sync_bounds()

    d = tmp_path / "store"
    train(25)
    t.checkpoint()
    assert sum(os.path.getsize(d / p) for p in os.listdir(d) if p.startswith("patch_")) > 0
    t.compact()
    assert sorted(p for p in os.listdir(d) if p.endswith(".seg")) == ["base.seg", "patch_000001.seg"]
    assert os.path.getsize(d / "patch_000001.seg") == 0
    for k in range(t.K):
        assert np.array_equal(t.read_block(k)["params"], truth[k]), k
    train(10)
    t.checkpoint()
    t.close()
    t2 = Tier(str(d), th.shape[0], Pool.empty(4, B, "cpu"), 4, 4, host_pool=True)
    t2.open()
    for k in range(t2.K):
        assert np.array_equal(t2.read_block(k)["params"], truth[k]), k
    t2.close()
