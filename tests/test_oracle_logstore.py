"""Pins of the log-store oracle (O14, Sec. 3.4) on the CPU, then the
library's persisted store read through it.

Model pins: a plain dictionary of each block's last written bytes (the
definition of what a read must return) over random operation sequences;
versions strictly increasing by one per append; no append overwriting an
earlier version's bytes; a torn append resolving to the previous complete
version; compaction keeping every read and version.

Library against the oracle: the tier (host-memory pool, real segment files)
trains random blocks between checkpoints; after each checkpoint the oracle
reads every block straight from the segment files through the persisted
Index and must find the bytes the test wrote, with versions that grew
exactly for the blocks changed since the previous checkpoint, entries inside
their segments and no two records of a segment overlapping.  A torn append
after the last checkpoint and a compaction keep those reads.
"""
import os

import numpy as np

from oracle import logstore
from paper_2605_20150_amd.raster import Pool
from paper_2605_20150_amd.tier import Tier
from test_tier_cpu import B, build, scene


def rand_bytes(rng, n):
    return rng.integers(0, 256, size=n, dtype=np.uint8).tobytes()


def test_model_reads_follow_the_last_write_over_random_sequences():
    rng = np.random.default_rng(140)
    for trial in range(20):
        K, rec = int(rng.integers(1, 9)), int(rng.integers(1, 40))
        base = [rand_bytes(rng, rec) for _ in range(K)]
        m = logstore.LogStoreModel(base)
        truth = {k: base[k] for k in range(K)}
        writes = {k: 0 for k in range(K)}
        history = []      # (fid, off, bytes) of every version ever appended
        for step in range(60):
            op = rng.integers(0, 10)
            if op < 7:
                k = int(rng.integers(0, K))
                data = rand_bytes(rng, rec)
                before = m.index[k][3]
                m.append(k, data)
                truth[k] = data
                writes[k] += 1
                assert m.index[k][3] == before + 1
                history.append((m.index[k][0], m.index[k][1], data))
            elif op < 8:
                m.persist()
            elif op < 9:
                m.new_patch()
            else:
                m.compact()
                history = []
            for k in range(K):
                assert m.read(k) == truth[k], (trial, step, k)
                assert m.index[k][3] == writes[k]
            # appends never overwrite: every earlier version is still in place
            for fid, off, data in history:
                assert bytes(m.segments[fid][off:off + rec]) == data


def test_model_torn_append_resolves_to_the_previous_complete_version():
    rng = np.random.default_rng(141)
    K, rec = 5, 24
    base = [rand_bytes(rng, rec) for _ in range(K)]
    m = logstore.LogStoreModel(base)
    for k in (1, 3):
        m.append(k, rand_bytes(rng, rec))
    m.persist()
    saved = [m.read(k) for k in range(K)]
    saved_ver = [e[3] for e in m.index]
    m.append(1, rand_bytes(rng, rec))       # in flight when the machine stops
    assert m.read(1) != saved[1]
    m.crash(torn_bytes=rec // 2)
    assert [m.read(k) for k in range(K)] == saved
    assert [e[3] for e in m.index] == saved_ver
    # the store keeps working after the restart: the next append is version + 1
    m.append(1, b"x" * rec)
    assert m.read(1) == b"x" * rec and m.index[1][3] == saved_ver[1] + 1


def test_model_compaction_keeps_reads_and_versions():
    rng = np.random.default_rng(142)
    K, rec = 6, 16
    m = logstore.LogStoreModel([rand_bytes(rng, rec) for _ in range(K)])
    for _ in range(15):
        m.append(int(rng.integers(0, K)), rand_bytes(rng, rec))
    reads = [m.read(k) for k in range(K)]
    vers = [e[3] for e in m.index]
    m.compact()
    assert [m.read(k) for k in range(K)] == reads
    assert [e[3] for e in m.index] == vers
    assert m.index == [(0, k * rec, rec, vers[k]) for k in range(K)]
    assert len(m.segments) == 2 and not m.segments[1]


def record_bytes(pool, slot):
    """A block record as the tier stores it: params, m, v [59][B] f32, step [B] u32."""
    return b"".join(np.ascontiguousarray(getattr(pool, n)[slot].numpy()).tobytes()
                    for n in ("params", "exp_avg", "exp_avg_sq", "step"))


def check_persisted(directory, truth, prev_versions, changed):
    K, rec, nseg, index = logstore.read_persisted(directory)
    assert K == len(truth) and nseg >= 1
    spans = {}
    for k, (fid, off, size, ver) in enumerate(index):
        assert 0 <= fid < nseg and size == rec and off >= 0
        assert logstore.read_block(directory, index, k) == truth[k], k
        if prev_versions is not None:
            if k in changed:
                assert ver > prev_versions[k], (k, ver, prev_versions[k])
            else:
                assert ver == prev_versions[k], (k, ver, prev_versions[k])
        spans.setdefault(fid, []).append((off, off + size))
    for fid, sp in spans.items():
        sp.sort()
        size = os.path.getsize(logstore.segment_path(directory, fid))
        assert sp[-1][1] <= size
        assert all(a[1] <= b[0] for a, b in zip(sp, sp[1:])), f"overlapping records in segment {fid}"
    return [e[3] for e in index]


def test_library_store_read_through_the_oracle(tmp_path):
    th = scene()
    t, pool = build(tmp_path, th, n_slots=4, capacity=4, cache=4)
    d = str(tmp_path / "store")
    t.checkpoint()
    truth = {k: b"" for k in range(t.K)}
    for k in range(t.K):
        r = t.read_block(k)
        truth[k] = b"".join(np.ascontiguousarray(r[n]).tobytes() for n in ("params", "exp_avg", "exp_avg_sq", "step"))
    vers = check_persisted(d, truth, None, set())
    assert vers == [0] * t.K
    rng = np.random.default_rng(143)
    for rnd in range(4):
        changed = set()
        for it in range(8):
            Kt = sorted(rng.choice(t.K, 2, replace=False).tolist())
            t.ensure_resident(Kt)
            slots = t.resident_slots()
            for k in Kt:
                if rng.random() < 0.7:
                    s = slots[k]
                    pool.params[s] += float(rng.normal())
                    pool.exp_avg[s] += 1.0
                    pool.step[s] += 1
                    t.dirty[k] = 1
                    changed.add(k)
                    truth[k] = record_bytes(pool, s)
            t.end_iteration()
            t.stream_delta([sorted(rng.choice(t.K, 2, replace=False).tolist())])
            t.sync_bounds()
        t.checkpoint()
        vers = check_persisted(d, truth, vers, changed)
        assert changed
    # a torn append after the last checkpoint: the persisted Index never
    # names the torn bytes
    t.close()
    patches = sorted(p for p in os.listdir(d) if p.startswith("patch_"))
    last = os.path.join(d, patches[-1])
    with open(last, "ab") as f:
        f.write(b"\x7f" * (t.rec_bytes // 3))
    check_persisted(d, truth, vers, set())
    # compaction: every entry in the new base at k * rec, versions kept
    pool2 = Pool.empty(4, B, "cpu")
    t2 = Tier(d, th.shape[0], pool2, 4, 4, host_pool=True)
    t2.open()
    t2.compact()
    t2.close()
    K, rec, nseg, index = logstore.read_persisted(d)
    assert [e[0] for e in index] == [0] * K
    assert [e[1] for e in index] == [k * rec for k in range(K)]
    check_persisted(d, truth, vers, set())
