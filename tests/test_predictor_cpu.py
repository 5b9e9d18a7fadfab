"""Host side of the layout and the predictor's data path (CPU): Morton
layout order, block spheres and the culling bitset against the oracle, pose
features against their definition, pair logging, and the street walks."""
import numpy as np

import oracle
from paper_2605_20150_amd import predictor as P
from paper_2605_20150_amd import synth


def test_morton_order_matches_oracle():
    th, _ = synth.city_scene(60_000, 30, extent=1000.0)
    assert np.array_equal(P.morton_order(th), oracle.morton_order(th[:, :3].astype(np.float64)))
    # degenerate inputs: one row, all rows equal, a flat axis
    assert P.morton_order(th[:1]).tolist() == [0]
    same = np.repeat(th[:1], 7, axis=0)
    assert P.morton_order(same).tolist() == list(range(7))
    flat = th[:5000].copy()
    flat[:, 2] = 3.0
    assert np.array_equal(P.morton_order(flat), oracle.morton_order(flat[:, :3].astype(np.float64)))


def test_block_spheres_and_cull_bits_match_oracle():
    th, city = synth.city_scene(40_000, 31, extent=1000.0)
    th = th[P.morton_order(th)]
    B = 256
    sp = P.block_spheres(th, B, kappa=1.32)
    ref = oracle.block_spheres(th.astype(np.float64), B, 1.32)
    assert np.allclose(sp[:, :3], ref[:, :3], rtol=1e-6, atol=1e-4)
    assert (sp[:, 3] >= ref[:, 3]).all() and np.allclose(sp[:, 3], ref[:, 3], rtol=1e-5)
    K = sp.shape[0]
    words = (K + 31) // 32
    walk = synth.street_walk(city, 40, 32, z_far=300.0)
    for i in range(0, 40, 4):
        cams = walk[i:i + 4]
        got = P.bits_to_ids(P.cull_bits(sp, cams, words), K)
        vis = oracle.cull_blocks(sp.astype(np.float64), synth.cams_array(cams)).any(0)
        assert got.tolist() == np.nonzero(vis)[0].tolist()
        assert 0 < len(got) < K


def test_pose_features_definition():
    th, city = synth.city_scene(1000, 33, extent=1000.0)
    cams = synth.street_walk(city, 8, 34)
    f = P.pose_features(cams).reshape(8, 14)
    prev = None
    for i, c in enumerate(cams):
        assert np.allclose(f[i, :9], c.R.reshape(9), atol=1e-7)
        assert np.allclose(f[i, 9:12], c.t / P.T_SCALE, atol=1e-7)
        eye = -c.R.T @ c.t
        d = np.zeros(2) if prev is None else eye[:2] - prev[:2]
        assert np.allclose(f[i, 12:14], d, atol=1e-5)
        prev = eye


def test_street_walk_stays_on_streets_and_never_turns_back():
    _, city = synth.city_scene(1000, 35, extent=1000.0)
    cams = synth.street_walk(city, 3000, 36)
    eyes = np.array([-c.R.T @ c.t for c in cams])
    steps = np.diff(eyes[:, :2], axis=0)
    assert np.allclose(np.linalg.norm(steps, axis=1), 1.0, atol=1e-9)
    on_x = np.isclose(np.mod(eyes[:, 0] + 500.0, 100.0), 0.0, atol=1e-6) | \
        np.isclose(np.mod(eyes[:, 0] + 500.0, 100.0), 100.0, atol=1e-6)
    on_y = np.isclose(np.mod(eyes[:, 1] + 500.0, 100.0), 0.0, atol=1e-6) | \
        np.isclose(np.mod(eyes[:, 1] + 500.0, 100.0), 100.0, atol=1e-6)
    assert (on_x | on_y).all()
    assert (np.abs(eyes[:, :2]) <= 500.0 + 1e-9).all()
    assert ((steps[1:] * steps[:-1]).sum(1) > -0.5).all()       # no U-turns
    assert ((steps[1:] * steps[:-1]).sum(1) < 0.5).any()        # but turns happen


def test_log_pairs_alignment():
    th, city = synth.city_scene(20_000, 37, extent=1000.0)
    th = th[P.morton_order(th)]
    sp = P.block_spheres(th, 128)
    K = sp.shape[0]
    words = (K + 31) // 32
    walk = synth.street_walk(city, 4 * 12, 38, z_far=300.0)
    batches = [walk[4 * t:4 * t + 4] for t in range(12)]
    X, Y = P.log_pairs(sp, batches, words)
    assert X.shape == (12 - 5, 112) and Y.shape == (12 - 5, 4 * words)
    for t in range(X.shape[0]):
        assert np.array_equal(X[t], P.pose_features(batches[t] + batches[t + 1]))
        for h in range(4):
            assert np.array_equal(Y[t, h * words:(h + 1) * words], P.cull_bits(sp, batches[t + 1 + h + 1], words))


def test_bit_helpers():
    v = P.valid_mask(40, 2)
    assert v.shape == (8,) and v[0] == 0xFFFFFFFF and v[1] == 0xFF and v[2] == 0xFFFFFFFF and v[3] == 0xFF
    assert P.bits_to_ids(np.array([0b1011 | (1 << 31), 1 << 3], dtype=np.uint32), 40).tolist() == [0, 1, 3, 31, 35]
    assert P.bits_to_ids(np.array([0, 1 << 31], dtype=np.uint32), 40).tolist() == []
    r, p = P.recall_precision(np.array([0b0110], np.uint32), np.array([0b0011], np.uint32))
    assert (r, p) == (0.5, 0.5)
