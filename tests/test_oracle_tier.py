"""Pins of the tier oracle (CPU): Level-1 conservativeness by brute force
against the exact rasterizer's culling, kappa closed forms, Alg. 1
hand-computed cases and set identities."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_20150_amd import synth


def random_cameras(rng, n, centre, spread, W=96, H=64):
    cams = []
    for _ in range(n):
        eye = centre + rng.normal(0, spread, size=3)
        target = centre + rng.normal(0, 0.6 * spread, size=3)
        if np.linalg.norm(target - eye) < 1e-3:
            continue
        up = rng.normal(size=3)
        f = rng.uniform(0.4, 1.5) * W
        cams.append(synth.look_at(eye, target, up, W, H, f, z_near=0.2, z_far=rng.uniform(0.5, 5.0)))
    return cams


def test_kappa_closed_forms():
    aerial = synth.cams_array(synth.orbit_cameras(4, 250.0, 150.0, (0, 0, 20)))
    lx, ly = 1.3 * 960 / synth.focal_for_hfov(1920, 60), 1.3 * 540 / synth.focal_for_hfov(1920, 60)
    assert abs(oracle.kappa(aerial) - math.sqrt(1 + lx * lx + ly * ly)) < 1e-14
    assert abs(oracle.kappa(aerial) - 1.3197) < 1e-4
    assert abs(oracle.kappa(synth.cams_array([synth.tiny_camera()])) - math.sqrt(1 + 2 * 0.65 ** 2)) < 1e-14


def test_sphere_contains_members():
    th = synth.dense_scene(1000, 31, logscale_mu=-3).astype(np.float64)
    sp = oracle.block_spheres(th, 100, 1.3)
    for k in range(10):
        mu = th[100 * k:100 * (k + 1), :3]
        c = mu.mean(0)
        assert np.allclose(sp[k, :3], c)
        d = np.linalg.norm(mu - c, axis=1) + 3 * 1.3 * np.exp(th[100 * k:100 * (k + 1), 3:6].max(1))
        assert abs(sp[k, 3] - d.max()) < 1e-12


def test_level1_culling_is_conservative_by_brute_force():
    """Every (Gaussian, camera) pair the exact rasterizer keeps lies in a
    block the six-plane sphere test keeps (recall 1.0) over 1200 random
    cameras, many of them grazing the scene."""
    rng = np.random.default_rng(32)
    th = synth.dense_scene(4000, 33, extent=2.0, logscale_mu=-2.4, logscale_sigma=0.7).astype(np.float64)
    # spatially coherent blocks: order rows by a coarse grid cell
    cell = np.floor((th[:, :3] + 2.0) / 0.5).astype(int)
    order = np.lexsort((cell[:, 2], cell[:, 1], cell[:, 0]))
    th = th[order]
    B = 32
    cams = random_cameras(rng, 1200, np.zeros(3), 2.5)
    cm = synth.cams_array(cams)
    kap = max(oracle.kappa(cm[i:i + 1]) for i in range(len(cams)))
    sp = oracle.block_spheres(th, B, kap)
    vis = oracle.cull_blocks(sp, cm)
    kept_pairs, culled_blocks = 0, 0
    for c0 in range(0, len(cams), 100):
        p = oracle.project(th, cm[c0:c0 + 100])
        keep = p["keep"]
        for c in range(keep.shape[0]):
            blocks = np.unique(np.where(keep[c])[0] // B)
            assert vis[c0 + c, blocks].all(), (c0 + c, blocks[~vis[c0 + c, blocks]])
            kept_pairs += int(keep[c].sum())
            culled_blocks += int((~vis[c0 + c]).sum())
    assert kept_pairs > 10000 and culled_blocks > 10000   # both sides of the test exercised


def test_culling_obvious_cases():
    cam = synth.cams_array([synth.tiny_camera()])          # at (0,0,-3) looking +z
    sp = np.array([[0, 0, 0, 0.1], [0, 0, -10, 0.1], [0, 0, 1e5, 0.1], [50, 0, 0, 0.1], [0, 0, -3.1, 0.5]])
    vis = oracle.cull_blocks(sp, cam)[0]
    assert vis.tolist() == [True, False, False, False, True]


def test_alg1_plain_score_order():
    # blocks 0..5; block 0 resident but idle, 1 and 2 resident and in use
    age = np.array([0, 0, 0, 9, 9, 9], dtype=float)
    Rn, sp, sm, ag, _ = oracle.alg1([0, 1, 2], [1, 2], [[2, 3], [3, 4]], age, 0.75, 0.9, 3)
    assert ag.tolist() == [1, 0, 0, 10, 10, 10]
    # scores: s0 = .25 .9, s1 = .25, s2 = 1, s3 = s4 = .75 + .25 .9^10 -> {2, 3, 4} (3 before 4 on the tie)
    assert Rn.tolist() == [2, 3, 4] and sp == [3, 4] and sm == [0, 1]


def test_alg1_camera_quota_covers_every_view():
    age = np.full(30, 50.0)
    age[:8] = 0
    R = list(range(8))
    # camera 1 sees 8 hot blocks, camera 2 one cold block; C = 8, J = 2 -> quota 1
    Rn, sp, sm, _, rank = oracle.alg1(R, R, [list(range(8)), [20]], age, 0.75, 0.9, 8)
    assert 20 in Rn.tolist() and len(Rn) == 8
    assert rank.tolist()[:2] == [0, 20]
    assert sp == [20] and sm == [7]


def test_alg1_identities_random():
    rng = np.random.default_rng(34)
    nb = 60
    age = np.full(nb, 30.0)
    R = sorted(rng.choice(nb, 12, replace=False).tolist())
    for _ in range(200):
        C = int(rng.integers(4, 30))
        J = int(rng.integers(1, 5))
        Kc = rng.choice(nb, int(rng.integers(0, 15)), replace=False).tolist()
        Kn = [rng.choice(nb, int(rng.integers(0, 10)), replace=False).tolist() for _ in range(J)]
        Rn, sp, sm, age, _ = oracle.alg1(R, Kc, Kn, age, 0.75, 0.9, C)
        Ct = set(R) | set(x for k in Kn for x in k)
        sR, sN = set(R), set(Rn.tolist())
        assert sN <= Ct
        assert len(sN) == min(C, len(Ct))
        assert not (set(sp) & sR) and not (set(sm) & sN)
        assert (sR - set(sm)) | set(sp) == sN
        Kunion = set(x for k in Kn for x in k)
        if C >= len(Kunion):
            assert Kunion <= sN
        R = Rn.tolist()


def test_morton_order_closed_forms():
    # the corners of a box sort along the Z curve: x is the lowest bit, then y, then z
    corners = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=np.float64) * [4, 2, 7]
    shuffle = np.random.default_rng(3).permutation(8)
    perm = oracle.morton_order(corners[shuffle])
    assert np.array_equal(corners[shuffle][perm], corners)
    # points on one axis line sort by that coordinate (a plain stable sort)
    rng = np.random.default_rng(4)
    x = rng.uniform(-5, 5, size=500)
    line = np.stack([x, np.full(500, 2.0), np.full(500, -1.0)], 1)
    assert np.array_equal(oracle.morton_order(line), np.argsort(x, kind="stable"))
    # equal centres keep their row order
    dup = np.repeat(rng.uniform(size=(10, 3)), 5, axis=0)[rng.permutation(50)]
    perm = oracle.morton_order(dup)
    for i in range(49):
        if np.array_equal(dup[perm[i]], dup[perm[i + 1]]):
            assert perm[i] < perm[i + 1]
    # the order is a permutation and is invariant under a positive affine map of the centres
    pts = rng.normal(size=(300, 3))
    p1 = oracle.morton_order(pts)
    assert sorted(p1.tolist()) == list(range(300))
    # x-major 2^k grid: the cells of a 4x4x1 grid interleave as a 2-D Z curve
    g = np.array([[i, j, 0.0] for j in range(4) for i in range(4)]) / 3.0 * (1 - 1e-12)
    order = oracle.morton_order(g)
    ij = [(int(round(g[o, 0] * 3)), int(round(g[o, 1] * 3))) for o in order]
    assert ij[:4] == [(0, 0), (1, 0), (0, 1), (1, 1)] and ij[4:8] == [(2, 0), (3, 0), (2, 1), (3, 1)]
