"""50M Gaussians resident in HBM, street-level views (MI355X).

The scale case of the differentiation check: an aerial blob layout over
2 x 2 km (3200 blobs x 15625 Gaussians, sigma 5 m, heights U(0, 40) m; blobs
laid out in Morton order of their centres, rows of a blob contiguous),
street-level cameras at 1.7 m, 1600x900, horizontal fov 60 deg, z_far
1000 m, blocks of 65536 rows.

1. Full-frame rates: forward and backward Gaussian-pixel visits/s and the
   algorithmic HBM rate of the compositing kernels, for a batch of 4 poses.
2. FP32 gradient on a 256x256 crop (16-aligned origin (672, 320), principal
   point shifted) against the FP64 oracle.  The oracle runs on the rows of
   the blocks its own six-plane culling keeps (conservative, pinned on the
   CPU); every GPU-active row must lie in them.
3. The FP64 instance of the same kernels against central differences
   (eps 1e-6) on 64 sampled parameters of the crop, with a linear loss
   L = sum(W * image), W seeded.  The difference L(theta + eps) -
   L(theta - eps) is taken as sum(W * (image+ - image-)), so that only the
   pixels the step changes carry rounding (a difference of two sums over
   196 608 terms would leave a noise of about 1e-6 in the derivative); the
   tolerance is then 1e-4 |fd| + 1e-8.

Near ties: decision margins below 1/16 of their single-precision error
bound (one ulp), counted and held under 1 % of the pixels or rows compared.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_20150_amd import _lib as L
from paper_2605_20150_amd import synth
from paper_2605_20150_amd.raster import Pool, Rasterizer, dense_grad

pytestmark = pytest.mark.gpu
B = 65536
NEAR_TIE = 1.0 / 16
TIE_CEILING = 0.01


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def scene():
    centres = synth.blob_centres(3200, 1000.0, (0.0, 40.0), 20)
    order = oracle.morton_order(centres)
    return synth.blob_scene_parallel(3200, 15625, 1000.0, (0.0, 40.0), 5.0, 20, order=order)


def cameras():
    f = synth.focal_for_hfov(1600, 60)
    full = [synth.look_at((3.0 + i, 7.0, 1.7), (103.0 + i, 7.0, 1.7), (0, 0, 1), 1600, 900, f, z_far=1000.0)
            for i in range(4)]
    crop = synth.look_at((3.0, 7.0, 1.7), (103.0, 7.0, 1.7), (0, 0, 1), 256, 256, f, z_far=1000.0,
                         cx=800.0 - 672.0, cy=450.0 - 320.0)
    return full, crop


def test_street_50m_rates_crop_gradient_and_finite_differences():
    theta = scene()
    N = theta.shape[0]
    full, crop = cameras()
    say(f"case: {N} Gaussians in {(N + B - 1) // B} blocks; 4 street-level views 1600x900; crop 256x256")

    # ---- 1. full-frame rates (FP32)
    pool = Pool.from_dense(torch.from_numpy(theta).cuda(), B)
    rast = Rasterizer("cuda")
    lib = L.load()
    rng = np.random.Generator(np.random.PCG64(23))
    W4 = torch.from_numpy(rng.normal(size=(4, 3, 900, 1600)).astype(np.float32)).cuda()
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("render_fwd", "render_bwd")}
    import ctypes
    for k, (a, b) in ev.items():
        a.record()
        b.record()
        lib.tide_timer_arm(k.encode(), ctypes.c_void_p(a.cuda_event), ctypes.c_void_p(b.cuda_event))
    for _ in range(2):          # the second pass is the timed one (events keep the last launch)
        proj, bins, fr = rast.forward(pool, full)
        rast.backward(pool, full, proj, bins, fr, W4)
    torch.cuda.synchronize()
    lib.tide_timer_clear()
    ms = {k: a.elapsed_time(b) for k, (a, b) in ev.items()}
    fv = int(fr.visits_fwd.sum())
    bv = int(fr.visits_bwd.sum())
    assert bv == int(fr.last.sum(dtype=torch.int64))
    pixels = 4 * 900 * 1600
    say(f"visible pairs {bins.n_vis}, instances {bins.n_inst}; forward {ms['render_fwd']:.3f} ms, "
        f"{fv / ms['render_fwd'] / 1e9:.3f} T visits/s, "
        f"{(bins.n_inst * 56 + pixels * 20) / ms['render_fwd'] / 1e6:.1f} GB/s algorithmic; backward "
        f"{ms['render_bwd']:.3f} ms, {bv / ms['render_bwd'] / 1e9:.3f} T visits/s, "
        f"{(bins.n_inst * 92 + pixels * 20) / ms['render_bwd'] / 1e6:.1f} GB/s algorithmic")
    assert fv > 0 and bv > 0

    # ---- 2. FP32 crop gradient against the oracle on the kept blocks
    cm = synth.cams_array([crop])
    Wc = rng.normal(size=(1, 3, 256, 256))
    proj, bins, fr = rast.forward(pool, [crop])
    g = rast.backward(pool, [crop], proj, bins, fr, torch.from_numpy(Wc.astype(np.float32)).cuda())
    gd = dense_grad(proj, g, N)
    active = torch.nonzero(gd.abs().sum(1) > 0).squeeze(1).cpu().numpy()
    K = (N + B - 1) // B
    kap = oracle.kappa(cm)
    spheres = np.concatenate([oracle.block_spheres(theta[k * B:(k + 1) * B].astype(np.float64), B, kap)
                              for k in range(K)])
    kept = np.nonzero(oracle.cull_blocks(spheres, cm)[0])[0]
    rows = np.concatenate([np.arange(k * B, min(N, (k + 1) * B)) for k in kept])
    say(f"oracle on {len(kept)} kept blocks ({len(rows)} rows); GPU-active rows {len(active)}")
    assert np.isin(active, rows).all()
    sub = theta[rows].astype(np.float64)
    ref = oracle.render(sub, cm)
    g_ref = oracle.backward(sub, cm, Wc)
    g_gpu = gd[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    img_err = np.abs(fr.image.double().cpu().numpy() - ref["image"]).max(axis=1)
    tie_px = ref["pix_margin"] < NEAR_TIE
    say(f"crop image max-abs error {img_err[~tie_px].max():.3e} ({int(tie_px.sum())} near-tie pixels of "
        f"{tie_px.size}; all pixels {img_err.max():.3e})")
    assert tie_px.mean() <= TIE_CEILING
    assert img_err[~tie_px].max() <= 1e-4
    # a near-tie decision that flips moves a pixel by at most one entry's
    # contribution at the 1/255 alpha floor (or by T below 1e-4)
    assert img_err.max() <= 1e-2
    tie_rows = (ref["pair_margin"] < NEAR_TIE).any(axis=0)
    ok = ~tie_rows
    act_sub = np.isin(rows, active)
    say(f"active rows compared: {int((act_sub & ok).sum())} of {int(act_sub.sum())}")
    assert (act_sub & ~ok).sum() <= TIE_CEILING * act_sub.sum()
    rel = np.linalg.norm(g_gpu[ok] - g_ref[ok]) / np.linalg.norm(g_ref[ok])
    bound = 1e-3 * np.abs(g_ref[ok]) + 1e-4 * np.abs(g_ref[ok]).max()
    bad = int((np.abs(g_gpu[ok] - g_ref[ok]) > bound).sum())
    say(f"crop gradient: relative L2 error {rel:.3e}, {int(tie_rows.sum())} near-tie rows, {bad} entries over "
        f"the elementwise bound")
    assert rel <= 1e-3 and bad == 0
    del pool, gd, g, proj, bins, fr, rast
    torch.cuda.empty_cache()

    # ---- 3. FP64 instance against central differences
    pool = Pool.from_dense(torch.from_numpy(theta).cuda().double(), B)
    rast = Rasterizer("cuda")
    Wt = torch.from_numpy(Wc).cuda()

    def image_and_state():
        proj, bins, fr = rast.forward(pool, [crop])
        return fr.image.clone(), proj, bins, fr

    _, proj, bins, fr = image_and_state()
    g64 = rast.backward(pool, [crop], proj, bins, fr, Wt)
    gd = dense_grad(proj, g64, N)
    base_tt = proj.tiles_touched.clone()
    base_last = fr.last.clone()
    act = torch.nonzero(gd.abs().sum(1) > 0).squeeze(1).cpu().numpy()
    gsel = gd[torch.from_numpy(act).cuda()].cpu().numpy()
    del gd
    eps = 1e-6
    done = replaced = 0
    worst = 0.0
    while done < 64:
        a = int(rng.integers(0, len(act)))
        i, j = int(act[a]), int(rng.integers(0, 59))
        slot, r = i // B, i % B
        orig = pool.params[slot, j, r].item()
        imgs = []
        flip = False
        for d in (eps, -eps):
            pool.params[slot, j, r] = orig + d
            im, p2, _, f2 = image_and_state()
            flip = flip or not torch.equal(p2.tiles_touched, base_tt) or not torch.equal(f2.last, base_last)
            imgs.append(im)
        pool.params[slot, j, r] = orig
        if flip:
            replaced += 1
            continue
        fd = float((Wt * (imgs[0] - imgs[1])).sum()) / (2 * eps)
        err = abs(gsel[a, j] - fd)
        worst = max(worst, err / (abs(fd) + 1e-12))
        assert err <= 1e-4 * abs(fd) + 1e-8, (i, j, gsel[a, j], fd)
        done += 1
    say(f"64 FP64 samples within 1e-4 |fd| + 1e-8 (largest relative error {worst:.2e}); "
        f"{replaced} replaced for a decision flip")
