"""Predictor MLP kernels on MI355X against the FP64 oracle, and the trained
predictor against exact Level-1 culling.

Error budget of a GPU product (derivation for the tolerances below): the
weights are the same bf16 values on both sides; an FP32 activation a is
split into hi + lo with |a - hi - lo| <= 2^-17 |a|; products are exact in
FP32 and accumulate in FP32 over K <= 512 terms, K 2^-24 <= 3.1e-5.  So a
layer's output differs by at most ~3.8e-5 * sum |w| |a| from the exact
value, and five layers by at most ~1.9e-4 * S, where S is the same network
evaluated with |W|, |b| and |x| (an upper bound of every sum |w||a|)."""
import ctypes as C
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_20150_amd import _lib as L
from paper_2605_20150_amd import predictor as P
from paper_2605_20150_amd import synth

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def seeded_net(dims, seed, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    Ws = [rng.normal(0, scale * math.sqrt(2.0 / dims[l]), size=(dims[l + 1], dims[l])).astype(np.float32)
          for l in range(len(dims) - 1)]
    bs = [rng.normal(0, 0.1, size=dims[l + 1]).astype(np.float32) for l in range(len(dims) - 1)]
    return Ws, bs


def oracle_weights(Ws):
    return [oracle.bf16_round(w.astype(np.float64)) for w in Ws]


def magnitude(x, Wr, bs):
    return oracle.mlp_forward(np.abs(x), [np.abs(w) for w in Wr], [np.abs(b.astype(np.float64)) for b in bs])


def bf16_rne(x32):
    """Nearest bfloat16 of FP32 values (ties to even), as float64."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def make(dims, seed, batch, device="cuda"):
    mlp = P.MLP(dims, device=device, seed=0)
    Ws, bs = seeded_net(dims, seed)
    mlp.set_weights(Ws, bs)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    x = rng.normal(0, 1, size=(batch, dims[0])).astype(np.float32)
    return mlp, Ws, bs, x


def test_bf16_copy_is_round_to_nearest_even():
    dims = [16, 64, 32]
    mlp = P.MLP(dims, seed=1)
    rng = np.random.Generator(np.random.PCG64(70))
    vals = np.concatenate([rng.normal(0, 1, mlp.P - 6), [1.00390625, 1.01171875, -2.0078125, 0.0, 3e-39, -1e30]])
    flat = vals.astype(np.float32)
    mlp.params.copy_(torch.from_numpy(flat))
    L.check(L.load().tide_mlp_sync_bf16(C.byref(mlp.s), None))
    torch.cuda.synchronize()
    got = (mlp.params_bf16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(got.astype(np.float64), oracle.bf16_round(flat.astype(np.float64)))


@pytest.mark.parametrize("batch", [1, 100])
def test_forward_matches_oracle(batch):
    dims = [112, 200, 512, 136, 1056]      # ragged against the 64 x 64 tiles and the 32-deep K steps
    mlp, Ws, bs, x = make(dims, 71, batch)
    say(f"case: forward dims {dims} batch {batch}")
    z = mlp.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    Wr = oracle_weights(Ws)
    ref = oracle.mlp_forward(x.astype(np.float64), Wr, [b.astype(np.float64) for b in bs])
    S = magnitude(x.astype(np.float64), Wr, bs)
    err = np.abs(z - ref)
    say(f"max |dz| = {err.max():.3e}, max |dz|/S = {(err / S).max():.3e}")
    assert (err <= 1.9e-4 * S + 1e-30).all()


def test_full_size_forward_on_sampled_rows():
    dims = list(P.DEFAULT_DIMS)
    mlp, Ws, bs, x = make(dims, 72, 256)
    say(f"case: full-size forward dims {dims} batch 256")
    z = mlp.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    z1 = mlp.forward(torch.from_numpy(x[200:201]).cuda()).cpu().numpy().astype(np.float64)
    Wr = oracle_weights(Ws)
    b64 = [b.astype(np.float64) for b in bs]
    rows = [0, 63, 64, 200, 255]
    ref = oracle.mlp_forward(x[rows].astype(np.float64), Wr, b64)
    S = magnitude(x[rows].astype(np.float64), Wr, bs)
    err = np.abs(z[rows] - ref)
    say(f"max |dz| = {err.max():.3e}, max |dz|/S = {(err / S).max():.3e}")
    assert (err <= 1.9e-4 * S).all()
    # the batch-1 inference shape gives the same logits for that row
    assert (np.abs(z1[0] - ref[3]) <= 1.9e-4 * S[3]).all()


def test_backward_matches_oracle():
    dims = [112, 200, 512, 136, 1056]
    batch = 100
    mlp, Ws, bs, x = make(dims, 73, batch)
    rng = np.random.Generator(np.random.PCG64(74))
    lab = (rng.uniform(size=(batch, dims[-1])) < 0.1).astype(np.uint8)
    valid = np.ones(dims[-1], dtype=np.uint8)
    valid[-40:] = 0
    say(f"case: backward dims {dims} batch {batch}")
    xd = torch.from_numpy(x).cuda()
    z = mlp.forward(xd)
    lbits = torch.from_numpy(np.packbits(lab, axis=1, bitorder="little").view(np.int32).copy()).cuda()
    vbits = torch.from_numpy(np.packbits(valid, bitorder="little").view(np.int32).copy()).cuda()
    loss = float(mlp.backward(xd, z, lbits, vbits).item())
    Wr = oracle_weights(Ws)
    L_ref, dW, db = oracle.mlp_loss_backward(x.astype(np.float64), Wr, [b.astype(np.float64) for b in bs], lab, valid)
    say(f"loss gpu {loss!r} oracle {L_ref!r}")
    assert abs(loss - L_ref) <= 1e-6 * abs(L_ref)
    g = mlp.split(mlp.grad)
    for l in range(len(Ws)):
        gw, gb = g[l][0].cpu().numpy().astype(np.float64), g[l][1].cpu().numpy().astype(np.float64)
        for name, a, b in (("W", gw, dW[l]), ("b", gb, db[l])):
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            mx = np.abs(a - b).max() / np.abs(b).max()
            say(f"layer {l} d{name}: norm-rel {rel:.2e}, max-rel {mx:.2e}")
            assert rel <= 1e-4 and mx <= 1e-3


def test_adam_matches_oracle():
    dims = [112, 200, 512, 136, 1056]
    mlp = P.MLP(dims, seed=5)
    rng = np.random.Generator(np.random.PCG64(75))
    flat = rng.normal(0, 0.1, mlp.P).astype(np.float32)
    mlp.params.copy_(torch.from_numpy(flat))
    p0 = flat.astype(np.float64)
    m0 = np.zeros(mlp.P)
    v0 = np.zeros(mlp.P)
    for t in range(1, 4):
        g = (rng.normal(0, 1e-2, mlp.P) * (rng.uniform(size=mlp.P) < 0.9)).astype(np.float32)
        mlp.grad.copy_(torch.from_numpy(g))
        mlp.adam(1e-3, 0.9, 0.999, 1e-8)
        # the call takes single-precision hyperparameters: the oracle gets the same values
        f = [float(np.float32(c)) for c in (1e-3, 0.9, 0.999, 1e-8)]
        p0, m0, v0 = oracle.mlp_adam(p0, g.astype(np.float64), m0, v0, t, *f)
    torch.cuda.synchronize()
    assert mlp.step == 3
    p = mlp.params.cpu().numpy().astype(np.float64)
    m = mlp.exp_avg.cpu().numpy().astype(np.float64)
    v = mlp.exp_avg_sq.cpu().numpy().astype(np.float64)
    assert np.abs(m - m0).max() <= 2e-6 * np.abs(m0).max()
    assert np.abs(v - v0).max() <= 2e-6 * np.abs(v0).max()
    assert np.abs(p - p0).max() <= 1e-6
    # the bf16 copy is the rounding of the new FP32 master
    wb = (mlp.params_bf16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(wb.astype(np.float64), bf16_rne(mlp.params.cpu().numpy()))


def test_threshold_bits():
    rng = np.random.Generator(np.random.PCG64(76))
    z = rng.normal(0, 2, size=(5, 256)).astype(np.float32)
    z[0, :8] = 0.25                      # exactly at the threshold: predicted visible
    mlp = P.MLP([16, 32], seed=0)
    bits = mlp.predict_bits(torch.from_numpy(z).cuda(), 0.25).cpu().numpy().view(np.uint32)
    ref = np.packbits((z >= np.float32(0.25)).astype(np.uint8), axis=1, bitorder="little").view(np.uint32)
    assert np.array_equal(bits, ref)


def test_trained_predictor_recall_precision_and_stall_gain():
    """Dry-run pairs from street walks over a synthetic city, training on the
    GPU kernels, then a held-out walk: recall / precision against exact
    culling, and the simulated-clock stall with and without its hints."""
    sys.path.insert(0, __import__("os").path.dirname(__file__))
    from tier_clock import ClockConfig, dry_city, simulate, walk_sets
    sp, city = dry_city(90, 1000.0)
    K = sp.shape[0]
    words = (K + 31) // 32
    z_far = 300.0
    say(f"case: city {K} blocks, z_far {z_far}")
    Xs, Ys = [], []
    for seed in range(100, 116):
        batches, _ = walk_sets(sp, city, seed, 400, z_far)
        X, Y = P.log_pairs(sp, batches, words)
        Xs.append(X)
        Ys.append(Y)
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    valid = P.valid_mask(K, words)
    base = np.unpackbits(Y.view(np.uint8)).sum() / (Y.shape[0] * P.HORIZON * K)
    mlp = P.MLP([112, 512, 512, 512, 512, P.HORIZON * words * 32], seed=3,
                out_bias=math.log(base / (1 - base)))
    out = P.train(mlp, X, Y, valid, epochs=20, batch=256, lr=1e-3, seed=4)
    l = out["losses"]
    say(f"pairs {X.shape[0]}, base rate {base:.4f}, loss {l[:10].mean():.4f} -> {l[-10:].mean():.4f}, "
        f"val recall {out['val_recall']:.4f} precision {out['val_precision']:.4f} thr {out['threshold_logit']:.3f}")
    assert l[-10:].mean() < 0.7 * l[:10].mean()
    # held-out walk
    batches, sets = walk_sets(sp, city, 34, 300, z_far)
    Xt, Yt = P.log_pairs(sp, batches, words)
    z = torch.cat([mlp.forward(torch.from_numpy(Xt[i:i + 256]).cuda()).clone() for i in range(0, Xt.shape[0], 256)])
    bits = mlp.predict_bits(z, out["threshold_logit"]).cpu().numpy().view(np.uint32) & valid[None, :]
    rec, prec = P.recall_precision(bits, Yt)
    say(f"held-out recall {rec:.4f} precision {prec:.4f}")
    assert rec >= 0.9 and prec >= 2 * base
    hints = [None] * len(sets)
    for t in range(Xt.shape[0]):
        hints[t] = sorted(set(int(k) for h in range(P.HORIZON)
                              for k in P.bits_to_ids(bits[t, h * words:(h + 1) * words], K)))
    sizes = [len(set(k for s in b for k in s)) for b in sets]
    cfg = ClockConfig(capacity=2 * max(sizes) + 8, host_blocks=4 * max(sizes), ssd_ms=8.0, h2d_ms=1.0, c0_ms=40.0,
                      c1_ms=0.0)
    exact = simulate(sets, cfg)
    pred = simulate(sets, cfg, hints=hints)
    say(f"|K_t| {min(sizes)}..{max(sizes)}; stall exact-only {exact.total_stall_ms:.1f} ms, with predictor "
        f"{pred.total_stall_ms:.1f} ms; prefetch reads {pred.prefetch_reads}, used {pred.prefetch_used}")
    assert pred.render_sets == exact.render_sets
    assert pred.total_stall_ms < exact.total_stall_ms


def test_city_walk_predictor_against_exact_streaming_simulated():
    """The 1B-Gaussian street-city protocol on the simulated clock: 15 259
    blocks over 4 x 4 km (block spheres from a 64-Gaussian sample per block),
    z_far 1000 m (|K_t| in the hundreds to ~1500 blocks), capacity 4000 and a
    1379-block host cache; the full-size predictor (4 x 512 hidden, 4 x 16384
    outputs) trained on 20 dry-run walks of 1000 iterations, judged on the
    held-out walk (seed 34).  Timing from this machine's measured rates:
    46.7 MB blocks at 2.2 GB/s from the SSD (21 ms) and ~40 GB/s to the GPU
    (1.2 ms), compute 5 ms + 0.24 ms per resident block."""
    sys.path.insert(0, __import__("os").path.dirname(__file__))
    from tier_clock import ClockConfig, dry_city, simulate, walk_sets
    sp, city = dry_city(30, 4000.0)
    K = sp.shape[0]
    words = P.DEFAULT_DIMS[-1] // (32 * P.HORIZON)
    z_far = 1000.0
    say(f"case: city {K} blocks, z_far {z_far}")

    def pairs(seed):
        cams = synth.street_walk(city, 4000, seed, z_far=z_far)
        return P.log_pairs(sp, [cams[4 * t:4 * t + 4] for t in range(1000)], words)
    res = [pairs(seed) for seed in range(100, 120)]
    X = np.concatenate([r[0] for r in res])
    Y = np.concatenate([r[1] for r in res])
    say(f"logged {X.shape[0]} pairs")
    valid = P.valid_mask(K, words)
    base = float(np.unpackbits(Y.view(np.uint8)).sum()) / (Y.shape[0] * P.HORIZON * K)
    mlp = P.MLP(P.DEFAULT_DIMS, seed=3, out_bias=math.log(base / (1 - base)))
    out = P.train(mlp, X, Y, valid, epochs=20, batch=256, lr=1e-3, seed=4)
    say(f"pairs {X.shape[0]}, base {base:.4f}, loss {out['losses'][:10].mean():.4f} -> "
        f"{out['losses'][-10:].mean():.4f}, val recall {out['val_recall']:.4f} precision {out['val_precision']:.4f}")
    batches, sets = walk_sets(sp, city, 34, 1000, z_far)
    Xt, Yt = P.log_pairs(sp, batches, words)
    z = torch.cat([mlp.forward(torch.from_numpy(Xt[i:i + 256]).cuda()).clone() for i in range(0, Xt.shape[0], 256)])
    bits = mlp.predict_bits(z, out["threshold_logit"]).cpu().numpy().view(np.uint32) & valid[None, :]
    rec, prec = P.recall_precision(bits, Yt)
    hints = [None] * len(sets)
    for t in range(Xt.shape[0]):
        seen, order = set(), []
        for h in range(P.HORIZON):
            for k in P.bits_to_ids(bits[t, h * words:(h + 1) * words], K).tolist():
                if k not in seen:
                    seen.add(k)
                    order.append(k)
        hints[t] = order
    future = [sorted(set(k for h in range(2, 6) if t + h < len(sets) for s in sets[t + h] for k in s))
              for t in range(len(sets))]
    sizes = [len(set(k for s in b for k in s)) for b in sets]
    cfg = ClockConfig(capacity=4000, host_blocks=1379, ssd_ms=21.0, h2d_ms=1.2, c0_ms=5.0, c1_ms=0.24, spec_cap=16)
    exact = simulate(sets, cfg)
    say(f"simulated exact-only: {exact.total_stall_ms:.0f} ms")
    pred = simulate(sets, cfg, hints=hints)
    say(f"simulated with the predictor: {pred.total_stall_ms:.0f} ms")
    best = simulate(sets, cfg, hints=future)
    T = len(sets)
    say(f"walk: {T} iterations, |K_t| {min(sizes)}..{max(sizes)} (mean {np.mean(sizes):.0f}); held-out recall "
        f"{rec:.4f} precision {prec:.4f}")
    say(f"stall s/iter: exact-only {exact.total_stall_ms / T / 1e3:.4f}, predictor {pred.total_stall_ms / T / 1e3:.4f} "
        f"(prefetch reads {pred.prefetch_reads}, used {pred.prefetch_used}); hints = the exact sets of "
        f"t+2..t+5: {best.total_stall_ms / T / 1e3:.4f}")
    assert rec >= 0.95
    assert pred.render_sets == exact.render_sets
    assert pred.total_stall_ms <= exact.total_stall_ms
