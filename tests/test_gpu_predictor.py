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
        p0, m0, v0 = oracle.mlp_adam(p0, g.astype(np.float64), m0, v0, t, 1e-3, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    assert mlp.step == 3
    p = mlp.params.cpu().numpy().astype(np.float64)
    m = mlp.exp_avg.cpu().numpy().astype(np.float64)
    v = mlp.exp_avg_sq.cpu().numpy().astype(np.float64)
    assert np.abs(m - m0).max() <= 1e-6 * np.abs(m0).max()
    assert np.abs(v - v0).max() <= 1e-6 * np.abs(v0).max()
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
