"""Pins of the predictor-MLP oracle (CPU): bfloat16 rounding against its
definition, the forward against numpy's matmul chain, BCE at zero logits,
gradients against central differences, and convergence on a separable toy
problem."""
import math

import numpy as np

import oracle


def bf16_reference(x):
    """Nearest bfloat16 (ties to even) by comparing the two neighbours."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32)
    lo = (u & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    hi = ((u & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    d_lo, d_hi = np.abs(f.astype(np.float64) - lo), np.abs(hi - f.astype(np.float64))
    lo_even = ((u >> np.uint32(16)) & np.uint32(1)) == 0
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & ~lo_even)
    return np.where(pick_hi, hi, lo)


def test_bf16_rounding_definition():
    rng = np.random.default_rng(60)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 1000), rng.normal(0, 1e4, 1000),
                        [1.0, 1.00390625, 1.01171875, -2.0078125, 0.0, 65504.0]]).astype(np.float32)
    assert np.array_equal(oracle.bf16_round(x.astype(np.float64)), bf16_reference(x))


def mlp(rng, dims, scale=0.5):
    Ws = [rng.normal(0, scale / math.sqrt(dims[i]), size=(dims[i + 1], dims[i])) for i in range(len(dims) - 1)]
    bs = [rng.normal(0, 0.1, size=dims[i + 1]) for i in range(len(dims) - 1)]
    return Ws, bs


def test_forward_matches_matmul_chain():
    rng = np.random.default_rng(61)
    dims = [14, 32, 32, 10]
    Ws, bs = mlp(rng, dims)
    x = rng.normal(size=(7, 14))
    a = x
    for l, (W, b) in enumerate(zip(Ws, bs)):
        a = a @ W.T + b
        if l < len(Ws) - 1:
            a = np.maximum(a, 0)
    assert np.abs(oracle.mlp_forward(x, Ws, bs) - a).max() < 1e-12


def test_bce_at_zero_logits_is_ln2():
    dims = [6, 5, 4]
    Ws = [np.zeros((dims[i + 1], dims[i])) for i in range(2)]
    bs = [np.zeros(dims[i + 1]) for i in range(2)]
    rng = np.random.default_rng(62)
    lab = rng.integers(0, 2, size=(3, 4))
    L, dW, db = oracle.mlp_loss_backward(rng.normal(size=(3, 6)), Ws, bs, lab, np.ones(4))
    assert abs(L - math.log(2)) < 1e-15
    # the output bias gradient at z = 0 is mean(0.5 - y)
    assert np.allclose(db[1], (0.5 - lab).sum(0) / 12)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(63)
    dims = [8, 12, 12, 6]
    Ws, bs = mlp(rng, dims, 1.0)
    x = rng.normal(size=(5, 8))
    lab = rng.integers(0, 2, size=(5, 6))
    valid = np.array([1, 1, 0, 1, 1, 0])
    L0, dW, db = oracle.mlp_loss_backward(x, Ws, bs, lab, valid)
    eps = 1e-6
    for l in range(3):
        for _ in range(8):
            i, j = rng.integers(0, Ws[l].shape[0]), rng.integers(0, Ws[l].shape[1])
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += eps
            Wm[l][i, j] -= eps
            fd = (oracle.mlp_loss_backward(x, Wp, bs, lab, valid)[0] -
                  oracle.mlp_loss_backward(x, Wm, bs, lab, valid)[0]) / (2 * eps)
            assert abs(fd - dW[l][i, j]) < 1e-7 * max(1, abs(fd)) + 1e-10
        i = rng.integers(0, bs[l].shape[0])
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][i] += eps
        bm[l][i] -= eps
        fd = (oracle.mlp_loss_backward(x, Ws, bp, lab, valid)[0] -
              oracle.mlp_loss_backward(x, Ws, bm, lab, valid)[0]) / (2 * eps)
        assert abs(fd - db[l][i]) < 1e-7 * max(1, abs(fd)) + 1e-10
    # invalid outputs do not feed the gradient
    lab2 = lab.copy()
    lab2[:, 2] = 1 - lab2[:, 2]
    assert oracle.mlp_loss_backward(x, Ws, bs, lab2, valid)[0] == L0


def test_separable_toy_problem_converges():
    rng = np.random.default_rng(64)
    dims = [4, 16, 3]
    Ws, bs = mlp(rng, dims, 1.0)
    x = rng.normal(size=(64, 4))
    A = rng.normal(size=(4, 3))
    lab = (x @ A > 0).astype(np.uint8)
    m = [np.zeros_like(p) for p in Ws + bs]
    v = [np.zeros_like(p) for p in Ws + bs]
    first = None
    for t in range(1, 401):
        L, dW, db = oracle.mlp_loss_backward(x, Ws, bs, lab, np.ones(3))
        first = L if first is None else first
        params, grads = Ws + bs, dW + db
        for k, (p, g) in enumerate(zip(params, grads)):
            m[k] = 0.9 * m[k] + 0.1 * g
            v[k] = 0.999 * v[k] + 0.001 * g * g
            p -= 1e-2 * (m[k] / (1 - 0.9 ** t)) / (np.sqrt(v[k] / (1 - 0.999 ** t)) + 1e-8)
    assert first > 0.5 and L < 0.1


def test_adam_closed_forms():
    rng = np.random.default_rng(65)
    g = rng.normal(size=200)
    p0 = rng.normal(size=200)
    # first step: m_hat = g, v_hat = g^2, so the move is lr g / (|g| + eps)
    p1, m, v = oracle.mlp_adam(p0, g, np.zeros(200), np.zeros(200), 1, 1e-3, eps=1e-8)
    assert np.allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    p = p1
    for t in range(2, 30):
        p_prev = p
        p, m, v = oracle.mlp_adam(p, g, m, v, t, 1e-3, eps=0.0)
        assert np.allclose(p_prev - p, 1e-3 * np.sign(g), rtol=1e-9, atol=1e-15)
    # zero gradient from a zero state leaves everything at zero
    z = oracle.mlp_adam(p0, np.zeros(200), np.zeros(200), np.zeros(200), 1, 1e-3)
    assert np.array_equal(z[0], p0) and not z[1].any() and not z[2].any()
