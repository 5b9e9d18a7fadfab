"""Learned block-visibility prefetch predictor (an addition to the paper's
method; exact Level-1 culling of Sec. 3.3 stays the fallback and the judge).

A ReLU MLP maps the last 8 camera poses (the current batch and the next,
which Alg. 1 already knows) to per-block visibility logits for the 4
batches after that.  Blocks it predicts are read from the SSD into the host
cache early (tide_prefetch_hint), so that Alg. 1's host-to-device transfers
find them there.  Nothing rendered depends on it: a missed block is streamed
by Alg. 1 as before.

Everything here is argument marshalling over libtide.so: pose features,
culling bitsets, the MLP's forward, backward, loss and Adam, and the
threshold all run in the library.  Training data are (pose history, exact
future block sets) pairs logged from dry-run walks with the exact culler.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L

HISTORY_POSES = 8       # two batches of 4 poses
HORIZON = 4             # predicts the block sets of batches t+2 .. t+5
POSE_DIM = 14           # [R | t / T_SCALE] (12) + ground-plane displacement (2)
T_SCALE = 2000.0
DEFAULT_DIMS = (HISTORY_POSES * POSE_DIM, 512, 512, 512, 512, HORIZON * 16384)


# ---------------------------------------------------------------- host helpers

def pose_features(cams) -> np.ndarray:
    """f32 [len(cams) * 14] features of consecutive poses (oldest first)."""
    lib = L.load()
    arr = L.camera_array(cams)
    out = np.zeros(len(cams) * POSE_DIM, dtype=np.float32)
    L.check(lib.tide_pose_features(arr, len(cams), T_SCALE, out.ctypes.data_as(C.POINTER(C.c_float))))
    return out


def cull_bits(spheres: np.ndarray, cams, n_words: int) -> np.ndarray:
    """Union over cams of the Level-1 block sets, as u32 [n_words] bits."""
    lib = L.load()
    sp = np.ascontiguousarray(spheres, dtype=np.float32)
    out = np.zeros(n_words, dtype=np.uint32)
    L.check(lib.tide_cull_bits(sp.ctypes.data_as(C.POINTER(C.c_float)), sp.shape[0], L.camera_array(cams), len(cams),
                               out.ctypes.data_as(C.POINTER(C.c_uint32)), n_words))
    return out


def morton_order(theta: np.ndarray) -> np.ndarray:
    """Layout order of the rows of a [N][59] (or [N][>=3]) table."""
    lib = L.load()
    th = np.ascontiguousarray(theta, dtype=np.float32)
    perm = np.zeros(th.shape[0], dtype=np.int64)
    L.check(lib.tide_morton_order(th.ctypes.data_as(C.POINTER(C.c_float)), th.shape[0], th.shape[1],
                                  perm.ctypes.data_as(C.POINTER(C.c_int64))))
    return perm


def block_spheres(theta_sorted: np.ndarray, B: int, kappa: float = 1.32) -> np.ndarray:
    """Spheres of the blocks of B consecutive rows (f32 [K][4]), as the store
    computes them at layout time."""
    lib = L.load()
    N = theta_sorted.shape[0]
    K = (N + B - 1) // B
    out = np.zeros((K, 4), dtype=np.float32)
    for k in range(K):
        rows = theta_sorted[k * B:(k + 1) * B, :6]
        cols = np.ascontiguousarray(rows.T, dtype=np.float32)
        L.check(lib.tide_block_sphere(cols.ctypes.data_as(C.POINTER(C.c_float)), cols.shape[1], cols.shape[1],
                                      kappa, out[k].ctypes.data_as(C.POINTER(C.c_float))))
    return out


def bits_to_ids(words: np.ndarray, n_blocks: int) -> np.ndarray:
    b = np.unpackbits(np.ascontiguousarray(words, dtype=np.uint32).view(np.uint8), bitorder="little")
    return np.nonzero(b[:n_blocks])[0].astype(np.int32)


# ---------------------------------------------------------------- pair logging

def log_pairs(spheres: np.ndarray, batches, words_per_h: int):
    """Training pairs from one walk (a list of camera batches of 4 poses):
    for every t with t+5 in range, x = features of batches t and t+1, and
    y = the exact block sets of batches t+2 .. t+5 as HORIZON bitsets."""
    vis = [cull_bits(spheres, b, words_per_h) for b in batches]
    X, Y = [], []
    for t in range(len(batches) - (HORIZON + 1)):
        X.append(pose_features(list(batches[t]) + list(batches[t + 1])))
        Y.append(np.concatenate([vis[t + 1 + h] for h in range(1, HORIZON + 1)]))
    if not X:
        return np.zeros((0, HISTORY_POSES * POSE_DIM), np.float32), np.zeros((0, HORIZON * words_per_h), np.uint32)
    return np.stack(X), np.stack(Y)


# ---------------------------------------------------------------- the network

class MLP:
    """Device parameters, gradients and Adam moments of the predictor MLP
    (flat layout of the tide_mlp struct: per layer W [out][in] then b)."""

    def __init__(self, dims=DEFAULT_DIMS, device="cuda", seed: int = 0, out_bias: float = 0.0):
        self.lib = L.load()
        self.dims = [int(d) for d in dims]
        self.L = len(self.dims) - 1
        darr = (C.c_int32 * (L.TIDE_MLP_MAX_LAYERS + 1))(*(self.dims + [0] * (L.TIDE_MLP_MAX_LAYERS + 1 - len(self.dims))))
        self.P = int(self.lib.tide_mlp_param_count(darr, self.L))
        if self.P < 0:
            raise ValueError(f"bad MLP dims {self.dims}")
        self.device = device
        self.params = torch.zeros(self.P, dtype=torch.float32, device=device)
        self.params_bf16 = torch.zeros(self.P, dtype=torch.int16, device=device)
        self.grad = torch.zeros(self.P, dtype=torch.float32, device=device)
        self.exp_avg = torch.zeros(self.P, dtype=torch.float32, device=device)
        self.exp_avg_sq = torch.zeros(self.P, dtype=torch.float32, device=device)
        s = L.tide_mlp()
        s.n_layers = self.L
        s.dims = darr
        s.params, s.params_bf16 = self.params.data_ptr(), self.params_bf16.data_ptr()
        s.grad, s.exp_avg, s.exp_avg_sq = self.grad.data_ptr(), self.exp_avg.data_ptr(), self.exp_avg_sq.data_ptr()
        s.step = 0
        self.s = s
        self._ws = {}
        self.offsets = []
        off = 0
        for l in range(self.L):
            wo = off
            off += self.dims[l] * self.dims[l + 1]
            self.offsets.append((wo, off))
            off += self.dims[l + 1]
        # He initialisation (seeded on the host); the output bias starts at a
        # given logit (e.g. the base rate of visible blocks)
        rng = np.random.Generator(np.random.PCG64(seed))
        Ws, bs = [], []
        for l in range(self.L):
            fan_in = self.dims[l]
            std = math.sqrt(2.0 / fan_in) if l + 1 < self.L else math.sqrt(1.0 / fan_in)
            Ws.append(rng.normal(0.0, std, size=(self.dims[l + 1], fan_in)))
            bs.append(np.full(self.dims[l + 1], out_bias if l + 1 == self.L else 0.0))
        self.set_weights(Ws, bs)

    @property
    def step(self) -> int:
        return int(self.s.step)

    def stream(self):
        return C.c_void_p(torch.cuda.current_stream().cuda_stream) if self.device != "cpu" else None

    def set_weights(self, Ws, bs):
        flat = np.zeros(self.P, dtype=np.float32)
        for l, (wo, bo) in enumerate(self.offsets):
            flat[wo:bo] = np.asarray(Ws[l], dtype=np.float32).reshape(-1)
            flat[bo:bo + self.dims[l + 1]] = np.asarray(bs[l], dtype=np.float32)
        self.params.copy_(torch.from_numpy(flat))
        L.check(self.lib.tide_mlp_sync_bf16(C.byref(self.s), self.stream()))

    def weights(self, bf16: bool = False):
        """(Ws, bs) as float64 numpy; with bf16=True the weights the
        products use (the bf16 copy), biases always from the FP32 master."""
        p = self.params.cpu().numpy().astype(np.float64)
        if bf16:
            wb = (self.params_bf16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
        Ws, bs = [], []
        for l, (wo, bo) in enumerate(self.offsets):
            src = wb if bf16 else p
            Ws.append(np.asarray(src[wo:bo], dtype=np.float64).reshape(self.dims[l + 1], self.dims[l]))
            bs.append(p[bo:bo + self.dims[l + 1]].copy())
        return Ws, bs

    def split(self, flat: torch.Tensor):
        """Per-layer (W, b) views of a flat [P] tensor (e.g. the gradient)."""
        out = []
        for l, (wo, bo) in enumerate(self.offsets):
            out.append((flat[wo:bo].view(self.dims[l + 1], self.dims[l]), flat[bo:bo + self.dims[l + 1]]))
        return out

    def ws(self, batch: int) -> torch.Tensor:
        n = int(self.lib.tide_mlp_ws_bytes(C.byref(self.s), int(batch)))
        key = n
        if key not in self._ws:
            self._ws = {key: torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)}
        return self._ws[key]

    def forward(self, x: torch.Tensor, logits: torch.Tensor | None = None) -> torch.Tensor:
        x = x.contiguous()
        B = x.shape[0]
        if logits is None:
            logits = torch.empty((B, self.dims[-1]), dtype=torch.float32, device=self.device)
        ws = self.ws(B)
        L.check(self.lib.tide_mlp_fwd(C.byref(self.s), C.c_void_p(x.data_ptr()), B, C.c_void_p(logits.data_ptr()),
                                      C.c_void_p(ws.data_ptr()), ws.numel(), self.stream()))
        return logits

    def backward(self, x: torch.Tensor, logits: torch.Tensor, label_bits: torch.Tensor, valid_bits: torch.Tensor,
                 loss_out: torch.Tensor | None = None) -> torch.Tensor:
        """Mean BCE (device f64 scalar) and its gradient into self.grad.
        Must follow forward() on the same x."""
        B = x.shape[0]
        if loss_out is None:
            loss_out = torch.zeros((), dtype=torch.float64, device=self.device)
        ws = self.ws(B)
        L.check(self.lib.tide_mlp_bwd(C.byref(self.s), C.c_void_p(x.data_ptr()), C.c_void_p(logits.data_ptr()),
                                      C.c_void_p(label_bits.data_ptr()), C.c_void_p(valid_bits.data_ptr()), B,
                                      C.c_void_p(loss_out.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                                      self.stream()))
        return loss_out

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        L.check(self.lib.tide_mlp_adam(C.byref(self.s), lr, beta1, beta2, eps, self.stream()))

    def predict_bits(self, logits: torch.Tensor, threshold_logit: float) -> torch.Tensor:
        B, n = logits.shape
        out = torch.empty((B, n // 32), dtype=torch.int32, device=self.device)
        L.check(self.lib.tide_mlp_predict_bits(C.c_void_p(logits.data_ptr()), B, n, float(threshold_logit),
                                               C.c_void_p(out.data_ptr()), self.stream()))
        return out


def valid_mask(n_blocks: int, words_per_h: int) -> np.ndarray:
    """u32 [HORIZON * words_per_h]: the first n_blocks outputs of every horizon."""
    one = np.zeros(words_per_h * 32, dtype=np.uint8)
    one[:n_blocks] = 1
    w = np.packbits(one, bitorder="little").view(np.uint32)
    return np.tile(w, HORIZON)


def recall_precision(pred_bits: np.ndarray, true_bits: np.ndarray):
    """Block recall and precision over all rows (u32 bitsets of equal shape)."""
    p = np.unpackbits(np.ascontiguousarray(pred_bits, dtype=np.uint32).view(np.uint8))
    t = np.unpackbits(np.ascontiguousarray(true_bits, dtype=np.uint32).view(np.uint8))
    tp = int(np.count_nonzero(p & t))
    return tp / max(int(t.sum()), 1), tp / max(int(p.sum()), 1)


def train(mlp: MLP, X: np.ndarray, Y: np.ndarray, valid: np.ndarray, epochs: int = 20, batch: int = 256,
          lr: float = 1e-3, seed: int = 0, val_frac: float = 0.1, target_recall: float = 0.99):
    """Mini-batch Adam on the GPU kernels.  The last val_frac of the pairs
    (in walk order) is held out; the threshold is the largest logit that
    keeps target_recall of the held-out visible blocks.  Returns a dict with
    per-step losses, threshold_logit and held-out recall / precision."""
    dev = mlp.device
    n = X.shape[0]
    n_val = max(1, int(round(val_frac * n)))
    n_tr = n - n_val
    rng = np.random.Generator(np.random.PCG64(seed))
    vmask = torch.from_numpy(valid.view(np.int32)).to(dev)
    steps = epochs * ((n_tr + batch - 1) // batch)
    losses = torch.zeros(steps, dtype=torch.float64, device=dev)
    s = 0
    for _ in range(epochs):
        perm = rng.permutation(n_tr)
        Xe = torch.from_numpy(np.ascontiguousarray(X[perm])).to(dev)
        Ye = torch.from_numpy(np.ascontiguousarray(Y[perm]).view(np.int32)).to(dev)
        for i in range(0, n_tr, batch):
            x, y = Xe[i:i + batch], Ye[i:i + batch]
            z = mlp.forward(x)
            mlp.backward(x, z, y, vmask, losses[s])
            mlp.adam(lr)
            s += 1
    # threshold on the held-out pairs
    Xv = torch.from_numpy(np.ascontiguousarray(X[n_tr:])).to(dev)
    Zv = torch.cat([mlp.forward(Xv[i:i + batch]).clone() for i in range(0, n_val, batch)]).cpu().numpy()
    Yv = Y[n_tr:]
    pos = np.unpackbits(np.ascontiguousarray(Yv).view(np.uint8), bitorder="little").reshape(Zv.shape).astype(bool)
    pos &= np.unpackbits(valid.view(np.uint8), bitorder="little").astype(bool)[None, :]
    zpos = np.sort(Zv[pos])
    thr = float(zpos[int(math.floor((1.0 - target_recall) * len(zpos)))]) if len(zpos) else 0.0
    pred = mlp.predict_bits(torch.from_numpy(Zv).to(dev), thr).cpu().numpy().view(np.uint32)
    pred &= valid[None, :]
    rec, prec = recall_precision(pred, Yv)
    return dict(losses=losses.cpu().numpy(), threshold_logit=thr, val_recall=rec, val_precision=prec,
                n_train=n_tr, n_val=n_val)


class Predictor:
    """Online use: features of the last 8 poses -> logits -> threshold ->
    prefetch hints for the blocks predicted for the next HORIZON batches.

    The network runs on a stream of its own, so that it overlaps the
    iteration's rendering instead of waiting behind it: launch() enqueues
    it, hint() waits for that stream only and passes the predicted blocks
    to the tier, nearest horizon first."""

    def __init__(self, mlp: MLP, threshold_logit: float, n_blocks: int, words_per_h: int):
        self.mlp = mlp
        self.thr = float(threshold_logit)
        self.K = int(n_blocks)
        self.words = int(words_per_h)
        self.x = torch.empty((1, HISTORY_POSES * POSE_DIM), dtype=torch.float32, device=mlp.device)
        self.logits = torch.empty((1, mlp.dims[-1]), dtype=torch.float32, device=mlp.device)
        self.stream = torch.cuda.Stream(device=mlp.device)
        self.host_x = torch.empty((1, HISTORY_POSES * POSE_DIM), dtype=torch.float32).pin_memory()
        self.host_bits = torch.empty((1, mlp.dims[-1] // 32), dtype=torch.int32).pin_memory()
        self.done = torch.cuda.Event()
        self.hinted = 0

    def launch(self, history):
        self.host_x.copy_(torch.from_numpy(pose_features(history)).view(1, -1))
        with torch.cuda.stream(self.stream):
            self.x.copy_(self.host_x, non_blocking=True)
            self.mlp.forward(self.x, self.logits)
            bits = self.mlp.predict_bits(self.logits, self.thr)
            self.host_bits.copy_(bits, non_blocking=True)
            self.done.record(self.stream)

    def collect(self) -> list[np.ndarray]:
        """Block ids predicted for each of the next HORIZON batches."""
        self.done.synchronize()
        bits = self.host_bits.numpy().view(np.uint32)[0]
        return [bits_to_ids(bits[h * self.words:(h + 1) * self.words], self.K) for h in range(HORIZON)]

    def predict(self, history) -> list[np.ndarray]:
        self.launch(history)
        return self.collect()

    def hint(self, tier):
        pred = self.collect()
        seen = set()
        order = []
        for ids in pred:                 # nearest horizon first
            for k in ids.tolist():
                if k not in seen:
                    seen.add(k)
                    order.append(k)
        if order:
            tier.prefetch(order, horizon=2)
            self.hinted += len(order)
        return pred
