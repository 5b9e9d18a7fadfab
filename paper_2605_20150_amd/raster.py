"""Torch-facing driver of the rasterizer hot path.

PyTorch only provides device memory and the stream; each step is one call
into libtide.so (preprocess -> bin/sort -> composite -> loss -> adjoint ->
masked Adam).  ``TideRasterize`` wraps forward and the hand-written adjoint
as a ``torch.autograd.Function`` over a dense (N, 59) table for tests and
gradient checks; the training loop calls the C ABI directly with compact
gradients.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

D = 59
TILE = 16


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float32:
        return L.TIDE_F32
    if dt == torch.float64:
        return L.TIDE_F64
    raise TypeError(f"unsupported dtype {dt}")


class Buffers:
    """Device byte buffers that grow on demand (reused across iterations)."""

    def __init__(self, device):
        self.device = device
        self.bufs: dict[str, torch.Tensor] = {}

    def get(self, name: str, nbytes: int) -> torch.Tensor:
        b = self.bufs.get(name)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
            self.bufs[name] = b
        return b


def _dptr(t: torch.Tensor) -> int:
    """Device address of t's first element.  An empty view of an allocated
    buffer (n_pidx = 0: nothing in the render order) reports 0 from
    data_ptr(); the library still wants a valid address, so take the
    buffer's."""
    p = t.data_ptr()
    if p == 0 and t.numel() == 0:
        p = t.untyped_storage().data_ptr() + t.storage_offset() * t.element_size()
    return p


class Pool:
    """Resident parameter pool, block-SoA [n_slots][59][block_rows]."""

    def __init__(self, params, exp_avg, exp_avg_sq, step, slot_block, slot_rows, order, n_order=None):
        self.params, self.exp_avg, self.exp_avg_sq, self.step = params, exp_avg, exp_avg_sq, step
        self.slot_block, self.slot_rows, self.order = slot_block, slot_rows, order
        self.n_slots, _, self.block_rows = params.shape
        self.n_order = int(order.numel()) if n_order is None else int(n_order)

    @classmethod
    def empty(cls, n_slots: int, block_rows: int, device, dtype=torch.float32):
        """Slots for the block tier: nothing resident, order has room for
        every slot (the tier fills it)."""
        z = lambda: torch.zeros((n_slots, D, block_rows), dtype=dtype, device=device)
        return cls(z(), z(), z(), torch.zeros((n_slots, block_rows), dtype=torch.int32, device=device),
                   torch.full((n_slots,), -1, dtype=torch.int32, device=device),
                   torch.zeros((n_slots,), dtype=torch.int32, device=device),
                   torch.zeros((n_slots,), dtype=torch.int32, device=device), n_order=0)

    @classmethod
    def from_dense(cls, theta: torch.Tensor, block_rows: int = 65536, extra_slots: int = 0):
        """All-resident pool holding rows of ``theta`` (N, 59) in blocks of
        ``block_rows``; block k sits in slot k."""
        N = theta.shape[0]
        K = max(1, math.ceil(N / block_rows))
        dev = theta.device
        pad = torch.zeros((K * block_rows, D), dtype=theta.dtype, device=dev)
        pad[:N] = theta
        params = pad.view(K, block_rows, D).transpose(1, 2).contiguous()
        if extra_slots:
            params = torch.cat([params, torch.zeros((extra_slots, D, block_rows), dtype=theta.dtype, device=dev)])
        S = K + extra_slots
        rows = [block_rows] * K
        rows[-1] = N - (K - 1) * block_rows
        rows += [0] * extra_slots
        sb = list(range(K)) + [-1] * extra_slots
        return cls(params, torch.zeros_like(params), torch.zeros_like(params),
                   torch.zeros((S, block_rows), dtype=torch.int32, device=dev),
                   torch.tensor(sb, dtype=torch.int32, device=dev),
                   torch.tensor(rows, dtype=torch.int32, device=dev),
                   torch.arange(K, dtype=torch.int32, device=dev))

    @property
    def n_pidx(self) -> int:
        return self.n_order * self.block_rows

    def c(self) -> L.tide_pool:
        p = L.tide_pool()
        p.params = self.params.data_ptr()
        p.exp_avg = self.exp_avg.data_ptr()
        p.exp_avg_sq = self.exp_avg_sq.data_ptr()
        p.step = self.step.data_ptr()
        p.slot_block = self.slot_block.data_ptr()
        p.slot_rows = self.slot_rows.data_ptr()
        p.order = self.order.data_ptr() if self.order.numel() else self.slot_block.data_ptr()
        p.n_slots = self.n_slots
        p.block_rows = self.block_rows
        p.n_order = self.n_order
        p.dtype = _dtype_code(self.params.dtype)
        return p

    def dense(self, n: int) -> torch.Tensor:
        """Rows 0..n-1 of the table, assuming block k sits in slot k."""
        return self.params[: math.ceil(n / self.block_rows)].transpose(1, 2).reshape(-1, D)[:n]


@dataclass
class Proj:
    rec: torch.Tensor
    depth: torch.Tensor
    rect: torch.Tensor
    tiles_touched: torch.Tensor
    active: torch.Tensor
    act_idx: torch.Tensor
    n_active: torch.Tensor
    n_cams: int
    n_pidx: int
    dtype: int

    def c(self) -> L.tide_proj:
        p = L.tide_proj()
        p.rec = _dptr(self.rec)
        p.depth = _dptr(self.depth)
        p.rect = _dptr(self.rect)
        p.tiles_touched = _dptr(self.tiles_touched)
        p.active = _dptr(self.active)
        p.act_idx = _dptr(self.act_idx)
        p.n_active = _dptr(self.n_active)
        p.n_pidx = self.n_pidx
        p.n_cams = self.n_cams
        p.dtype = self.dtype
        return p


@dataclass
class Frame:
    image: torch.Tensor
    t_final: torch.Tensor
    last: torch.Tensor
    visits: torch.Tensor      # [2][V]: forward visits, backward visits per view
    width: int
    height: int

    @property
    def visits_fwd(self) -> torch.Tensor:
        return self.visits[0]

    @property
    def visits_bwd(self) -> torch.Tensor:
        return self.visits[1]

    def c(self) -> L.tide_frame:
        f = L.tide_frame()
        f.image = self.image.data_ptr()
        f.t_final = self.t_final.data_ptr()
        f.last = self.last.data_ptr()
        f.visits = self.visits.data_ptr()
        f.width = self.width
        f.height = self.height
        return f


def adam_cfg(lr59, beta1=0.9, beta2=0.999, eps=1e-15, kappa=1.32) -> L.tide_adam_cfg:
    c = L.tide_adam_cfg()
    c.lr = (C.c_float * D)(*[float(x) for x in lr59])
    c.beta1, c.beta2, c.eps, c.kappa = beta1, beta2, eps, kappa
    return c


LR59 = [1.6e-4] * 3 + [5e-3] * 3 + [1e-3] * 4 + [5e-2] + [2.5e-3] * 48


class Rasterizer:
    """Holds the per-iteration device buffers and calls the C ABI."""

    def __init__(self, device="cuda"):
        self.lib = L.load()
        self.device = torch.device(device)
        self.buf = Buffers(self.device)
        self.inst_cap = 0

    # ------------------------------------------------------------- forward
    def preprocess(self, pool: Pool, cams, cam_arr=None) -> Proj:
        V = len(cams)
        N = pool.n_pidx
        dt = pool.params.dtype
        dev = self.device
        proj = Proj(rec=self.buf.get("rec", V * N * 12 * pool.params.element_size()).view(dt)[: V * N * 12],
                    depth=self.buf.get("depth", V * N * 4).view(torch.float32)[: V * N],
                    rect=self.buf.get("rect", V * N * 8).view(torch.int32)[: 2 * V * N],
                    tiles_touched=self.buf.get("tt", V * N * 4).view(torch.int32)[: V * N],
                    active=self.buf.get("active", N * 4).view(torch.int32)[:N],
                    act_idx=self.buf.get("act_idx", N * 4).view(torch.int32)[:N],
                    n_active=self.buf.get("n_active", 4).view(torch.int32)[:1],
                    n_cams=V, n_pidx=N, dtype=_dtype_code(dt))
        cam_arr = cam_arr if cam_arr is not None else L.camera_array(cams)
        wsb = self.lib.tide_preprocess_ws_bytes(N)
        ws = self.buf.get("pre_ws", wsb)
        pc = pool.c()
        self._pc = proj.c()
        L.check(self.lib.tide_preprocess(C.byref(pc), cam_arr, V, C.byref(self._pc), C.c_void_p(ws.data_ptr()),
                                         wsb, C.c_void_p(_stream())))
        return proj

    def bin_sort(self, proj: Proj, tiles_x: int, tiles_y: int) -> L.tide_bins:
        V, N = proj.n_cams, proj.n_pidx
        if self.inst_cap == 0:
            self.inst_cap = max(4 * V * N, 1 << 16)
        bins = L.tide_bins()
        pc = proj.c()
        for _ in range(4):
            wsb = self.lib.tide_bin_sort_ws_bytes(V, N, tiles_x, tiles_y, self.inst_cap)
            ws = self.buf.get("bin_ws", wsb)
            code = self.lib.tide_bin_sort(C.byref(pc), tiles_x, tiles_y, C.c_void_p(ws.data_ptr()), ws.numel(),
                                          C.byref(bins), C.c_void_p(_stream()))
            if code == L.TIDE_ECAPACITY:
                self.inst_cap = int(bins.n_inst * 1.25) + 4096
                continue
            L.check(code)
            return bins
        raise L.TideError(L.TIDE_ECAPACITY, "bin_sort capacity retries exhausted")

    def new_frame(self, V: int, width: int, height: int, dtype) -> Frame:
        dev = self.device
        return Frame(image=torch.empty((V, 3, height, width), dtype=dtype, device=dev),
                     t_final=torch.empty((V, height, width), dtype=dtype, device=dev),
                     last=torch.empty((V, height, width), dtype=torch.int32, device=dev),
                     visits=torch.zeros((2, V), dtype=torch.int64, device=dev), width=width, height=height)

    def render(self, proj: Proj, bins: L.tide_bins, width: int, height: int, bg=(0.0, 0.0, 0.0),
               fr: Frame | None = None) -> Frame:
        if fr is None:
            fr = self.new_frame(proj.n_cams, width, height, torch.float32 if proj.dtype == L.TIDE_F32
                                else torch.float64)
        bgc = (C.c_float * 3)(*[float(x) for x in bg])
        fc = fr.c()
        pc = proj.c()
        L.check(self.lib.tide_render_fwd(C.byref(pc), C.byref(bins), bgc, C.byref(fc), C.c_void_p(_stream())))
        return fr

    def forward(self, pool: Pool, cams, bg=(0.0, 0.0, 0.0)):
        W, H = int(cams[0].width), int(cams[0].height)
        cam_arr = L.camera_array(cams)
        proj = self.preprocess(pool, cams, cam_arr)
        # the frame is made before the binning, which returns only once its
        # counts have reached the host
        fr = self.new_frame(len(cams), W, H, pool.params.dtype)
        bins = self.bin_sort(proj, (W + TILE - 1) // TILE, (H + TILE - 1) // TILE)
        self.render(proj, bins, W, H, bg, fr)
        return proj, bins, fr

    # ----------------------------------------------------------------- loss
    def loss(self, image: torch.Tensor, target: torch.Tensor):
        V, _, H, W = image.shape
        dt = _dtype_code(image.dtype)
        wsb = self.lib.tide_loss_ws_bytes(V, H, W, dt)
        ws = self.buf.get("loss_ws", wsb)
        out = torch.empty((1,), dtype=torch.float64, device=self.device)
        g = torch.empty_like(image)
        L.check(self.lib.tide_loss(C.c_void_p(image.data_ptr()), C.c_void_p(target.data_ptr()), V, H, W, dt,
                                   C.c_void_p(out.data_ptr()), C.c_void_p(g.data_ptr()), C.c_void_p(ws.data_ptr()),
                                   ws.numel(), C.c_void_p(_stream())))
        return out, g

    # ------------------------------------------------------------- backward
    def backward(self, pool: Pool, cams, proj: Proj, bins: L.tide_bins, fr: Frame, dimage: torch.Tensor,
                 bg=(0.0, 0.0, 0.0), grad: torch.Tensor | None = None) -> torch.Tensor:
        N = proj.n_pidx
        dt = pool.params.dtype
        if grad is None or grad.shape[1] < N:
            grad = torch.empty((D, max(N, 1)), dtype=dt, device=self.device)
        wsb = self.lib.tide_render_bwd_ws_bytes(C.byref(bins), proj.dtype)
        ws = self.buf.get("bwd_ws", wsb)
        cam_arr = L.camera_array(cams)
        bgc = (C.c_float * 3)(*[float(x) for x in bg])
        pc, qc, fc = pool.c(), proj.c(), fr.c()
        dimage = dimage.contiguous()
        L.check(self.lib.tide_render_bwd(C.byref(pc), cam_arr, len(cams), C.byref(qc), C.byref(bins), C.byref(fc),
                                         bgc, C.c_void_p(dimage.data_ptr()), C.c_void_p(grad.data_ptr()),
                                         grad.shape[1], C.c_void_p(ws.data_ptr()), ws.numel(),
                                         C.c_void_p(_stream())))
        return grad

    def adam(self, pool: Pool, proj: Proj, grad: torch.Tensor, cfg: L.tide_adam_cfg, spheres=None, dirty=None):
        pc, qc = pool.c(), proj.c()
        nb = int(spheres.shape[0]) if spheres is not None else (int(dirty.shape[0]) if dirty is not None else 0)
        wsb = self.lib.tide_adam_ws_bytes(proj.n_pidx)
        ws = self.buf.get("adam_ws", wsb)
        L.check(self.lib.tide_adam_sparse(C.byref(pc), C.byref(qc), C.c_void_p(grad.data_ptr()), grad.shape[1],
                                          C.byref(cfg), C.c_void_p(spheres.data_ptr() if spheres is not None else 0),
                                          C.c_void_p(dirty.data_ptr() if dirty is not None else 0), nb,
                                          C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(_stream())))


    def backward_adam(self, pool: Pool, cams, proj: Proj, bins: L.tide_bins, fr: Frame, dimage: torch.Tensor,
                      cfg: L.tide_adam_cfg, spheres=None, dirty=None, bg=(0.0, 0.0, 0.0)) -> None:
        """backward then adam, with no gradient stored in between (same bits)."""
        nb = int(spheres.shape[0]) if spheres is not None else (int(dirty.shape[0]) if dirty is not None else 0)
        wsb = self.lib.tide_render_bwd_ws_bytes(C.byref(bins), proj.dtype)
        ws = self.buf.get("bwd_ws", wsb)
        cam_arr = L.camera_array(cams)
        bgc = (C.c_float * 3)(*[float(x) for x in bg])
        pc, qc, fc = pool.c(), proj.c(), fr.c()
        dimage = dimage.contiguous()
        L.check(self.lib.tide_render_bwd_adam(C.byref(pc), cam_arr, len(cams), C.byref(qc), C.byref(bins),
                                              C.byref(fc), bgc, C.c_void_p(dimage.data_ptr()), C.byref(cfg),
                                              C.c_void_p(spheres.data_ptr() if spheres is not None else 0),
                                              C.c_void_p(dirty.data_ptr() if dirty is not None else 0), nb,
                                              C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(_stream())))


def dense_grad(proj: Proj, grad: torch.Tensor, n: int) -> torch.Tensor:
    """Compact [59][n_active] gradient -> dense (n, 59) for an all-resident
    pool whose pidx equals the global row id."""
    act = proj.active[:n].bool()
    idx = proj.act_idx[:n][act].long()
    out = torch.zeros((n, D), dtype=grad.dtype, device=grad.device)
    out[act] = grad[:, idx].T
    return out


class TideRasterize(torch.autograd.Function):
    """image = render(theta); backward = the library's adjoint (dense dtheta)."""

    @staticmethod
    def forward(ctx, theta, cams, bg, block_rows, rast):
        pool = Pool.from_dense(theta.detach().contiguous(), block_rows)
        proj, bins, fr = rast.forward(pool, cams, bg)
        ctx.save = (pool, cams, proj, bins, fr, bg, rast, theta.shape[0])
        return fr.image

    @staticmethod
    def backward(ctx, dimage):
        pool, cams, proj, bins, fr, bg, rast, n = ctx.save
        g = rast.backward(pool, cams, proj, bins, fr, dimage.contiguous(), bg)
        return dense_grad(proj, g, n), None, None, None, None


def render(theta: torch.Tensor, cams, bg=(0.0, 0.0, 0.0), block_rows: int = 4096, rast: Rasterizer | None = None):
    """Differentiable render of a dense (N, 59) table (float32 or float64).
    Each call gets its own buffers unless ``rast`` is given, so that saved
    forward state survives further renders before backward."""
    rast = rast or Rasterizer(theta.device)
    return TideRasterize.apply(theta, cams, bg, block_rows, rast)


def bins_views(rast: Rasterizer, bins: L.tide_bins) -> dict:
    """Torch views of the arrays tide_bin_sort left in the workspace (for
    inspection and tests)."""
    ws = rast.buf.bufs["bin_ws"]
    base = ws.data_ptr()

    def view(ptr, count):
        off = int(ptr) - base
        assert 0 <= off and off + 4 * count <= ws.numel()
        return ws[off: off + 4 * count].view(torch.int32)

    V, T = bins.n_cams, bins.tiles_x * bins.tiles_y
    tv_off = int(bins.tile_visits) - base
    assert tv_off % 8 == 0 and 0 <= tv_off and tv_off + 16 * V * T <= ws.numel()
    return dict(vis_rec=view(bins.vis_rec, bins.n_vis), inst_off=view(bins.inst_off, bins.n_vis + 1),
                inst_e=view(bins.inst_e, bins.n_inst), inst_rec=view(bins.inst_rec, bins.n_inst),
                ranges=view(bins.ranges, 2 * V * T).view(V * T, 2), tile_order=view(bins.tile_order, V * T),
                tile_visits=ws[tv_off: tv_off + 16 * V * T].view(torch.int64).view(2, V * T)[0])
