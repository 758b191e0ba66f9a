"""torch.autograd.Function wrappers of the variable-coefficient heat run and of
its loss: argument marshalling only.

HeatVC.apply(u0, kappa, dt, steps, ckpt=0) -> u_T runs hx_heat_vc_forward
(keeping sqrt(T) checkpoints) and, in backward, hx_heat_vc_backward (segment
recompute + reverse sweep, conductivity gradient folded in FP64) followed by
hx_launch_cast64.  HeatLoss.apply(u, y) -> 0.5 ||u - y||^2 (FP64 scalar)
runs hx_launch_loss; its backward is hx_launch_scale of the saved residual.

Every hx operation is queued on torch's current stream (the context is
created with that stream as its only compute stream), so torch's ordering and
its caching allocator see the hx work as ordinary stream work.
"""
from __future__ import annotations

import torch

from . import (HX_F32, HX_F64, hx_buffer_destroy, hx_buffer_wrap, hx_ctx_create,
               hx_event_release, hx_heat_vc_backward, hx_heat_vc_forward, hx_launch_cast64,
               hx_launch_loss, hx_launch_scale, hx_vc_args, hx_vc_schedule)

_CTXS = {}


def _context():
    stream = torch.cuda.current_stream()
    key = (stream.device.index, stream.cuda_stream)
    c = _CTXS.get(key)
    if c is None:
        c = hx_ctx_create(stream.device.index or 0, compute_streams=1,
                          external_stream=stream.cuda_stream)
        _CTXS[key] = c
    return c


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return HX_F32
    if t.dtype == torch.float64:
        return HX_F64
    raise TypeError("hx kernels take float32 or float64 tensors")


class _Wrapped:
    """Non-owning hx buffers over torch tensors for the duration of one call."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.handles = []

    def __call__(self, t):
        if t is None or t.numel() == 0:
            return 0
        h = hx_buffer_wrap(self.ctx, t.data_ptr(), t.numel() * t.element_size())
        self.handles.append(h)
        return h

    def close(self):
        for h in self.handles:
            hx_buffer_destroy(self.ctx, h)


def _check(u0: torch.Tensor, kappa: torch.Tensor):
    if u0.dim() != 2 or u0.shape != kappa.shape:
        raise ValueError("u0 and kappa must be 2D tensors of one shape")
    if u0.dtype != kappa.dtype or not u0.is_cuda or u0.device != kappa.device:
        raise ValueError("u0 and kappa must share dtype and GPU")


class HeatVC(torch.autograd.Function):
    """u_T = A(kappa)^T u0 with gradients for u0 and kappa."""

    @staticmethod
    def forward(ctx, u0, kappa, dt, steps, ckpt=0):
        _check(u0, kappa)
        u0 = u0.contiguous()
        kappa = kappa.contiguous()
        ny, nx = u0.shape
        S, nseg = hx_vc_schedule(int(steps), int(ckpt))
        uT = torch.empty_like(u0)
        ck = torch.empty((max(nseg - 1, 0), ny, nx), dtype=u0.dtype, device=u0.device)
        work = torch.empty((2 if steps > 1 else 0, ny, nx), dtype=u0.dtype, device=u0.device)
        c = _context()
        w = _Wrapped(c)
        try:
            a = hx_vc_args(_dtype_code(u0), nx, ny, float(dt), int(steps), int(ckpt),
                           w(u0), w(kappa), w(uT), w(ck), w(work), 0, 0, 0, 0, 0, 0)
            hx_event_release(c, hx_heat_vc_forward(c, a))
        finally:
            w.close()
        ctx.save_for_backward(u0, kappa, ck)
        ctx.cfg = (float(dt), int(steps), int(ckpt), S)
        return uT

    @staticmethod
    def backward(ctx, g):
        u0, kappa, ck = ctx.saved_tensors
        dt, steps, ckpt, S = ctx.cfg
        ny, nx = u0.shape
        g = g.contiguous()
        lam0 = torch.empty_like(u0)
        gk64 = torch.empty((ny, nx), dtype=torch.float64, device=u0.device)
        gacc = torch.empty_like(u0)
        seg = torch.empty((max(S - 1, 0), ny, nx), dtype=u0.dtype, device=u0.device)
        work = torch.empty((2 if steps > 1 else 0, ny, nx), dtype=u0.dtype, device=u0.device)
        gk = torch.empty_like(kappa)
        c = _context()
        w = _Wrapped(c)
        try:
            code = _dtype_code(u0)
            a = hx_vc_args(code, nx, ny, dt, steps, ckpt, w(u0), w(kappa), 0, w(ck), w(work),
                           w(seg), w(g), w(lam0), w(gk64), w(gacc), 0)
            hx_event_release(c, hx_heat_vc_backward(c, a))
            hx_event_release(c, hx_launch_cast64(c, code, nx * ny, w(gk64), w(gk)))
        finally:
            w.close()
        return lam0, gk, None, None, None


class HeatLoss(torch.autograd.Function):
    """0.5 ||u - y||^2 reduced in FP64 (a 0-dim float64 tensor)."""

    @staticmethod
    def forward(ctx, u, y):
        if u.shape != y.shape or u.dtype != y.dtype:
            raise ValueError("u and y must have one shape and dtype")
        u = u.contiguous()
        y = y.contiguous()
        resid = torch.empty_like(u)
        out = torch.empty((), dtype=torch.float64, device=u.device)
        work = torch.empty(4096, dtype=torch.float64, device=u.device)
        c = _context()
        w = _Wrapped(c)
        try:
            hx_event_release(c, hx_launch_loss(c, _dtype_code(u), u.numel(), w(u), w(y),
                                               w(resid), w(out), w(work)))
        finally:
            w.close()
        ctx.save_for_backward(resid)
        return out

    @staticmethod
    def backward(ctx, g):
        (resid,) = ctx.saved_tensors
        g = g.to(torch.float64).contiguous().reshape(())
        grad = torch.empty_like(resid)
        c = _context()
        w = _Wrapped(c)
        try:
            hx_event_release(c, hx_launch_scale(c, _dtype_code(resid), resid.numel(), w(resid),
                                                w(g), w(grad)))
        finally:
            w.close()
        return grad, None
