"""torch.autograd.Function over the rasterizer: fgs_render_fwd in forward, fgs_render_bwd in
backward. The forward state (projected records, sorted tile lists, per-pixel last contributor)
stays with the autograd graph until backward runs.

Tensors are SoA planes on the GPU: mean (3, N), log_scale (3, N), quat (4, N) as (w, x, y, z),
opacity_logit (N,), rgb (3, N); float32, contiguous. Outputs: rgb (3, H, W), depth (H, W),
alpha (H, W).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import (CGaussians, Context, FgsError, ERR_CAPACITY, RenderOpts, _check, _f32, _lib, camera,
               ctx_required_pairs, state_bytes)

_default_ctx: dict = {}


def _context(device) -> Context:
    key = (device.index, torch.cuda.current_stream(device).cuda_stream)
    if key not in _default_ctx:
        _default_ctx[key] = Context(torch.cuda.current_stream(device))
    return _default_ctx[key]


def _planes(mean, log_scale, quat, opacity_logit, rgb) -> CGaussians:
    n = mean.shape[1]
    for t, rows in ((mean, 3), (log_scale, 3), (quat, 4), (rgb, 3)):
        assert t.shape == (rows, n) and t.is_contiguous() and t.dtype == torch.float32 and t.is_cuda
    assert opacity_logit.shape == (n,) and opacity_logit.is_contiguous() and opacity_logit.dtype == torch.float32
    g = CGaussians()
    g.n, g.stride = n, n
    g.mean, g.log_scale, g.quat = _f32(mean), _f32(log_scale), _f32(quat)
    g.opacity_logit, g.rgb = _f32(opacity_logit), _f32(rgb)
    return g


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(actx, mean, log_scale, quat, opacity_logit, rgb, cam, opts, fctx):
        n = mean.shape[1]
        H, W = int(cam.height), int(cam.width)
        dev = mean.device
        g = _planes(mean, log_scale, quat, opacity_logit, rgb)
        pairs = 64 * n + (1 << 16)
        for _ in range(2):
            state = torch.empty(state_bytes(n, W, H, pairs, opts), dtype=torch.uint8, device=dev)
            out_rgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
            out_d = torch.empty((H, W), dtype=torch.float32, device=dev)
            out_a = torch.empty((H, W), dtype=torch.float32, device=dev)
            from . import CImage
            img = CImage(_f32(out_rgb), _f32(out_d), _f32(out_a), None, None)
            _check(_lib.fgs_render_fwd(fctx.handle, C.byref(g), C.byref(camera(cam)), C.byref(opts.c()),
                                       C.byref(img), C.c_void_p(state.data_ptr()), state.numel()), fctx.handle)
            try:
                fctx.check()
                break
            except FgsError as e:
                if e.status != ERR_CAPACITY:
                    raise
                pairs = ctx_required_pairs(e) + 1024
        actx.save_for_backward(mean, log_scale, quat, opacity_logit, rgb)
        actx.state, actx.cam, actx.opts, actx.fctx = state, cam, opts, fctx
        return out_rgb, out_d, out_a

    @staticmethod
    def backward(actx, g_rgb, g_depth, g_alpha):
        mean, log_scale, quat, opacity_logit, rgb = actx.saved_tensors
        g = _planes(mean, log_scale, quat, opacity_logit, rgb)
        grads = [torch.zeros_like(t) for t in (mean, log_scale, quat, opacity_logit, rgb)]
        gg = _planes(*grads)

        def prep(t, shape):
            if t is None:
                return torch.zeros(shape, dtype=torch.float32, device=mean.device)
            return t.contiguous().float()
        H, W = int(actx.cam.height), int(actx.cam.width)
        gr, gd = prep(g_rgb, (3, H, W)), prep(g_depth, (H, W))
        ga = None if g_alpha is None else g_alpha.contiguous().float()
        _check(_lib.fgs_render_bwd(actx.fctx.handle, C.byref(g), C.byref(camera(actx.cam)), C.byref(actx.opts.c()),
                                   C.c_void_p(actx.state.data_ptr()), actx.state.numel(), _f32(gr), _f32(gd),
                                   _f32(ga), C.byref(gg)), actx.fctx.handle)
        return (*grads, None, None, None)


def render(mean, log_scale, quat, opacity_logit, rgb, cam, opts: RenderOpts | None = None, ctx: Context | None = None):
    """Differentiable render: returns (rgb (3,H,W), depth (H,W), alpha (H,W))."""
    opts = opts or RenderOpts()
    ctx = ctx or _context(mean.device)
    return RenderFunction.apply(mean, log_scale, quat, opacity_logit, rgb, cam, opts, ctx)
