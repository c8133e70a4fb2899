"""MI355X (gfx950) implementation of the FGS-SLAM mapping hot path (arXiv 2503.01109).

This module is a thin ctypes binding of ``libfgs.so`` (include/fgs.h): it marshals torch
tensors (device memory) and plain Python values into the C structs and calls the library.
Every step of rendering, differentiation, loss, optimisation and seeding runs in the
library's HIP kernels; nothing here computes any part of the method. There is no CPU
fallback: without the built library the import fails.

Gaussian parameters live in one float32 device tensor of shape (14, capacity), rows:
0-2 mean, 3-5 log-scale, 6-9 quaternion (w, x, y, z), 10 opacity logit, 11-13 rgb;
the first n columns are the gaussians.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfgs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(the HIP library is required; there is no fallback)")

# torch ships its own HIP runtime (same soname as /opt/rocm's). Loading torch first makes the
# library bind to that one runtime instead of pulling in a second copy from /opt/rocm.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

OK, ERR_INVALID_ARG, ERR_CAPACITY, ERR_HIP, ERR_UNSUPPORTED = 0, -1, -2, -3, -5
_fp = C.POINTER(C.c_float)
_i32p = C.POINTER(C.c_int32)


class FgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} [{_lib.fgs_status_str(status).decode()}]")
        self.status = status


class CCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R_cw", C.c_float * 9), ("t_cw", C.c_float * 3),
                ("z_near", C.c_float)]


class CGaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("stride", C.c_int64), ("mean", _fp), ("log_scale", _fp), ("quat", _fp),
                ("opacity_logit", _fp), ("rgb", _fp)]


class CRenderOpts(C.Structure):
    _fields_ = [("sigma_cut", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("T_min", C.c_float), ("lowpass", C.c_float), ("bg", C.c_float * 3), ("bg_depth", C.c_float),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32)]


class CImage(C.Structure):
    _fields_ = [("rgb", _fp), ("depth", _fp), ("alpha", _fp), ("T_final", _fp), ("n_contrib", _i32p)]


class CAdam(C.Structure):
    _fields_ = [("m", CGaussians), ("v", CGaussians), ("step", C.c_int64), ("lr", C.c_float * 5),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class CTarget(C.Structure):
    _fields_ = [("rgb", _fp), ("depth", _fp)]


class CLossOpts(C.Structure):
    _fields_ = [("lambda_rgb", C.c_float), ("lambda_depth", C.c_float), ("lambda_reg", C.c_float),
                ("reg_dev", _fp)]


class CSeedOpts(C.Structure):
    _fields_ = [("D0", C.c_double), ("m", C.c_int32), ("n", C.c_int32), ("tile", C.c_int32),
                ("alpha_h", C.c_float), ("alpha_l", C.c_float), ("opacity_logit", C.c_float),
                ("depth_min", C.c_float), ("depth_max", C.c_float), ("use_prior", C.c_int32), ("prior", C.c_void_p),
                ("render_alpha", _fp), ("render_depth", _fp), ("render_rgb", _fp), ("miss_alpha", C.c_float),
                ("miss_depth", C.c_float), ("miss_rgb", C.c_float)]


class CSeedOut(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("pixel", _i32p), ("is_high", C.POINTER(C.c_uint8)), ("mean", _fp),
                ("radius", _fp), ("rgb", _fp), ("tile_count", _i32p), ("n_dev", C.POINTER(C.c_int64)),
                ("params", CGaussians), ("E", C.POINTER(C.c_double)), ("hist", C.POINTER(C.c_uint32)),
                ("threshold", _i32p), ("from_prior", C.POINTER(C.c_uint8)), ("missing", C.POINTER(C.c_uint8))]


class CPruneOpts(C.Structure):
    _fields_ = [("min_opacity", C.c_float), ("max_scale", C.c_float)]


class CCloudOpts(C.Structure):
    _fields_ = [("cell", C.c_float), ("k", C.c_int32), ("eps", C.c_double), ("keep_knn", C.c_int32)]


class CGicpOpts(C.Structure):
    _fields_ = [("d_max", C.c_float), ("max_iter", C.c_int32), ("eps_rot", C.c_double), ("eps_trans", C.c_double)]


class CGicpResult(C.Structure):
    _fields_ = [("T", C.c_double * 16), ("iterations", C.c_int32), ("status", C.c_int32),
                ("correspondences", C.c_int64), ("cost", C.c_double)]


class CPriorAdam(C.Structure):
    _fields_ = [("m", _fp), ("v", _fp), ("step", C.c_int64), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


_vp = C.c_void_p
_P = C.POINTER
_sigs = {
    "fgs_ctx_create": [_P(_vp), _vp],
    "fgs_ctx_destroy": [_vp],
    "fgs_ctx_set_stream": [_vp, _vp],
    "fgs_ctx_check": [_vp],
    "fgs_ctx_stats": [_vp, _P(C.c_int64)],
    "fgs_last_error": [_vp, C.c_char_p, C.c_size_t],
    "fgs_state_bytes": [C.c_int64, C.c_int32, C.c_int32, C.c_int64, _P(CRenderOpts), _P(C.c_int64)],
    "fgs_render_fwd": [_vp, _P(CGaussians), _P(CCamera), _P(CRenderOpts), _P(CImage), _vp, C.c_int64],
    "fgs_render_bwd": [_vp, _P(CGaussians), _P(CCamera), _P(CRenderOpts), _vp, C.c_int64, _fp, _fp, _fp,
                       _P(CGaussians)],
    "fgs_render_bwd_noalloc": [_vp, _P(CGaussians), _P(CCamera), _P(CRenderOpts), _vp, C.c_int64, _fp, _fp, _fp,
                               _P(CGaussians)],
    "fgs_map_step": [_vp, _P(CGaussians), _P(CAdam), C.c_int32, _P(CCamera), _P(CTarget), _P(CRenderOpts),
                     _P(CLossOpts), _fp, _fp, _P(CGaussians)],
    "fgs_loss_l1": [_vp, C.c_int64, _fp, _fp, _P(CTarget), _P(CLossOpts), _fp, _fp, _fp, _fp],
    "fgs_ssim": [_vp, C.c_int32, C.c_int32, _fp, _fp, _fp, _fp],
    "fgs_adam_step": [_vp, _P(CGaussians), _P(CGaussians), _P(CAdam)],
    "fgs_frame_points": [_vp, _fp, _P(CCamera), _P(C.c_double), C.c_int32, C.c_float, C.c_float, _fp, C.c_int64,
                         _P(C.c_int64), _P(C.c_int64)],
    "fgs_cloud_create": [_vp, C.c_int64, C.c_int64, _fp, _P(CCloudOpts), _P(_vp)],
    "fgs_cloud_destroy": [_vp],
    "fgs_cloud_read": [_vp, _P(C.c_double), _P(C.c_int32), _P(C.c_int64), _P(C.c_int32)],
    "fgs_gicp_linearize": [_vp, _vp, _vp, _P(C.c_double), C.c_float, _P(C.c_double), _P(C.c_int32)],
    "fgs_gicp_align": [_vp, _vp, _vp, _P(C.c_double), _P(CGicpOpts), _P(CGicpResult)],
    "fgs_prune": [_vp, _P(CPruneOpts), C.c_int32, _P(CGaussians), _P(CGaussians), _P(C.c_int64), _P(C.c_uint8),
                  _P(C.c_int64)],
    "fgs_ctx_profile": [_vp, C.c_int32],
    "fgs_ctx_profile_stage": [_vp, C.c_char_p, _P(C.c_double), _P(C.c_int64)],
    "fgs_ctx_profile_counts": [_vp, _P(C.c_int64)],
    "fgs_ctx_profile_work": [_vp, _P(C.c_int64)],
    "fgs_seed_gaussians": [_vp, _fp, _fp, _P(CCamera), _P(CSeedOpts), _P(CSeedOut), _P(C.c_int64)],
    "fgs_tile_features": [_vp, _fp, _fp, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_int64, _P(C.c_int32), _fp,
                          _P(C.c_int32)],
    "fgs_prior_forward": [_vp, C.c_int64, _fp, _fp, _fp],
    "fgs_prior_train_step": [_vp, C.c_int64, _fp, _fp, _fp, _P(CPriorAdam), _fp, _fp],
    "fgs_window_create": [_vp, C.c_int32, _P(CCamera), _P(C.c_int32), C.c_int32, _P(_vp)],
    "fgs_window_destroy": [_vp],
    "fgs_window_step": [_vp, _P(CGaussians), _P(CAdam), _P(CTarget), _P(CRenderOpts), _P(CLossOpts), _fp, _fp,
                        _P(CGaussians), C.c_int32],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.fgs_status_str.argtypes = [C.c_int]
_lib.fgs_status_str.restype = C.c_char_p

EXPORTED = sorted(list(_sigs) + ["fgs_status_str"])


def last_error(ctx=None) -> str:
    buf = C.create_string_buffer(1024)
    _lib.fgs_last_error(ctx, buf, len(buf))
    return buf.value.decode()


def _check(st: int, ctx=None):
    if st != OK:
        raise FgsError(st, last_error(ctx))


def _f32(t):
    """Device float pointer of a contiguous float32 tensor (None -> NULL)."""
    if t is None:
        return None
    assert t.dtype.is_floating_point and t.element_size() == 4, "float32 tensor expected"
    assert t.is_contiguous(), "contiguous tensor expected"
    return C.cast(C.c_void_p(t.data_ptr()), _fp)


@dataclass
class RenderOpts:
    """Compositing cutoffs and the rasterizer tile (see fgs_render_opts)."""
    sigma_cut: float = 3.0
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    lowpass: float = 0.3
    bg: tuple = (0.0, 0.0, 0.0)
    bg_depth: float = 0.0
    tile_w: int = 16
    tile_h: int = 16

    def c(self) -> CRenderOpts:
        o = CRenderOpts()
        o.sigma_cut, o.alpha_min, o.alpha_max, o.T_min = self.sigma_cut, self.alpha_min, self.alpha_max, self.T_min
        o.lowpass, o.bg_depth, o.tile_w, o.tile_h = self.lowpass, self.bg_depth, self.tile_w, self.tile_h
        o.bg[:] = [float(v) for v in self.bg]
        return o


def camera(cam) -> CCamera:
    """C camera from any object with width, height, fx, fy, cx, cy, R (3x3), t (3,), z_near."""
    c = CCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = [float(v) for row in cam.R for v in row]
    c.R_cw[:] = R
    c.t_cw[:] = [float(v) for v in cam.t]
    c.z_near = float(getattr(cam, "z_near", 0.2))
    return c


def gaussians(block, n: int | None = None) -> CGaussians:
    """C view of a (14, capacity) float32 device tensor holding n gaussians."""
    assert block.dim() == 2 and block.shape[0] == 14
    assert block.is_contiguous()
    cap = block.shape[1]
    n = cap if n is None else n
    base = block.data_ptr()
    g = CGaussians()
    g.n, g.stride = n, cap

    def row(k):
        return C.cast(C.c_void_p(base + 4 * k * cap), _fp)
    g.mean, g.log_scale, g.quat, g.opacity_logit, g.rgb = row(0), row(3), row(6), row(10), row(11)
    return g


class Context:
    """An fgs_ctx bound to a HIP stream (default: torch's current stream on the current device)."""

    def __init__(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        p = C.c_void_p()
        _check(_lib.fgs_ctx_create(C.byref(p), C.c_void_p(h)))
        self._p = p

    @property
    def handle(self):
        return self._p

    def close(self):
        if getattr(self, "_p", None):
            _lib.fgs_ctx_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(_lib.fgs_ctx_set_stream(self._p, C.c_void_p(h)), self._p)

    def check(self):
        """Waits for the stream and raises FgsError(ERR_CAPACITY) on a recorded overflow."""
        _check(_lib.fgs_ctx_check(self._p), self._p)

    STAGES = ("project", "depth_sort", "bin", "tile_sort", "raster_fwd", "ssim", "loss", "raster_bwd",
              "project_bwd", "adam")

    def profile(self, level: int = 2):
        """Start (clearing earlier records) or stop (0) HIP-event timing and work counters:
        level 1 times the rasterizer kernels only, level 2 every pipeline stage, level 3 every
        stage with the forward rasterizer's work counters (a slower counting variant)."""
        _check(_lib.fgs_ctx_profile(self._p, int(level)), self._p)

    def profile_report(self) -> dict:
        """{stage: (total_ms, launches)} plus 'counts': pairs examined, pairs blended, entries staged,
        forward launches."""
        rep = {}
        for s in self.STAGES:
            t = C.c_double()
            k = C.c_int64()
            _check(_lib.fgs_ctx_profile_stage(self._p, s.encode(), C.byref(t), C.byref(k)), self._p)
            rep[s] = (t.value, k.value)
        c = (C.c_int64 * 12)()
        _check(_lib.fgs_ctx_profile_work(self._p, c), self._p)
        rep["counts"] = dict(pairs_examined=c[0], pairs_blended=c[1], entries_staged=c[2], K_c=c[3], L_f=c[4],
                             L_b=c[5], forwards=c[6], bwd_wave_evals=c[7], bwd_wave_takes=c[8],
                             bwd_wave_few=c[9], bwd_pairs_blended=c[10], backwards=c[11])
        return rep

    def stats(self) -> dict:
        s = (C.c_int64 * 4)()
        _check(_lib.fgs_ctx_stats(self._p, s), self._p)
        return dict(pairs=s[0], visible=s[1], overflow=s[2], seeds=s[3])


def state_bytes(n: int, width: int, height: int, max_pairs: int, opts: RenderOpts | None = None) -> int:
    b = C.c_int64()
    _check(_lib.fgs_state_bytes(n, width, height, max_pairs, C.byref((opts or RenderOpts()).c()), C.byref(b)))
    return b.value


def render_fwd(ctx: Context, params, n: int, cam, opts: RenderOpts, rgb, depth, state, alpha=None, T_final=None,
               n_contrib=None):
    img = CImage(_f32(rgb), _f32(depth), _f32(alpha), _f32(T_final),
                 None if n_contrib is None else C.cast(C.c_void_p(n_contrib.data_ptr()), _i32p))
    _check(_lib.fgs_render_fwd(ctx.handle, C.byref(gaussians(params, n)), C.byref(camera(cam)),
                               C.byref(opts.c()), C.byref(img), C.c_void_p(state.data_ptr()),
                               state.numel() * state.element_size()), ctx.handle)


def render_bwd(ctx: Context, params, n: int, cam, opts: RenderOpts, state, dL_drgb, dL_ddepth, dL_dalpha, grad):
    _check(_lib.fgs_render_bwd(ctx.handle, C.byref(gaussians(params, n)), C.byref(camera(cam)),
                               C.byref(opts.c()), C.c_void_p(state.data_ptr()),
                               state.numel() * state.element_size(), _f32(dL_drgb), _f32(dL_ddepth),
                               _f32(dL_dalpha), C.byref(gaussians(grad, n))), ctx.handle)


NOALLOC_MAX_GAUSSIANS = 1 << 19


def render_bwd_noalloc(ctx: Context, params, n: int, cam, opts: RenderOpts, state, dL_drgb, dL_ddepth, dL_dalpha,
                       grad):
    """render_bwd through the entry point that allocates nothing (a static per-GPU scratch of
    NOALLOC_MAX_GAUSSIANS gradient records; calls that overlap on one GPU race)."""
    _check(_lib.fgs_render_bwd_noalloc(ctx.handle, C.byref(gaussians(params, n)), C.byref(camera(cam)),
                                       C.byref(opts.c()), C.c_void_p(state.data_ptr()),
                                       state.numel() * state.element_size(), _f32(dL_drgb), _f32(dL_ddepth),
                                       _f32(dL_dalpha), C.byref(gaussians(grad, n))), ctx.handle)


@dataclass
class Adam:
    """Adam state over a (14, capacity) parameter block (moments share its layout)."""
    m: object
    v: object
    step: int = 0
    lr: tuple = (1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3)
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15

    @staticmethod
    def like(params, **kw):
        import torch
        return Adam(torch.zeros_like(params), torch.zeros_like(params), **kw)

    def c(self, n: int) -> CAdam:
        a = CAdam()
        a.m, a.v = gaussians(self.m, n), gaussians(self.v, n)
        a.step = self.step
        a.lr[:] = [float(x) for x in self.lr]
        a.beta1, a.beta2, a.eps = self.beta1, self.beta2, self.eps
        return a


@dataclass
class LossOpts:
    """Weights of the mapping loss (Eq. 16): lambda_rgb on the L1 colour term, 1 - lambda_rgb on
    the SSIM term, lambda_depth on the L1 depth term, lambda_reg on the scale regulariser (Eq. 15).
    reg (optional float32 device tensor of one element) receives the regulariser's value."""
    lambda_rgb: float = 1.0
    lambda_depth: float = 0.1
    lambda_reg: float = 0.0
    reg: object = None

    def c(self) -> CLossOpts:
        return CLossOpts(self.lambda_rgb, self.lambda_depth, self.lambda_reg, _f32(self.reg))


def map_step(ctx: Context, params, n: int, adam: Adam, cams, targets, opts: RenderOpts,
             loss_opts: LossOpts | None = None, loss=None, psnr=None, grad_out=None):
    """One mapping iteration over len(cams) views. targets: list of (rgb (3,H,W), depth (H,W)) tensors."""
    V = len(cams)
    ccams = (CCamera * V)(*[camera(c) for c in cams])
    ctg = (CTarget * V)(*[CTarget(_f32(r), _f32(d)) for r, d in targets])
    ca = adam.c(n)
    st = _lib.fgs_map_step(ctx.handle, C.byref(gaussians(params, n)), C.byref(ca), V, ccams, ctg,
                           C.byref(opts.c()), C.byref((loss_opts or LossOpts()).c()), _f32(loss), _f32(psnr),
                           None if grad_out is None else C.byref(gaussians(grad_out, n)))
    adam.step = ca.step  # also on an overflow report, which sets the count back
    _check(st, ctx.handle)


class Window:
    """A keyframe window (fgs_window): n views of possibly different sizes mapped together, every
    view's tiles rendered by one persistent launch and back-propagated by another, the gradients
    summed per gaussian and Adam applied in one pass; optionally captured in a hipGraph."""

    def __init__(self, ctx: Context, cams, tiles=None, blocks_per_cu: int = 0):
        V = len(cams)
        ccams = (CCamera * V)(*[camera(c) for c in cams])
        ct = None
        if tiles is not None:
            flat = [int(x) for t in tiles for x in t]
            ct = (C.c_int32 * len(flat))(*flat)
        p = C.c_void_p()
        _check(_lib.fgs_window_create(ctx.handle, V, ccams, ct, int(blocks_per_cu), C.byref(p)), ctx.handle)
        self._p, self.ctx, self.n_views = p, ctx, V

    def close(self):
        if getattr(self, "_p", None):
            _lib.fgs_window_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, params, n: int, adam: Adam, targets, opts: RenderOpts, loss_opts: LossOpts | None = None,
             loss=None, psnr=None, grad_out=None, graph: bool = True):
        """One mapping iteration over the window. targets: list of (rgb (3,H,W), depth (H,W));
        loss / psnr: optional float32 device tensors of n_views entries."""
        if len(targets) != self.n_views:
            raise ValueError(f"window has {self.n_views} views, got {len(targets)} targets")
        for t in (loss, psnr):
            if t is not None and t.numel() < self.n_views:
                raise ValueError("loss / psnr need one entry per view")
        ctg = (CTarget * self.n_views)(*[CTarget(_f32(r), _f32(d)) for r, d in targets])
        ca = adam.c(n)
        st = _lib.fgs_window_step(self._p, C.byref(gaussians(params, n)), C.byref(ca), ctg, C.byref(opts.c()),
                                  C.byref((loss_opts or LossOpts()).c()), _f32(loss), _f32(psnr),
                                  None if grad_out is None else C.byref(gaussians(grad_out, n)), int(bool(graph)))
        adam.step = ca.step  # also on an overflow report, which sets the count back
        _check(st, self.ctx.handle)


def loss_l1(ctx: Context, rgb, depth, target_rgb, target_depth, loss_opts: LossOpts | None, dL_drgb, dL_ddepth,
            loss=None, psnr=None):
    tg = CTarget(_f32(target_rgb), _f32(target_depth))
    _check(_lib.fgs_loss_l1(ctx.handle, depth.numel(), _f32(rgb), _f32(depth), C.byref(tg),
                            C.byref((loss_opts or LossOpts()).c()), _f32(dL_drgb), _f32(dL_ddepth), _f32(loss),
                            _f32(psnr)), ctx.handle)


def ssim(ctx: Context, img, tgt, value=None, grad=None):
    """Structural similarity of img to tgt ((3, H, W) float32 device tensors; the SSIM term of
    Eq. 16): value (one-element tensor) receives the mean index, grad ((3, H, W)) its gradient."""
    _, H, W = img.shape
    _check(_lib.fgs_ssim(ctx.handle, W, H, _f32(img), _f32(tgt), _f32(value), _f32(grad)), ctx.handle)


def adam_step(ctx: Context, params, grad, n: int, adam: Adam):
    ca = adam.c(n)
    _check(_lib.fgs_adam_step(ctx.handle, C.byref(gaussians(params, n)), C.byref(gaussians(grad, n)),
                              C.byref(ca)), ctx.handle)
    adam.step = ca.step


@dataclass
class PruneOpts:
    """Pruning thresholds (Sec. III-D; see fgs_prune_opts): gaussians with opacity below
    min_opacity or any scale above max_scale (world units; 0 = no size test) are removed."""
    min_opacity: float = 0.005
    max_scale: float = 0.0

    def c(self) -> CPruneOpts:
        return CPruneOpts(self.min_opacity, self.max_scale)


def prune(ctx: Context, params, n: int, opts: PruneOpts | None = None, adam: Adam | None = None, keep=None,
          n_kept=None, sync: bool = True):
    """Prunes the first n gaussians of the (14, capacity) block `params` (Sec. III-D) into a new
    block of the same capacity, and the Adam moments with them. Returns (params, n_kept, adam):
    n_kept is an int when sync, else None (the count lands in the device int64 tensor n_kept when
    given); the returned Adam keeps the step count. keep (optional uint8 device tensor of n
    elements) receives 1 for survivors."""
    import torch
    blocks = [params] + ([adam.m, adam.v] if adam is not None else [])
    # moments beyond the survivors start at zero, for gaussians a caller appends later
    outs = [torch.empty_like(params)] + [torch.zeros_like(b) for b in blocks[1:]]
    k = len(blocks)
    src = (CGaussians * k)(*[gaussians(b, n) for b in blocks])
    dst = (CGaussians * k)(*[gaussians(b, n) for b in outs])
    host = C.c_int64(-1)
    _check(_lib.fgs_prune(ctx.handle, C.byref((opts or PruneOpts()).c()), k, src, dst,
                          _ptr(n_kept, C.POINTER(C.c_int64)), _ptr(keep, C.POINTER(C.c_uint8)),
                          C.byref(host) if sync else None), ctx.handle)
    new_adam = None
    if adam is not None:
        new_adam = Adam(outs[1], outs[2], step=adam.step, lr=adam.lr, beta1=adam.beta1, beta2=adam.beta2, eps=adam.eps)
    return outs[0], (host.value if sync else None), new_adam


# ------------------------------------ GICP tracking ------------------------------------

def _pose16(T):
    a = (C.c_double * 16)(*[float(v) for v in np.asarray(T, np.float64).reshape(16)])
    return a


def frame_points(ctx: Context, depth, cam, stride: int = 4, depth_min: float = 0.1, depth_max: float = 10.0,
                 pose_wc=None, capacity: int | None = None):
    """Lattice points of a depth frame ((H, W) float32 device tensor) as a (3, capacity) float32
    device tensor and their count (Sec. III-B, uniform downsampling). pose_wc: optional 4x4
    camera-to-world pose (host array); without it the points stay in the camera frame."""
    import torch
    H, W = int(cam.height), int(cam.width)
    cap = capacity if capacity is not None else ((W + stride - 1) // stride) * ((H + stride - 1) // stride)
    xyz = torch.empty((3, max(cap, 1)), dtype=torch.float32, device=depth.device)
    n = C.c_int64(-1)
    pose = None if pose_wc is None else _pose16(pose_wc)
    _check(_lib.fgs_frame_points(ctx.handle, _f32(depth), C.byref(camera(cam)), pose, int(stride), float(depth_min),
                                 float(depth_max), _f32(xyz), cap, None, C.byref(n)), ctx.handle)
    return xyz, n.value


@dataclass
class CloudOpts:
    """Grid cell (world units), neighbours per covariance, the regularised smallest eigenvalue,
    and whether to keep the neighbour lists (see fgs_cloud_opts)."""
    cell: float = 0.1
    k: int = 20
    eps: float = 1e-3
    keep_knn: bool = False

    def c(self) -> CCloudOpts:
        return CCloudOpts(self.cell, self.k, self.eps, int(bool(self.keep_knn)))


class Cloud:
    """A point cloud on the GPU with its grid, neighbours and plane-regularised covariances
    (fgs_cloud). xyz: (3, >= n) float32 device tensor; its first n columns are copied."""

    def __init__(self, ctx: Context, xyz, n: int | None = None, opts: CloudOpts | None = None):
        assert xyz.dim() == 2 and xyz.shape[0] == 3 and xyz.is_contiguous()
        self.ctx = ctx
        self.n = int(xyz.shape[1] if n is None else n)
        self.opts = opts or CloudOpts()
        h = C.c_void_p()
        _check(_lib.fgs_cloud_create(ctx.handle, self.n, xyz.shape[1], _f32(xyz), C.byref(self.opts.c()),
                                     C.byref(h)), ctx.handle)
        self._h = h

    @property
    def handle(self):
        return self._h

    def read(self):
        """(cov (6, n) float64 device tensor, knn (n, k) int32 device tensor or None)."""
        import torch
        cov = torch.empty((6, self.n), dtype=torch.float64, device="cuda")
        knn = torch.empty((self.n, self.opts.k), dtype=torch.int32, device="cuda") if self.opts.keep_knn else None
        _check(_lib.fgs_cloud_read(self._h, C.cast(C.c_void_p(cov.data_ptr()), C.POINTER(C.c_double)),
                                   _ptr(knn, _i32p), None, None), self.ctx.handle)
        return cov, knn

    def close(self):
        if getattr(self, "_h", None):
            _lib.fgs_cloud_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


@dataclass
class GicpOpts:
    """Correspondence radius, iteration limit and convergence thresholds (see fgs_gicp_opts)."""
    d_max: float = 0.1
    max_iter: int = 30
    eps_rot: float = 1e-6
    eps_trans: float = 1e-6

    def c(self) -> CGicpOpts:
        return CGicpOpts(self.d_max, self.max_iter, self.eps_rot, self.eps_trans)


def gicp_align(ctx: Context, source: Cloud, target: Cloud, T_init, opts: GicpOpts | None = None) -> dict:
    """Aligns source to target from the 4x4 pose T_init (Eq. 14); waits for the result:
    dict(T (4, 4) float64 numpy, iterations, status, correspondences, cost)."""
    r = CGicpResult()
    _check(_lib.fgs_gicp_align(ctx.handle, source.handle, target.handle, _pose16(T_init),
                               C.byref((opts or GicpOpts()).c()), C.byref(r)), ctx.handle)
    return dict(T=np.array(r.T[:], np.float64).reshape(4, 4), iterations=r.iterations, status=r.status,
                correspondences=r.correspondences, cost=r.cost)


def gicp_linearize(ctx: Context, source: Cloud, target: Cloud, T, d_max: float, corr: bool = True):
    """One linearisation of Eq. 14 at the 4x4 pose T: (29 float64 device tensor: H's upper
    triangle, b, cost, count; correspondences (n int32 device tensor) or None)."""
    import torch
    out = torch.empty(29, dtype=torch.float64, device="cuda")
    cr = torch.empty(source.n, dtype=torch.int32, device="cuda") if corr else None
    _check(_lib.fgs_gicp_linearize(ctx.handle, source.handle, target.handle, _pose16(T), float(d_max),
                                   C.cast(C.c_void_p(out.data_ptr()), C.POINTER(C.c_double)), _ptr(cr, _i32p)),
           ctx.handle)
    return out, cr


def render(ctx: Context, params, n: int, cam, opts: RenderOpts | None = None, max_pairs: int | None = None,
           aux: bool = True) -> dict:
    """Allocate output planes and a forward state, render, and check for a pair overflow (growing the
    state once to the reported size). Returns a dict of device tensors plus the state."""
    import torch
    opts = opts or RenderOpts()
    dev = params.device
    H, W = int(cam.height), int(cam.width)
    pairs = max_pairs if max_pairs is not None else 64 * n + (1 << 16)
    for _ in range(2):
        nbytes = state_bytes(n, W, H, pairs, opts)
        state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        out = dict(rgb=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                   depth=torch.empty((H, W), dtype=torch.float32, device=dev))
        if aux:
            out.update(alpha=torch.empty((H, W), dtype=torch.float32, device=dev),
                       T_final=torch.empty((H, W), dtype=torch.float32, device=dev),
                       n_contrib=torch.empty((H, W), dtype=torch.int32, device=dev))
        render_fwd(ctx, params, n, cam, opts, out["rgb"], out["depth"], state, out.get("alpha"),
                   out.get("T_final"), out.get("n_contrib"))
        try:
            ctx.check()
        except FgsError as e:
            if e.status != ERR_CAPACITY:
                raise
            pairs = ctx_required_pairs(e) + 1024
            continue
        out["state"] = state
        out["pairs"] = pairs
        return out
    raise FgsError(ERR_CAPACITY, "forward state still too small after growing it")


def ctx_required_pairs(err: FgsError) -> int:
    import re
    m = re.search(r"(\d+) \(tile, gaussian\) pairs needed", str(err))
    if not m:
        raise err
    return int(m.group(1))


@dataclass
class SeedOpts:
    """Fourier seeding constants (see fgs_seed_opts)."""
    D0: float = 30.0
    m: int = 2
    n: int = 8
    tile: int = 16
    alpha_h: float = 1.0
    alpha_l: float = 4.0
    opacity_logit: float = 0.0
    depth_min: float = 0.1
    depth_max: float = 10.0
    use_prior: int = 0
    prior: object = None
    # missing-region check (Sec. III-A, Eq. 9, 10): the current map rendered at the frame's pose
    # (float32 device tensors: opacity (H, W), depth (H, W), rgb (3, H, W)); None: no map yet
    render_alpha: object = None
    render_depth: object = None
    render_rgb: object = None
    miss_alpha: float = 0.5
    miss_depth: float = 0.1
    miss_rgb: float = 0.3

    def c(self) -> CSeedOpts:
        o = CSeedOpts()
        o.D0, o.m, o.n, o.tile = self.D0, self.m, self.n, self.tile
        o.alpha_h, o.alpha_l, o.opacity_logit = self.alpha_h, self.alpha_l, self.opacity_logit
        o.depth_min, o.depth_max, o.use_prior = self.depth_min, self.depth_max, self.use_prior
        o.prior = None if self.prior is None else C.c_void_p(self.prior.data_ptr())
        o.render_alpha, o.render_depth, o.render_rgb = (_f32(self.render_alpha), _f32(self.render_depth),
                                                        _f32(self.render_rgb))
        o.miss_alpha, o.miss_depth, o.miss_rgb = self.miss_alpha, self.miss_depth, self.miss_rgb
        return o


def _ptr(t, ctype):
    return None if t is None else C.cast(C.c_void_p(t.data_ptr()), ctype)


def seed_gaussians(ctx: Context, rgb, depth, cam, opts: SeedOpts | None = None, capacity: int | None = None,
                   params=None, diagnostics: bool = False, sync: bool = True) -> dict:
    """Seed gaussians from an RGB-D frame (rgb (3,H,W), depth (H,W) float32 device tensors).
    params: optional (14, >= capacity) block that receives the seeds as gaussians."""
    import torch
    o = opts or SeedOpts()
    H, W = int(cam.height), int(cam.width)
    cap = capacity if capacity is not None else (W * H) // (o.m * o.m) + W + H + 16
    dev = rgb.device
    tx, ty = (W + o.tile - 1) // o.tile, (H + o.tile - 1) // o.tile
    r = dict(pixel=torch.empty(cap, dtype=torch.int32, device=dev), is_high=torch.empty(cap, dtype=torch.uint8, device=dev),
             mean=torch.empty((3, cap), dtype=torch.float32, device=dev), radius=torch.empty(cap, dtype=torch.float32, device=dev),
             rgb=torch.empty((3, cap), dtype=torch.float32, device=dev),
             tile_count=torch.empty((ty, tx), dtype=torch.int32, device=dev),
             n_dev=torch.zeros(1, dtype=torch.int64, device=dev))
    if diagnostics:
        r.update(E=torch.empty((H, W), dtype=torch.float64, device=dev), hist=torch.empty(256, dtype=torch.int32, device=dev),
                 threshold=torch.empty(1, dtype=torch.int32, device=dev))
    out = CSeedOut()
    out.capacity = cap
    out.pixel, out.is_high = _ptr(r["pixel"], _i32p), _ptr(r["is_high"], C.POINTER(C.c_uint8))
    out.mean, out.radius, out.rgb = _f32(r["mean"]), _f32(r["radius"]), _f32(r["rgb"])
    out.tile_count, out.n_dev = _ptr(r["tile_count"], _i32p), _ptr(r["n_dev"], C.POINTER(C.c_int64))
    if params is not None:
        assert params.shape[1] >= cap
        out.params = gaussians(params, cap)
    if diagnostics:
        out.E, out.hist = _ptr(r["E"], C.POINTER(C.c_double)), _ptr(r["hist"], C.POINTER(C.c_uint32))
        out.threshold = _ptr(r["threshold"], _i32p)
    if o.use_prior:
        r["from_prior"] = torch.zeros(cap, dtype=torch.uint8, device=dev)
        out.from_prior = _ptr(r["from_prior"], C.POINTER(C.c_uint8))
    if diagnostics:
        r["missing"] = torch.empty((H, W), dtype=torch.uint8, device=dev)
        out.missing = _ptr(r["missing"], C.POINTER(C.c_uint8))
    n = C.c_int64(-1)
    _check(_lib.fgs_seed_gaussians(ctx.handle, _f32(rgb), _f32(depth), C.byref(camera(cam)), C.byref(o.c()),
                                   C.byref(out), C.byref(n) if sync else None), ctx.handle)
    r["n"] = n.value
    r["capacity"] = cap
    return r


# ------------------------------------- learned prior -------------------------------------

PRIOR_INPUTS, PRIOR_HIDDEN, PRIOR_OUTPUTS, PRIOR_PARAMS = 260, 256, 4, 133636


def tile_features(ctx: Context, rgb, depth, depth_min: float = 0.1, depth_max: float = 10.0, tile_ids=None):
    """Features of 16x16 tiles of a frame (rgb (3,H,W), depth (H,W)): ([T, 260] float32, [T] int32
    valid-depth counts). tile_ids: optional int32 device tensor of row-major tile indices."""
    import torch
    H, W = int(depth.shape[0]), int(depth.shape[1])
    T = int(tile_ids.numel()) if tile_ids is not None else ((W + 15) // 16) * ((H + 15) // 16)
    feat = torch.empty((T, PRIOR_INPUTS), dtype=torch.float32, device=depth.device)
    valid = torch.empty(T, dtype=torch.int32, device=depth.device)
    _check(_lib.fgs_tile_features(ctx.handle, _f32(rgb), _f32(depth), W, H, depth_min, depth_max, T,
                                  _ptr(tile_ids, C.POINTER(C.c_int32)), _f32(feat),
                                  _ptr(valid, C.POINTER(C.c_int32))), ctx.handle)
    return feat, valid


def prior_forward(ctx: Context, x, weights, y=None):
    """y [rows, 4] = network(x [rows, 260]) with packed FP32 weights (PRIOR_PARAMS)."""
    import torch
    rows = int(x.shape[0])
    if y is None:
        y = torch.empty((rows, PRIOR_OUTPUTS), dtype=torch.float32, device=x.device)
    _check(_lib.fgs_prior_forward(ctx.handle, rows, _f32(x), _f32(weights), _f32(y)), ctx.handle)
    return y


@dataclass
class PriorAdam:
    """Adam state of the prior's packed weights."""
    m: object
    v: object
    step: int = 0
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    @staticmethod
    def like(weights, **kw):
        import torch
        return PriorAdam(torch.zeros_like(weights), torch.zeros_like(weights), **kw)


def prior_train_step(ctx: Context, x, target, weights, adam: PriorAdam, loss=None, grad_out=None):
    """One Adam step of the network on the MSE against target [rows, 4] (weights updated in place)."""
    a = CPriorAdam(_f32(adam.m), _f32(adam.v), adam.step, adam.lr, adam.beta1, adam.beta2, adam.eps)
    _check(_lib.fgs_prior_train_step(ctx.handle, int(x.shape[0]), _f32(x), _f32(target), _f32(weights), C.byref(a),
                                     _f32(loss), _f32(grad_out)), ctx.handle)
    adam.step = a.step
