"""FP64 CPU oracle of the FGS mapping hot path (arXiv 2503.01109), as a ctypes binding.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU
baseline leg use it to check and time the HIP library. The product path never imports
it, and it shares no code with the HIP library.

Inputs are numpy arrays; gaussian parameters are the (14, N) SoA block described in
``synth``. Cameras are any object with width, height, fx, fy, cx, cy, R (3x3), t (3,),
z_near attributes.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("z_near", C.c_double)]


class _RenderOpts(C.Structure):
    _fields_ = [("sigma_cut", C.c_double), ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("T_min", C.c_double), ("lowpass", C.c_double), ("bg", C.c_double * 3),
                ("bg_depth", C.c_double)]


class _SeedOpts(C.Structure):
    _fields_ = [("D0", C.c_double), ("m", C.c_int32), ("n", C.c_int32), ("tile", C.c_int32),
                ("alpha_h", C.c_double), ("alpha_l", C.c_double), ("opacity_logit", C.c_double),
                ("depth_min", C.c_double), ("depth_max", C.c_double)]


class _Missing(C.Structure):
    _fields_ = [("alpha", _fp), ("depth", _fp), ("rgb", _fp), ("tau_alpha", C.c_float), ("tau_depth", C.c_float),
                ("tau_rgb", C.c_float)]


@dataclass
class MissingCheck:
    """The current map rendered at the frame's pose (binary32 planes: opacity (H, W), depth (H, W),
    rgb (3, H, W)) and the thresholds of the missing-region check (Sec. III-A, Eq. 9, 10)."""
    alpha: object
    depth: object
    rgb: object
    tau_alpha: float = 0.5
    tau_depth: float = 0.1
    tau_rgb: float = 0.3


@dataclass
class RenderOpts:
    """Cutoffs of the compositing (3-sigma, alpha >= 1/255, alpha <= 0.99, stop before T < 1e-4)."""
    sigma_cut: float = 3.0
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    lowpass: float = 0.3
    bg: tuple = (0.0, 0.0, 0.0)
    bg_depth: float = 0.0

    def c(self) -> _RenderOpts:
        o = _RenderOpts()
        o.sigma_cut, o.alpha_min, o.alpha_max = self.sigma_cut, self.alpha_min, self.alpha_max
        o.T_min, o.lowpass, o.bg_depth = self.T_min, self.lowpass, self.bg_depth
        o.bg[:] = [float(v) for v in self.bg]
        return o


@dataclass
class SeedOpts:
    """Fourier seeding constants: high-pass radius D0 (frequency samples), lattice strides m < n,
    tile edge for the per-tile count, Eq. 11 radius factors, initial opacity logit, depth range."""
    D0: float = 30.0
    m: int = 2
    n: int = 8
    tile: int = 16
    alpha_h: float = 1.0
    alpha_l: float = 4.0
    opacity_logit: float = 0.0
    depth_min: float = 0.1
    depth_max: float = 10.0

    def c(self) -> _SeedOpts:
        o = _SeedOpts()
        for k in ("D0", "m", "n", "tile", "alpha_h", "alpha_l", "opacity_logit", "depth_min", "depth_max"):
            setattr(o, k, getattr(self, k))
        return o


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.fgso_project.argtypes = [C.c_int64, _dp, C.POINTER(_Camera), C.POINTER(_RenderOpts), _dp]
        L.fgso_render_fwd.argtypes = [C.c_int64, _dp, C.POINTER(_Camera), C.POINTER(_RenderOpts), C.c_int,
                                      C.c_int64, _i64p, _dp, _dp, _dp, _dp, _i32p, _u8p, C.c_double, _dp]
        L.fgso_render_bwd.argtypes = [C.c_int64, _dp, C.POINTER(_Camera), C.POINTER(_RenderOpts), C.c_int,
                                      C.c_int64, _i64p, _dp, _dp, _dp, _dp, _dp, _dp]
        L.fgso_tile_counts.argtypes = [C.c_int64, _dp, C.POINTER(_Camera), C.POINTER(_RenderOpts), _i64p]
        L.fgso_count_duplicates.argtypes = [C.c_int64, _dp, C.POINTER(_Camera), C.POINTER(_RenderOpts),
                                            C.c_int32, C.c_int32]
        L.fgso_count_duplicates.restype = C.c_int64
        L.fgso_loss_l1.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp, _dp]
        L.fgso_adam.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_int64, _dp, C.c_double, C.c_double,
                                C.c_double]
        L.fgso_ssim.argtypes = [C.c_int32, C.c_int32, _dp, _dp, _dp, _dp, _dp]
        L.fgso_scale_reg.argtypes = [C.c_int64, _dp, _dp, _dp]
        L.fgso_prune_thresholds.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.fgso_prune_keep.argtypes = [C.c_int64, _dp, C.c_double, C.c_double, _u8p]
        L.fgso_prune_keep.restype = C.c_int64
        L.fgso_compact.argtypes = [C.c_int64, C.c_int32, _dp, _u8p, _dp, C.c_int64]
        L.fgso_compact.restype = C.c_int64
        L.fgso_frame_points.argtypes = [C.c_int32, C.c_int32, _fp, C.c_float, C.c_float, C.c_float, C.c_float, _fp,
                                        _fp, C.c_int32, C.c_float, C.c_float, C.c_int64, _fp]
        L.fgso_frame_points.restype = C.c_int64
        L.fgso_knn.argtypes = [C.c_int64, _fp, C.c_int32, _i32p, _fp]
        L.fgso_knn_some.argtypes = [C.c_int64, _fp, C.c_int32, C.c_int64, _i64p, _i32p, _fp]
        L.fgso_cloud_cov_some.argtypes = [C.c_int64, _fp, C.c_int32, C.c_double, C.c_int64, _i64p, _dp]
        L.fgso_gicp_corr_some.argtypes = [C.c_int64, _fp, C.c_int64, _fp, _dp, _dp, C.c_float, C.c_int64, _i64p,
                                          _i32p]
        L.fgso_sym3_eigen.argtypes = [_dp, _dp, _dp]
        L.fgso_cloud_cov.argtypes = [C.c_int64, _fp, C.c_int32, C.c_double, _dp]
        L.fgso_gicp_linearize.argtypes = [C.c_int64, _fp, _dp, C.c_int64, _fp, _dp, _dp, _dp, C.c_float, _dp, _dp,
                                          _dp, _i64p, _i32p]
        L.fgso_so3_exp.argtypes = [_dp, _dp]
        L.fgso_so3_exp.restype = None
        L.fgso_gicp_align.argtypes = [C.c_int64, _fp, _dp, C.c_int64, _fp, _dp, _dp, _dp, C.c_float, C.c_int32,
                                      C.c_double, C.c_double, _dp, _dp, _i32p, _i32p, _dp, _i64p]
        L.fgso_highpass.argtypes = [C.c_int32, C.c_int32, _fp, C.c_double, _dp, _i64p, _i32p, _dp]
        L.fgso_triangle.argtypes = [_i64p]
        L.fgso_triangle.restype = C.c_int32
        L.fgso_seed.argtypes = [C.c_int32, C.c_int32, _fp, _fp, _fp, _fp, C.c_float, C.c_float, C.c_float,
                                C.c_float, C.POINTER(_SeedOpts), C.c_int64, _i32p, _u8p, _fp, _fp, _fp,
                                _i32p, _i32p, _dp, C.POINTER(_Missing), _u8p]
        L.fgso_seed.restype = C.c_int64
        L.fgso_tile_features.argtypes = [C.c_int32, C.c_int32, _fp, _fp, C.c_int32, C.c_int32, C.c_double,
                                         C.c_double, _dp]
        L.fgso_mlp_fwd.argtypes = [C.c_int64, _dp, _dp, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.fgso_mlp_bwd.argtypes = [C.c_int64, _dp, _dp, C.c_int, _dp, _dp, _dp]
        _lib = L
    return _lib


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cam(cam) -> _Camera:
    c = _Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float64).reshape(9)]
    c.t[:] = [float(v) for v in np.asarray(cam.t, np.float64).reshape(3)]
    c.z_near = float(cam.z_near)
    return c


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments (status {rc})")


def project(params, cam, opts: RenderOpts | None = None) -> np.ndarray:
    """(N, 16) per-gaussian projection: valid, t(3), cov2(3), conic(3), mean2(2), depth, opacity, 0, 0."""
    p = _d(params)
    n = p.shape[1]
    out = np.zeros((n, 16))
    _check(lib().fgso_project(n, _ptr(p, _dp), C.byref(_cam(cam)), C.byref((opts or RenderOpts()).c()),
                              _ptr(out, _dp)), "project")
    return out


def render_fwd(params, cam, opts: RenderOpts | None = None, mode: int = 0, pix=None,
               amb_rel: float = 1e-5) -> dict:
    """Eq. 1 for every pixel (or for the pixel indices `pix`). mode 0: tile-bucketed, 1: brute force."""
    p = _d(params)
    n = p.shape[1]
    pixa = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    m = cam.width * cam.height if pixa is None else pixa.shape[0]
    rgb = np.zeros((3, m)); depth = np.zeros(m); alpha = np.zeros(m); T = np.zeros(m)
    nc = np.zeros(m, np.int32); amb = np.zeros(m, np.uint8); stats = np.zeros(4)
    rc = lib().fgso_render_fwd(n, _ptr(p, _dp), C.byref(_cam(cam)), C.byref((opts or RenderOpts()).c()),
                               mode, m, _ptr(pixa, _i64p), _ptr(rgb, _dp), _ptr(depth, _dp),
                               _ptr(alpha, _dp), _ptr(T, _dp), _ptr(nc, _i32p), _ptr(amb, _u8p),
                               float(amb_rel), _ptr(stats, _dp))
    _check(rc, "render_fwd")
    # amb: a cutoff decision within amb_rel of its threshold (the pixel's result may legitimately
    # differ in FP32); amb_tie: equal binary32 depths blended in index order (unambiguous)
    out = dict(rgb=rgb, depth=depth, alpha=alpha, T_final=T, n_contrib=nc, amb=(amb & 1).astype(bool),
               amb_cut=(amb & 1).astype(bool), amb_tie=(amb & 2).astype(bool),
               E_f=stats[0], E_c=stats[1], n_amb=int(stats[2]))
    if pixa is None:
        H, W = cam.height, cam.width
        for k in ("depth", "alpha", "T_final", "n_contrib", "amb", "amb_cut", "amb_tie"):
            out[k] = out[k].reshape(H, W)
        out["rgb"] = rgb.reshape(3, H, W)
    return out


def render_bwd(params, cam, g_rgb, g_depth, g_alpha=None, opts: RenderOpts | None = None,
               mode: int = 0, pix=None, mass: bool = False):
    """Analytic backward: returns (dL/dparams (14, N), dL/d2D (10, N)), and with mass=True also
    the absolute mass (14, N) of every gradient entry (the bound on its rounding error, see
    fgso.h)."""
    p = _d(params)
    n = p.shape[1]
    pixa = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    m = cam.width * cam.height if pixa is None else pixa.shape[0]
    gr = _d(np.reshape(g_rgb, (3, m))); gd = _d(np.reshape(g_depth, (m,)))
    ga = None if g_alpha is None else _d(np.reshape(g_alpha, (m,)))
    grad = np.zeros((14, n)); grad2d = np.zeros((10, n))
    ms = np.zeros((14, n)) if mass else None
    rc = lib().fgso_render_bwd(n, _ptr(p, _dp), C.byref(_cam(cam)), C.byref((opts or RenderOpts()).c()),
                               mode, m, _ptr(pixa, _i64p), _ptr(gr, _dp), _ptr(gd, _dp), _ptr(ga, _dp),
                               _ptr(grad, _dp), _ptr(grad2d, _dp), _ptr(ms, _dp))
    _check(rc, "render_bwd")
    return (grad, grad2d, ms) if mass else (grad, grad2d)


def tile_counts(params, cam, opts: RenderOpts | None = None) -> dict:
    """Work of the 16x16-tile formulation: K_c (tile, gaussian) pairs with a blended pixel, L_f and
    L_b list entries consumed by the forward and the backward before each tile terminates, K the
    list entries (the oracle's own box binning)."""
    p = _d(params)
    c = np.zeros(4, np.int64)
    _check(lib().fgso_tile_counts(p.shape[1], _ptr(p, _dp), C.byref(_cam(cam)), C.byref((opts or RenderOpts()).c()),
                                  _ptr(c, _i64p)), "tile_counts")
    return dict(K_c=int(c[0]), L_f=int(c[1]), L_b=int(c[2]), K=int(c[3]))


def count_duplicates(params, cam, tile_w=16, tile_h=16, opts: RenderOpts | None = None) -> int:
    p = _d(params)
    return int(lib().fgso_count_duplicates(p.shape[1], _ptr(p, _dp), C.byref(_cam(cam)),
                                           C.byref((opts or RenderOpts()).c()), tile_w, tile_h))


def loss_l1(rgb, depth, rgb_t, depth_t, lambda_rgb=1.0, lambda_depth=0.1):
    """Returns (loss, psnr, dL/drgb, dL/ddepth)."""
    r, d, rt, dt = _d(rgb).ravel(), _d(depth).ravel(), _d(rgb_t).ravel(), _d(depth_t).ravel()
    P = d.shape[0]
    gr = np.zeros_like(r); gd = np.zeros_like(d)
    L = C.c_double(); ps = C.c_double()
    _check(lib().fgso_loss_l1(P, _ptr(r, _dp), _ptr(d, _dp), _ptr(rt, _dp), _ptr(dt, _dp), lambda_rgb,
                              lambda_depth, _ptr(gr, _dp), _ptr(gd, _dp), C.byref(L), C.byref(ps)), "loss")
    return L.value, ps.value, gr.reshape(np.shape(rgb)), gd.reshape(np.shape(depth))


def ssim(img, tgt):
    """Structural similarity of img to tgt ((3, H, W) each) as in Eq. 16's SSIM term: returns
    (ssim, d ssim / d img (3, H, W), per-pixel index map (3, H, W))."""
    x, y = _d(img), _d(tgt)
    _, H, W = x.shape
    s = C.c_double()
    g = np.zeros_like(x)
    m = np.zeros_like(x)
    _check(lib().fgso_ssim(W, H, _ptr(x, _dp), _ptr(y, _dp), C.byref(s), _ptr(g, _dp), _ptr(m, _dp)), "ssim")
    return s.value, g, m


def scale_reg(log_scale):
    """Scale regulariser of Eq. 15 over the (3, n) log-scales: returns (value, d value / d log-scale)."""
    ls = _d(log_scale)
    v = C.c_double()
    g = np.zeros_like(ls)
    _check(lib().fgso_scale_reg(ls.shape[1], _ptr(ls, _dp), C.byref(v), _ptr(g, _dp)), "scale_reg")
    return v.value, g


def prune_thresholds(min_opacity, max_scale):
    """(L_o, L_s): the pruning thresholds of Sec. III-D carried onto the opacity logit and the
    log-scales, rounded to binary32 (-inf / +inf when a test is off)."""
    lo, ls = C.c_double(), C.c_double()
    _check(lib().fgso_prune_thresholds(float(min_opacity), float(max_scale), C.byref(lo), C.byref(ls)),
           "prune_thresholds")
    return lo.value, ls.value


def prune_keep(params, min_opacity, max_scale):
    """Keep mask (uint8, n) of the (14, n) block under the pruning test of Sec. III-D."""
    p = _d(params)
    n = p.shape[1]
    keep = np.zeros(n, np.uint8)
    k = lib().fgso_prune_keep(n, _ptr(p, _dp), float(min_opacity), float(max_scale), _ptr(keep, _u8p))
    _check(k, "prune_keep")
    return keep


def compact(block, keep):
    """Stable compaction of the (planes, n) block to its kept columns: (planes, kept)."""
    b = _d(block)
    planes, n = b.shape
    kp = np.ascontiguousarray(keep, np.uint8)
    kept = int(np.count_nonzero(kp))
    out = np.zeros((planes, max(kept, 1)))
    _check(lib().fgso_compact(n, planes, _ptr(b, _dp), _ptr(kp, _u8p), _ptr(out, _dp), out.shape[1]), "compact")
    return out[:, :kept]


def prune(params, min_opacity, max_scale, *companions):
    """Pruning of Sec. III-D: (kept params (14, k), keep mask, compacted companions (e.g. Adam
    moments of the same layout))."""
    keep = prune_keep(params, min_opacity, max_scale)
    return (compact(params, keep), keep) + tuple(compact(c, keep) for c in companions)


def _f32c(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def frame_points(depth, cam, stride=4, dmin=0.1, dmax=10.0, pose_wc=None):
    """Lattice points of a depth frame (Sec. III-B, uniform downsampling): (3, count) binary32 in
    the camera frame, or in the world with pose_wc = (R_wc (3x3), t_wc (3,))."""
    d = _f32c(depth)
    H, W = d.shape
    cap = ((W + stride - 1) // stride) * ((H + stride - 1) // stride)
    out = np.zeros((3, max(cap, 1)), np.float32)
    R = t = None
    if pose_wc is not None:
        R, t = _f32c(np.asarray(pose_wc[0]).reshape(9)), _f32c(np.asarray(pose_wc[1]).reshape(3))
    n = lib().fgso_frame_points(W, H, _ptr(d, _fp), float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy),
                                _ptr(R, _fp), _ptr(t, _fp), int(stride), float(dmin), float(dmax), out.shape[1],
                                _ptr(out, _fp))
    _check(n, "frame_points")
    return np.ascontiguousarray(out[:, :n])


def knn(xyz, k):
    """(idx (n, k) int32, d2 (n, k) binary32): the k nearest points of every point of the (3, n)
    binary32 cloud, itself included, in (distance, index) order."""
    p = _f32c(xyz)
    n = p.shape[1]
    idx = np.zeros((n, k), np.int32)
    d2 = np.zeros((n, k), np.float32)
    _check(lib().fgso_knn(n, _ptr(p, _fp), int(k), _ptr(idx, _i32p), _ptr(d2, _fp)), "knn")
    return idx, d2


def knn_some(xyz, k, q):
    """(idx (len(q), k), d2 (len(q), k)): knn() for the points q only."""
    p = _f32c(xyz)
    qq = np.ascontiguousarray(q, np.int64)
    idx = np.zeros((qq.size, k), np.int32)
    d2 = np.zeros((qq.size, k), np.float32)
    _check(lib().fgso_knn_some(p.shape[1], _ptr(p, _fp), int(k), qq.size, _ptr(qq, _i64p), _ptr(idx, _i32p),
                               _ptr(d2, _fp)), "knn_some")
    return idx, d2


def cloud_cov_some(xyz, q, k=20, eps=1e-3):
    """cloud_cov() for the points q only: (6, len(q))."""
    p = _f32c(xyz)
    qq = np.ascontiguousarray(q, np.int64)
    cov = np.zeros((6, max(qq.size, 1)))
    _check(lib().fgso_cloud_cov_some(p.shape[1], _ptr(p, _fp), int(k), float(eps), qq.size, _ptr(qq, _i64p),
                                     _ptr(cov, _dp)), "cloud_cov_some")
    return cov[:, :qq.size]


def gicp_corr_some(src, tgt, R, t, d_max, q):
    """Correspondences (target index or -1) of the source points q at the pose (R, t)."""
    s, tg = _f32c(src), _f32c(tgt)
    Rm, tv = _d(np.asarray(R).reshape(9)), _d(np.asarray(t).reshape(3))
    qq = np.ascontiguousarray(q, np.int64)
    out = np.zeros(max(qq.size, 1), np.int32)
    _check(lib().fgso_gicp_corr_some(s.shape[1], _ptr(s, _fp), tg.shape[1], _ptr(tg, _fp), _ptr(Rm, _dp),
                                     _ptr(tv, _dp), float(d_max), qq.size, _ptr(qq, _i64p), _ptr(out, _i32p)),
           "gicp_corr_some")
    return out[:qq.size]


def sym3_eigen(A6):
    """(evals (3,), evecs (3, 3) with eigenvector c in column c) of the symmetric matrix given by
    (xx, xy, xz, yy, yz, zz)."""
    a = _d(A6)
    ev = np.zeros(3)
    V = np.zeros(9)
    lib().fgso_sym3_eigen(_ptr(a, _dp), _ptr(ev, _dp), _ptr(V, _dp))
    return ev, V.reshape(3, 3).T.copy()


def cloud_cov(xyz, k=20, eps=1e-3):
    """Regularised local covariances (6, n) FP64 (xx, xy, xz, yy, yz, zz) of the (3, n) cloud."""
    p = _f32c(xyz)
    n = p.shape[1]
    cov = np.zeros((6, n))
    _check(lib().fgso_cloud_cov(n, _ptr(p, _fp), int(k), float(eps), _ptr(cov, _dp)), "cloud_cov")
    return cov


def gicp_linearize(src, src_cov, tgt, tgt_cov, R, t, d_max):
    """One linearisation of Eq. 14 at (R, t): dict(H (6, 6), b (6,), cost, count, corr (ns,))."""
    s, tg = _f32c(src), _f32c(tgt)
    sc, tc = _d(src_cov), _d(tgt_cov)
    Rm, tv = _d(np.asarray(R).reshape(9)), _d(np.asarray(t).reshape(3))
    H, b = np.zeros(36), np.zeros(6)
    cost, count = C.c_double(), C.c_int64()
    corr = np.zeros(max(s.shape[1], 1), np.int32)
    _check(lib().fgso_gicp_linearize(s.shape[1], _ptr(s, _fp), _ptr(sc, _dp), tg.shape[1], _ptr(tg, _fp),
                                     _ptr(tc, _dp), _ptr(Rm, _dp), _ptr(tv, _dp), float(d_max), _ptr(H, _dp),
                                     _ptr(b, _dp), C.byref(cost), C.byref(count), _ptr(corr, _i32p)), "gicp_linearize")
    return dict(H=H.reshape(6, 6), b=b, cost=cost.value, count=count.value, corr=corr[:s.shape[1]])


def so3_exp(w):
    w = _d(w)
    E = np.zeros(9)
    lib().fgso_so3_exp(_ptr(w, _dp), _ptr(E, _dp))
    return E.reshape(3, 3)


def gicp_align(src, src_cov, tgt, tgt_cov, R0, t0, d_max, max_iter=30, eps_rot=1e-6, eps_trans=1e-6):
    """Gauss-Newton alignment of Eq. 14: dict(R, t, iterations, status, cost, count)."""
    s, tg = _f32c(src), _f32c(tgt)
    sc, tc = _d(src_cov), _d(tgt_cov)
    R0m, t0v = _d(np.asarray(R0).reshape(9)), _d(np.asarray(t0).reshape(3))
    R, t = np.zeros(9), np.zeros(3)
    it, st = C.c_int32(), C.c_int32()
    cost, count = C.c_double(), C.c_int64()
    _check(lib().fgso_gicp_align(s.shape[1], _ptr(s, _fp), _ptr(sc, _dp), tg.shape[1], _ptr(tg, _fp),
                                 _ptr(tc, _dp), _ptr(R0m, _dp), _ptr(t0v, _dp), float(d_max), int(max_iter),
                                 float(eps_rot), float(eps_trans), _ptr(R, _dp), _ptr(t, _dp), C.byref(it),
                                 C.byref(st), C.byref(cost), C.byref(count)), "gicp_align")
    return dict(R=R.reshape(3, 3), t=t, iterations=it.value, status=st.value, cost=cost.value, count=count.value)


def adam(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam update; returns new (params, m, v) as float64 copies."""
    p, mm, vv, g = _d(params).copy(), _d(m).copy(), _d(v).copy(), _d(grad)
    lra = _d(lr)
    _check(lib().fgso_adam(p.shape[1], _ptr(p, _dp), _ptr(mm, _dp), _ptr(vv, _dp), _ptr(g, _dp), int(step),
                           _ptr(lra, _dp), beta1, beta2, eps), "adam")
    return p, mm, vv


def highpass(rgb, D0=30.0):
    """Returns (E (H, W), hist (256,), threshold, margin)."""
    r = np.ascontiguousarray(rgb, dtype=np.float32)
    _, H, W = r.shape
    E = np.zeros((H, W)); hist = np.zeros(256, np.int64); t = C.c_int32(); mg = C.c_double()
    _check(lib().fgso_highpass(W, H, _ptr(r, _fp), D0, _ptr(E, _dp), _ptr(hist, _i64p), C.byref(t),
                               C.byref(mg)), "highpass")
    return E, hist, t.value, mg.value


def triangle(hist) -> int:
    h = np.ascontiguousarray(hist, dtype=np.int64)
    assert h.shape == (256,)
    return int(lib().fgso_triangle(_ptr(h, _i64p)))


def seed(rgb, depth, cam, opts: SeedOpts | None = None, capacity: int | None = None,
         miss: MissingCheck | None = None) -> dict:
    """Fourier seeding of one RGB-D frame; float outputs are binary32. miss: the missing-region
    check against the current map (None: no map yet); the result's "missing" is M_m."""
    o = opts or SeedOpts()
    r = np.ascontiguousarray(rgb, dtype=np.float32)
    d = np.ascontiguousarray(depth, dtype=np.float32)
    _, H, W = r.shape
    cap = capacity if capacity is not None else (W * H) // (o.m * o.m) + W + H + 16
    pixel = np.zeros(cap, np.int32); hi = np.zeros(cap, np.uint8)
    mean = np.zeros((3, cap), np.float32); rad = np.zeros(cap, np.float32)
    srgb = np.zeros((3, cap), np.float32)
    tx, ty = (W + o.tile - 1) // o.tile, (H + o.tile - 1) // o.tile
    tc = np.zeros(tx * ty, np.int32)
    t = C.c_int32(); mg = C.c_double()
    R = np.ascontiguousarray(cam.R, np.float32).reshape(9)
    tt = np.ascontiguousarray(cam.t, np.float32).reshape(3)
    missing = np.zeros(H * W, np.uint8)
    cm = None
    if miss is not None:
        ma = np.ascontiguousarray(miss.alpha, np.float32).reshape(H * W)
        md = np.ascontiguousarray(miss.depth, np.float32).reshape(H * W)
        mr = np.ascontiguousarray(miss.rgb, np.float32).reshape(3 * H * W)
        cm = _Missing(_ptr(ma, _fp), _ptr(md, _fp), _ptr(mr, _fp), miss.tau_alpha, miss.tau_depth, miss.tau_rgb)
    n = lib().fgso_seed(W, H, _ptr(r, _fp), _ptr(d, _fp), _ptr(R, _fp), _ptr(tt, _fp), cam.fx, cam.fy, cam.cx,
                        cam.cy, C.byref(o.c()), cap, _ptr(pixel, _i32p), _ptr(hi, _u8p), _ptr(mean, _fp),
                        _ptr(rad, _fp), _ptr(srgb, _fp), _ptr(tc, _i32p), C.byref(t), C.byref(mg),
                        None if cm is None else C.byref(cm), _ptr(missing, _u8p))
    _check(n, "seed")
    k = min(n, cap)
    return dict(n=int(n), pixel=pixel[:k], is_high=hi[:k].astype(bool), mean=mean[:, :k], radius=rad[:k],
                rgb=srgb[:, :k], tile_count=tc.reshape(ty, tx), threshold=t.value, margin=mg.value,
                missing=missing.reshape(H, W).astype(bool))


def tile_features(rgb, depth, tx, ty, depth_min=0.1, depth_max=10.0):
    r = np.ascontiguousarray(rgb, dtype=np.float32)
    d = np.ascontiguousarray(depth, dtype=np.float32)
    _, H, W = r.shape
    f = np.zeros(260)
    nv = lib().fgso_tile_features(W, H, _ptr(r, _fp), _ptr(d, _fp), tx, ty, depth_min, depth_max, _ptr(f, _dp))
    _check(nv, "tile_features")
    return f, nv


MLP_PARAMS = 133636


def mlp_fwd(x, w, bf16=True):
    xx = _d(x)
    rows = xx.shape[0]
    y = np.zeros((rows, 4))
    _check(lib().fgso_mlp_fwd(rows, _ptr(xx, _dp), _ptr(_d(w), _dp), int(bf16), _ptr(y, _dp), None, None,
                              None, None), "mlp_fwd")
    return y


def mlp_bwd(x, w, target, bf16=True):
    """Gradient of the mean squared error w.r.t. the packed weights; returns (grad, loss)."""
    xx, ww, tt = _d(x), _d(w), _d(target)
    g = np.zeros(MLP_PARAMS); L = C.c_double()
    _check(lib().fgso_mlp_bwd(xx.shape[0], _ptr(xx, _dp), _ptr(ww, _dp), int(bf16), _ptr(tt, _dp),
                              _ptr(g, _dp), C.byref(L)), "mlp_bwd")
    return g, L.value
