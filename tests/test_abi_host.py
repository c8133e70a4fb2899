"""Host-side tests of the C ABI (no GPU needed): exported symbols, struct layouts, argument checks."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2503_01109_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names.update(re.findall(r"\b(fgs_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(F.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", F.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fgs_\w+)", out))
    assert set(names) <= exported
    assert set(F.EXPORTED) <= exported


LAYOUT_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "fgs.h"
#include "fgs_prior.h"
#include "fgs_gicp.h"
#define S(T) printf(#T " %zu\n", sizeof(T));
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  S(fgs_camera) O(fgs_camera, R_cw) O(fgs_camera, z_near)
  S(fgs_gaussians) O(fgs_gaussians, rgb)
  S(fgs_render_opts) O(fgs_render_opts, bg) O(fgs_render_opts, tile_h)
  S(fgs_image) S(fgs_adam) O(fgs_adam, step) O(fgs_adam, lr) O(fgs_adam, eps)
  S(fgs_target) S(fgs_loss_opts) S(fgs_prune_opts) O(fgs_prune_opts, max_scale)
  S(fgs_cloud_opts) O(fgs_cloud_opts, eps) O(fgs_cloud_opts, keep_knn)
  S(fgs_gicp_opts) O(fgs_gicp_opts, eps_rot) S(fgs_gicp_result) O(fgs_gicp_result, status) O(fgs_gicp_result, cost)
  S(fgs_prior_adam) O(fgs_prior_adam, step) O(fgs_prior_adam, eps)
  %EXTRA%
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    extra = ""
    if hasattr(F, "CSeedOpts"):
        extra = ("S(fgs_seed_opts) O(fgs_seed_opts, use_prior) O(fgs_seed_opts, render_rgb) O(fgs_seed_opts, miss_rgb) "
                 "S(fgs_seed_out) O(fgs_seed_out, tile_count) O(fgs_seed_out, from_prior) O(fgs_seed_out, missing)")
    src = tmp_path / "probe.c"
    src.write_text(LAYOUT_PROBE.replace("%EXTRA%", extra))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                             check=True).stdout.splitlines())
    mine = {
        "fgs_camera": C.sizeof(F.CCamera), "fgs_camera.R_cw": F.CCamera.R_cw.offset,
        "fgs_camera.z_near": F.CCamera.z_near.offset,
        "fgs_gaussians": C.sizeof(F.CGaussians), "fgs_gaussians.rgb": F.CGaussians.rgb.offset,
        "fgs_render_opts": C.sizeof(F.CRenderOpts), "fgs_render_opts.bg": F.CRenderOpts.bg.offset,
        "fgs_render_opts.tile_h": F.CRenderOpts.tile_h.offset,
        "fgs_image": C.sizeof(F.CImage), "fgs_adam": C.sizeof(F.CAdam), "fgs_adam.step": F.CAdam.step.offset,
        "fgs_adam.lr": F.CAdam.lr.offset, "fgs_adam.eps": F.CAdam.eps.offset,
        "fgs_target": C.sizeof(F.CTarget), "fgs_loss_opts": C.sizeof(F.CLossOpts),
        "fgs_prune_opts": C.sizeof(F.CPruneOpts), "fgs_prune_opts.max_scale": F.CPruneOpts.max_scale.offset,
        "fgs_cloud_opts": C.sizeof(F.CCloudOpts), "fgs_cloud_opts.eps": F.CCloudOpts.eps.offset,
        "fgs_cloud_opts.keep_knn": F.CCloudOpts.keep_knn.offset, "fgs_gicp_opts": C.sizeof(F.CGicpOpts),
        "fgs_gicp_opts.eps_rot": F.CGicpOpts.eps_rot.offset, "fgs_gicp_result": C.sizeof(F.CGicpResult),
        "fgs_gicp_result.status": F.CGicpResult.status.offset, "fgs_gicp_result.cost": F.CGicpResult.cost.offset,
        "fgs_prior_adam": C.sizeof(F.CPriorAdam), "fgs_prior_adam.step": F.CPriorAdam.step.offset,
        "fgs_prior_adam.eps": F.CPriorAdam.eps.offset,
    }
    if extra:
        mine.update({"fgs_seed_opts": C.sizeof(F.CSeedOpts), "fgs_seed_opts.use_prior": F.CSeedOpts.use_prior.offset,
                     "fgs_seed_opts.render_rgb": F.CSeedOpts.render_rgb.offset,
                     "fgs_seed_opts.miss_rgb": F.CSeedOpts.miss_rgb.offset,
                     "fgs_seed_out": C.sizeof(F.CSeedOut), "fgs_seed_out.tile_count": F.CSeedOut.tile_count.offset,
                     "fgs_seed_out.from_prior": F.CSeedOut.from_prior.offset,
                     "fgs_seed_out.missing": F.CSeedOut.missing.offset})
    for k, v in mine.items():
        assert int(got[k]) == v, f"{k}: header {got[k]} vs binding {v}"


def test_state_bytes_layout_and_errors():
    o = F.RenderOpts()
    b0 = F.state_bytes(100, 64, 48, 0, o)
    b1 = F.state_bytes(100, 64, 48, 1000, o)
    assert b1 - b0 == 4000
    assert b0 >= 100 * 48 + 12 * 8 + 64 * 48 * 8  # records, tile ranges, per-pixel words
    with pytest.raises(F.FgsError) as e:
        F.state_bytes(100, 0, 48, 10, o)
    assert e.value.status == F.ERR_INVALID_ARG
    with pytest.raises(F.FgsError) as e:
        F.state_bytes(100, 64, 48, 10, F.RenderOpts(tile_w=12, tile_h=12))
    assert "unsupported tile" in str(e.value)
    with pytest.raises(F.FgsError):
        F.state_bytes(100, 64, 48, 10, F.RenderOpts(alpha_max=1.5))


def _cam(**kw):
    import synth
    c = synth.camera_small()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _call_fwd(n=10, cam=None, opts=None, state_bytes=1 << 20, null_rgb=False, stride=None):
    g = F.CGaussians()
    g.n, g.stride = n, n if stride is None else stride
    dummy = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_float))
    g.mean = g.log_scale = g.quat = g.opacity_logit = g.rgb = dummy
    img = F.CImage(None if null_rgb else dummy, dummy, None, None, None)
    cc = F.camera(cam or _cam())
    st = F._lib.fgs_render_fwd(None, C.byref(g), C.byref(cc), C.byref((opts or F.RenderOpts()).c()), C.byref(img),
                               C.c_void_p(0x2000), state_bytes)
    return st, F.last_error()


def test_render_fwd_rejects_bad_arguments_on_host():
    assert _call_fwd() == (F.ERR_INVALID_ARG, "fgs_render_fwd: ctx is NULL")
    st, msg = _call_fwd(n=-1)
    assert st == F.ERR_INVALID_ARG and "g.n" in msg
    st, msg = _call_fwd(stride=5)
    assert st == F.ERR_INVALID_ARG and "stride" in msg
    st, msg = _call_fwd(cam=_cam(fx=-1.0))
    assert st == F.ERR_INVALID_ARG and "focal" in msg
    st, msg = _call_fwd(cam=_cam(width=0))
    assert st == F.ERR_INVALID_ARG and "image size" in msg
    st, msg = _call_fwd(opts=F.RenderOpts(sigma_cut=0.0))
    assert st == F.ERR_INVALID_ARG and "sigma_cut" in msg
    st, msg = _call_fwd(null_rgb=True)
    assert st == F.ERR_INVALID_ARG and "image" in msg
    st, msg = _call_fwd(state_bytes=100)
    assert st == F.ERR_CAPACITY and "fixed part" in msg
    import numpy as np
    st, msg = _call_fwd(cam=_cam(t=np.array([np.nan, 0, 0], np.float32)))
    assert st == F.ERR_INVALID_ARG and "t_cw" in msg


def test_status_strings():
    for s in (F.OK, F.ERR_INVALID_ARG, F.ERR_CAPACITY, F.ERR_HIP, F.ERR_UNSUPPORTED):
        assert F._lib.fgs_status_str(s)


def test_seed_rejects_bad_arguments_on_host():
    import numpy as np
    o = F.SeedOpts()
    out = F.CSeedOut()
    out.capacity = 10
    dummy = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_float))

    def call(cam, opts=o, capacity=10):
        out.capacity = capacity
        out.pixel = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_int32))
        out.is_high = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_uint8))
        out.mean = out.radius = out.rgb = dummy
        st = F._lib.fgs_seed_gaussians(None, dummy, dummy, C.byref(F.camera(cam)), C.byref(opts.c()), C.byref(out),
                                       None)
        return st, F.last_error()

    import synth
    assert call(synth.camera_tum()) == (F.ERR_INVALID_ARG, "fgs_seed_gaussians: ctx is NULL")
    st, msg = call(synth.centred_camera(74, 48, 60.0))  # 74 = 2 * 37
    assert st == F.ERR_UNSUPPORTED and "prime factors" in msg
    st, msg = call(synth.centred_camera(2048, 64, 60.0))
    assert st == F.ERR_UNSUPPORTED
    st, msg = call(synth.camera_tum(), F.SeedOpts(D0=0.0))
    assert st == F.ERR_INVALID_ARG and "D0" in msg
    st, msg = call(synth.camera_tum(), F.SeedOpts(m=0))
    assert st == F.ERR_INVALID_ARG
    st, msg = call(synth.camera_tum(), capacity=-1)
    assert st == F.ERR_INVALID_ARG and "output" in msg


def test_window_rejects_bad_arguments_on_host():
    import synth
    cams = [synth.camera_small(), synth.camera_tum()]

    def call(cams, tiles=None, blocks=0):
        V = len(cams)
        cc = (F.CCamera * max(V, 1))(*[F.camera(c) for c in cams])
        ct = None if tiles is None else (C.c_int32 * (2 * V))(*[x for t in tiles for x in t])
        p = C.c_void_p()
        st = F._lib.fgs_window_create(None, V, cc, ct, blocks, C.byref(p))
        return st, F.last_error()

    assert call(cams) == (F.ERR_INVALID_ARG, "fgs_window_create: ctx is NULL")
    st, msg = call([])
    assert st == F.ERR_INVALID_ARG and "n_views" in msg
    st, msg = call(cams, tiles=[(16, 16), (12, 12)])
    assert st == F.ERR_INVALID_ARG and "view 1" in msg and "12x12" in msg
    st, msg = call(cams, tiles=[(16, 16), (32, 16)])
    assert st == F.ERR_INVALID_ARG
    st, msg = call(cams, blocks=17)
    assert st == F.ERR_INVALID_ARG and "blocks_per_cu" in msg
    st, msg = call([cams[0], _cam(fx=0.0)])
    assert st == F.ERR_INVALID_ARG and "focal" in msg
    st = F._lib.fgs_window_step(None, None, None, None, None, None, None, None, None, 1)
    assert st == F.ERR_INVALID_ARG and "window is NULL" in F.last_error()


def test_prior_rejects_bad_arguments_on_host():
    d = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_float))
    assert F._lib.fgs_prior_forward(None, 10, d, d, d) == F.ERR_INVALID_ARG
    assert "ctx is NULL" in F.last_error()
    assert F._lib.fgs_prior_forward(None, -1, d, d, d) == F.ERR_INVALID_ARG
    assert "rows" in F.last_error()
    assert F._lib.fgs_prior_forward(None, 5, None, d, d) == F.ERR_INVALID_ARG
    a = F.CPriorAdam(d, d, 0, 1e-3, 0.9, 0.999, 1e-8)
    assert F._lib.fgs_prior_train_step(None, 0, d, d, d, C.byref(a), None, None) == F.ERR_INVALID_ARG
    bad = F.CPriorAdam(d, d, 0, 1e-3, 1.5, 0.999, 1e-8)
    assert F._lib.fgs_prior_train_step(None, 4, d, d, d, C.byref(bad), None, None) == F.ERR_INVALID_ARG
    assert "hyper" in F.last_error()
    assert F._lib.fgs_tile_features(None, d, d, 64, 48, 0.1, 10.0, 13, None, d, None) == F.ERR_INVALID_ARG
    assert "more tiles" in F.last_error()
    assert F._lib.fgs_tile_features(None, d, d, 0, 48, 0.1, 10.0, 1, None, d, None) == F.ERR_INVALID_ARG
    assert F._lib.fgs_tile_features(None, d, d, 64, 48, 0.1, 10.0, 12, None, d, None) == F.ERR_INVALID_ARG
    assert "ctx is NULL" in F.last_error()


def test_noalloc_backward_rejects_more_gaussians_than_its_scratch_on_host():
    g = F.CGaussians()
    g.n = g.stride = F.NOALLOC_MAX_GAUSSIANS + 1
    d = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_float))
    g.mean = g.log_scale = g.quat = g.opacity_logit = g.rgb = d
    st = F._lib.fgs_render_bwd_noalloc(None, C.byref(g), C.byref(F.camera(_cam())), C.byref(F.RenderOpts().c()),
                                      C.c_void_p(0x2000), 1 << 30, d, d, None, C.byref(g))
    assert st == F.ERR_CAPACITY and "static scratch" in F.last_error()
    g.n = g.stride = 10
    st = F._lib.fgs_render_bwd_noalloc(None, C.byref(g), C.byref(F.camera(_cam())), C.byref(F.RenderOpts().c()),
                                      C.c_void_p(0x2000), 1 << 30, d, d, None, C.byref(g))
    assert st == F.ERR_INVALID_ARG and "ctx is NULL" in F.last_error()


def test_prune_rejects_bad_arguments_on_host():
    def block(base, n, stride):
        g = F.CGaussians()
        g.n, g.stride = n, stride
        f = lambda k: C.cast(C.c_void_p(base + 4 * k * stride), C.POINTER(C.c_float))
        g.mean, g.log_scale, g.quat, g.opacity_logit, g.rgb = f(0), f(3), f(6), f(10), f(11)
        return g

    def call(opts, src, dst, n_sets=None):
        k = len(src) if n_sets is None else n_sets
        a = (F.CGaussians * max(len(src), 1))(*src)
        b = (F.CGaussians * max(len(dst), 1))(*dst)
        st = F._lib.fgs_prune(None, C.byref(opts), k, a, b, None, None, None)
        return st, F.last_error()

    ok = F.CPruneOpts(0.005, 0.5)
    A, B, M, Mo = 0x100000, 0x200000, 0x300000, 0x400000
    n = 1000
    assert call(ok, [block(A, n, n)], [block(B, n, n)]) == (F.ERR_INVALID_ARG, "fgs_prune: ctx is NULL")
    for bad in (F.CPruneOpts(1.0, 0.5), F.CPruneOpts(-0.1, 0.5), F.CPruneOpts(float("nan"), 0.5)):
        st, msg = call(bad, [block(A, n, n)], [block(B, n, n)])
        assert st == F.ERR_INVALID_ARG and "min_opacity" in msg
    st, msg = call(F.CPruneOpts(0.005, float("nan")), [block(A, n, n)], [block(B, n, n)])
    assert st == F.ERR_INVALID_ARG and "max_scale" in msg
    assert call(ok, [block(A, n, n)], [block(B, n, n)], n_sets=0)[0] == F.ERR_INVALID_ARG
    assert call(ok, [block(A, n, n)] * 5, [block(B, n, n)] * 5)[0] == F.ERR_INVALID_ARG
    st, msg = call(ok, [block(A, n, n)], [block(B, n, n - 1)])
    assert st == F.ERR_INVALID_ARG and "stride" in msg
    st, msg = call(ok, [block(A, n, n), block(M, n - 1, n)], [block(B, n, n), block(Mo, n, n)])
    assert st == F.ERR_INVALID_ARG and "src[1].n" in msg
    # a destination overlapping a source, or another destination
    st, msg = call(ok, [block(A, n, n)], [block(A + 4 * 13 * n, n, n)])
    assert st == F.ERR_INVALID_ARG and "overlaps src[0]" in msg
    st, msg = call(ok, [block(A, n, n), block(M, n, n)], [block(B, n, n), block(B + 8, n, n)])
    assert st == F.ERR_INVALID_ARG and "overlaps dst" in msg
    # disjoint blocks pass every check before the context's
    assert call(ok, [block(A, n, n), block(M, n, n)], [block(B, n, n), block(Mo, n, n)]) == (
        F.ERR_INVALID_ARG, "fgs_prune: ctx is NULL")


def test_tracking_calls_reject_bad_arguments_on_host():
    d = C.cast(C.c_void_p(0x1000), C.POINTER(C.c_float))
    cam = F.camera(_cam())
    n = C.c_int64(0)
    assert F._lib.fgs_frame_points(None, d, C.byref(cam), None, 0, 0.1, 10.0, d, 10, None, None) == F.ERR_INVALID_ARG
    assert "stride" in F.last_error()
    assert F._lib.fgs_frame_points(None, d, C.byref(cam), None, 2, float("nan"), 10.0, d, 10, None, None) == \
        F.ERR_INVALID_ARG
    bad_pose = (C.c_double * 16)(*([float("nan")] + [0.0] * 15))
    assert F._lib.fgs_frame_points(None, d, C.byref(cam), bad_pose, 2, 0.1, 10.0, d, 10, None, None) == \
        F.ERR_INVALID_ARG and "pose" in F.last_error()
    assert F._lib.fgs_frame_points(None, d, C.byref(cam), None, 2, 0.1, 10.0, d, 10, None, C.byref(n)) == \
        F.ERR_INVALID_ARG and "ctx is NULL" in F.last_error()
    h = C.c_void_p()

    def create(n, stride, opts):
        st = F._lib.fgs_cloud_create(None, n, stride, d, C.byref(opts), C.byref(h))
        return st, F.last_error()

    ok = F.CCloudOpts(0.1, 20, 1e-3, 0)
    assert create(100, 100, ok) == (F.ERR_INVALID_ARG, "fgs_cloud_create: ctx is NULL")
    assert "k must be" in create(100, 100, F.CCloudOpts(0.1, 40, 1e-3, 0))[1]
    assert "k must be" in create(100, 100, F.CCloudOpts(0.1, 2, 1e-3, 0))[1]
    assert "outside [k" in create(10, 10, ok)[1]
    assert "stride" in create(100, 50, ok)[1]
    assert "cell" in create(100, 100, F.CCloudOpts(0.0, 20, 1e-3, 0))[1]
    assert "eps" in create(100, 100, F.CCloudOpts(0.1, 20, 0.0, 0))[1]
    T = (C.c_double * 16)(*np.eye(4).reshape(16))
    r = F.CGicpResult()
    assert F._lib.fgs_gicp_align(None, None, None, T, C.byref(F.CGicpOpts(0.1, 0, 1e-6, 1e-6)), C.byref(r)) == \
        F.ERR_INVALID_ARG and "max_iter" in F.last_error()
    assert F._lib.fgs_gicp_align(None, None, None, T, C.byref(F.CGicpOpts(0.1, 10, 1e-6, 1e-6)), C.byref(r)) == \
        F.ERR_INVALID_ARG and "ctx is NULL" in F.last_error()
    out = C.cast(C.c_void_p(0x2000), C.POINTER(C.c_double))
    assert F._lib.fgs_gicp_linearize(None, None, None, T, 0.1, out, None) == F.ERR_INVALID_ARG
    assert F._lib.fgs_cloud_read(None, None, None, None, None) == F.ERR_INVALID_ARG
    assert F._lib.fgs_cloud_destroy(None) == F.OK
