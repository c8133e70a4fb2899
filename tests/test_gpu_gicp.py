"""GICP tracking (Sec. III-B, Eq. 12-14) on the GPU against the oracle: lattice points bit-exact;
neighbour lists exact and covariances within 1e-9 (FP64 on both sides, different summation and
rotation order); correspondences exact; one linearisation's H, b and cost within 1e-9 of their
largest entry; whole alignments to the same pose. Frames are ray-cast synthetic rooms (small
160x120 ones that the brute-force oracle handles whole, and the 640x480 tracking workload:
8 keyframes and the current frame at stride 4, checked on sampled points)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import dev, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fgs():
    need_gpu()
    import paper_2503_01109_amd as F
    return F


@pytest.fixture(scope="module")
def ctx(fgs):
    c = fgs.Context()
    yield c
    c.close()


def pose4(R, t):
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = R, t
    return T


def bits(a):
    return np.ascontiguousarray(np.asarray(a, np.float32)).view(np.uint32)


def frames(seed, w=160, h=120, f=131.25, n_key=3):
    room = synth.room_scene(seed)
    keys, cur = synth.tracking_cameras(seed, n_key=n_key, width=w, height=h, f=f)
    kd = [synth.room_depth(room, c, 100 + i) for i, c in enumerate(keys)]
    return keys, kd, cur, synth.room_depth(room, cur, 99)


def gpu_points(F, ctx, depth, cam, stride, world):
    pose = pose4(*synth.pose_wc(cam)) if world else None
    xyz, n = F.frame_points(ctx, dev(depth), cam, stride, pose_wc=pose)
    return xyz, n


def clouds(F, ctx, seed, stride=2, opts=None, **kw):
    """(GPU source, GPU target, oracle source points, oracle target points, keys, cur)."""
    keys, kd, cur, cd = frames(seed, **kw)
    parts, ref = [], []
    for c, d in zip(keys, kd):
        xyz, n = gpu_points(F, ctx, d, c, stride, True)
        parts.append(xyz[:, :n])
        ref.append(oracle.frame_points(d, c, stride, pose_wc=synth.pose_wc(c)))
    import torch
    tg = torch.cat(parts, 1).contiguous()
    sx, sn = gpu_points(F, ctx, cd, cur, stride, False)
    src_ref = oracle.frame_points(cd, cur, stride)
    o = opts or F.CloudOpts(cell=0.1, k=20, eps=1e-3, keep_knn=True)
    S, T = F.Cloud(ctx, sx, sn, o), F.Cloud(ctx, tg, None, o)
    return S, T, src_ref, np.concatenate(ref, 1), keys, cur


@pytest.mark.parametrize("w,h,stride,world", [(640, 480, 4, False), (640, 480, 3, True), (101, 77, 2, True)])
def test_frame_points_are_bit_exact(fgs, ctx, w, h, stride, world):
    keys, kd, cur, cd = frames(1, w=w, h=h, f=0.82 * w, n_key=1)
    cd[5, ::7] = np.nan
    cd[8, ::5] = 20.0
    cd[0, 0] = 0.05
    xyz, n = gpu_points(fgs, ctx, cd, cur, stride, world)
    ref = oracle.frame_points(cd, cur, stride, pose_wc=synth.pose_wc(cur) if world else None)
    assert n == ref.shape[1]
    assert np.array_equal(bits(host(xyz)[:, :n]), bits(ref))


def test_frame_points_report_a_full_output(fgs, ctx):
    import torch
    keys, kd, cur, cd = frames(2)
    out = torch.empty((3, 100), device="cuda")
    import ctypes as C
    n = C.c_int64(-1)
    st = fgs._lib.fgs_frame_points(ctx.handle, fgs._f32(dev(cd)), C.byref(fgs.camera(cur)), None, 2, 0.1, 10.0,
                                   fgs._f32(out), 100, None, C.byref(n))
    assert st == fgs.ERR_CAPACITY and n.value == oracle.frame_points(cd, cur, 2).shape[1]


def test_neighbours_and_covariances_match_oracle(fgs, ctx):
    S, T, src, tgt, _, _ = clouds(fgs, ctx, 3)
    for cl, pts in ((S, src), (T, tgt)):
        cov, knn = cl.read()
        idx, _ = oracle.knn(pts, 20)
        assert np.array_equal(host(knn), idx)
        ref = oracle.cloud_cov(pts, 20, 1e-3)
        err = np.abs(host(cov) - ref).max()
        print(f"cloud of {pts.shape[1]}: covariance max err {err:.2e}")
        assert err < 1e-9


def rings_cloud():
    g = np.random.default_rng(4)
    p = g.uniform(0, 1, (3, 3000)).astype(np.float32)
    p[:, 100:110] = p[:, 100:101]  # ten copies of one point
    p[:, 2990:] = g.uniform(3, 4, (3, 10)).astype(np.float32)
    return p


@pytest.mark.parametrize("cell,k", [(0.02, 20), (0.3, 3)])
def test_neighbours_across_several_rings_ties_and_outliers(fgs, ctx, cell, k):
    """A small cell (most neighbours lie beyond the first ring, and the isolated points beyond the
    four rings after which a point scans the whole cloud), duplicated points (ties broken by index)
    and isolated points far from the rest."""
    check_rings_cloud(fgs, ctx, cell, k)


@pytest.mark.skip(reason="k = 32 (no sentinel slot) faulted the GPU before the fix of the neighbour insertion, "
                         "which never wrote the front slot and left index 0xffffffff; not run on the GPU again yet")
def test_neighbours_with_the_largest_k(fgs, ctx):
    check_rings_cloud(fgs, ctx, 0.05, 32)


def check_rings_cloud(fgs, ctx, cell, k):
    p = rings_cloud()
    cl = fgs.Cloud(ctx, dev(p), None, fgs.CloudOpts(cell=cell, k=k, eps=1e-2, keep_knn=True))
    cov, knn = cl.read()
    idx, _ = oracle.knn(p, k)
    assert np.array_equal(host(knn), idx), (cell, k)
    ref = oracle.cloud_cov(p, k, 1e-2)
    assert np.abs(host(cov) - ref).max() < 1e-9, (cell, k)
    cl.close()


def test_cloud_rejects_non_finite_points(fgs, ctx):
    p = rings_cloud()[:, :500].copy()
    for bad in (np.nan, np.inf):
        q = p.copy()
        q[1, 17] = bad
        with pytest.raises(fgs.FgsError) as ei:
            fgs.Cloud(ctx, dev(q), None, fgs.CloudOpts(cell=0.1, k=10))
        assert ei.value.status == fgs.ERR_INVALID_ARG and "non-finite" in str(ei.value)


def test_cloud_of_exactly_k_points(fgs, ctx):
    """n = k: every point's neighbours are the whole cloud, in (distance, index) order."""
    p = rings_cloud()[:, :16].copy()
    cl = fgs.Cloud(ctx, dev(p), None, fgs.CloudOpts(cell=0.05, k=16, eps=1e-3, keep_knn=True))
    cov, knn = cl.read()
    idx, _ = oracle.knn(p, 16)
    assert np.array_equal(host(knn), idx)
    assert np.abs(host(cov) - oracle.cloud_cov(p, 16, 1e-3)).max() < 1e-9
    cl.close()


def test_linearisation_matches_oracle(fgs, ctx):
    S, T, src, tgt, keys, _ = clouds(fgs, ctx, 5)
    R0, t0 = synth.pose_wc(keys[0])
    out, corr = fgs.gicp_linearize(ctx, S, T, pose4(R0, t0), 0.1)
    sc, tc = oracle.cloud_cov(src, 20, 1e-3), oracle.cloud_cov(tgt, 20, 1e-3)
    ref = oracle.gicp_linearize(src, sc, tgt, tc, R0, t0, 0.1)
    assert np.array_equal(host(corr), ref["corr"])
    o = host(out)
    H = np.zeros((6, 6))
    H[np.triu_indices(6)] = o[:21]
    H = H + np.triu(H, 1).T
    assert int(o[28]) == ref["count"] > 1000
    for got, want, what in ((H, ref["H"], "H"), (o[21:27], ref["b"], "b"), (o[27], ref["cost"], "cost")):
        e = np.abs(got - want).max() / np.abs(want).max()
        print(f"{what}: rel err {e:.2e}")
        assert e < 1e-9, what


def test_alignment_matches_oracle(fgs, ctx):
    """Eight Gauss-Newton updates with convergence switched off, then the default run to convergence."""
    S, T, src, tgt, keys, cur = clouds(fgs, ctx, 6)
    sc, tc = oracle.cloud_cov(src, 20, 1e-3), oracle.cloud_cov(tgt, 20, 1e-3)
    R0, t0 = synth.pose_wc(keys[0])
    for eps, it in ((0.0, 8), (1e-6, 30)):
        r = fgs.gicp_align(ctx, S, T, pose4(R0, t0), fgs.GicpOpts(0.1, it, eps, eps))
        ref = oracle.gicp_align(src, sc, tgt, tc, R0, t0, 0.1, it, eps, eps)
        dR, dt = np.abs(r["T"][:3, :3] - ref["R"]).max(), np.abs(r["T"][:3, 3] - ref["t"]).max()
        print(f"eps {eps}: {r['iterations']} vs {ref['iterations']} iterations, dR {dR:.2e}, dt {dt:.2e}")
        assert (r["iterations"], r["status"], r["correspondences"]) == (ref["iterations"], ref["status"], ref["count"])
        assert dR < 1e-9 and dt < 1e-9
        assert r["cost"] == pytest.approx(ref["cost"], rel=1e-9)
    R1, t1 = synth.pose_wc(cur)
    assert np.linalg.norm(r["T"][:3, 3] - t1) < 0.005


def test_alignment_without_correspondences_keeps_the_pose(fgs, ctx):
    S, T, _, _, keys, _ = clouds(fgs, ctx, 7)
    R0, t0 = synth.pose_wc(keys[0])
    T0 = pose4(R0, t0 + 5.0)
    r = fgs.gicp_align(ctx, S, T, T0, fgs.GicpOpts(0.05, 10))
    assert r["status"] == 2 and r["iterations"] == 0 and r["correspondences"] < 6
    assert np.array_equal(r["T"], T0)


def test_tracking_workload_on_sampled_points(fgs, ctx):
    """The benchmark's tracking workload: 8 keyframes and the current frame, 640x480 at stride 4.
    Neighbours and covariances of 300 sampled target points, correspondences of 500 sampled source
    points at the initial pose, against the oracle computing just those; then the alignment, which
    must land within 5 mm and 0.05 degrees of the true pose."""
    S, T, src, tgt, keys, cur = clouds(fgs, ctx, 8, stride=4, w=640, h=480, f=525.0, n_key=8)
    print(f"source {src.shape[1]} points, target {tgt.shape[1]}")
    g = np.random.default_rng(9)
    q = np.sort(g.choice(tgt.shape[1], 300, replace=False))
    cov, knn = T.read()
    idx, _ = oracle.knn_some(tgt, 20, q)
    assert np.array_equal(host(knn)[q], idx)
    assert np.abs(host(cov)[:, q] - oracle.cloud_cov_some(tgt, q, 20, 1e-3)).max() < 1e-9
    R0, t0 = synth.pose_wc(keys[0])
    _, corr = fgs.gicp_linearize(ctx, S, T, pose4(R0, t0), 0.1)
    qs = np.sort(g.choice(src.shape[1], 500, replace=False))
    assert np.array_equal(host(corr)[qs], oracle.gicp_corr_some(src, tgt, R0, t0, 0.1, qs))
    r = fgs.gicp_align(ctx, S, T, pose4(R0, t0), fgs.GicpOpts(0.1, 30, 1e-6, 1e-6))
    R1, t1 = synth.pose_wc(cur)
    ang = np.degrees(np.arccos(np.clip((np.trace(r["T"][:3, :3].T @ R1) - 1) / 2, -1, 1)))
    dt = np.linalg.norm(r["T"][:3, 3] - t1)
    print(f"tracking: status {r['status']}, {r['iterations']} iterations, {r['correspondences']} pairs, "
          f"error {ang:.4f} deg, {dt * 1e3:.2f} mm")
    assert r["status"] == 0 and ang < 0.05 and dt < 0.005
