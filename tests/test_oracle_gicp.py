"""Pins of the oracle's GICP tracking (Sec. III-B, Eq. 12-14) against facts that do not come from
the oracle itself: scipy's k-d tree for the neighbours, numpy's symmetric eigensolver, the exact
covariance of points on a plane, re-projection of the lattice points, scipy's rotation vectors for
Exp, central differences of the fixed-weight cost for b and of the residuals for H, and recovery of
a known rigid motion."""
import numpy as np
import pytest

import oracle
import synth


def cloud(n, seed):
    g = np.random.default_rng(seed)
    return g.uniform(0.0, 1.0, (3, n)).astype(np.float32)


def test_knn_matches_a_kd_tree():
    spatial = pytest.importorskip("scipy.spatial")
    n, k = 3000, 20
    p = cloud(n, 1)
    idx, d2 = oracle.knn(p, k)
    x = p.T.astype(np.float64)
    dd, ii = spatial.cKDTree(x).query(x, k + 1)
    # compare where the k-th and (k+1)-th distances are clearly apart (binary32 vs FP64 order)
    clear = dd[:, k] - dd[:, k - 1] > 1e-5 * dd[:, k]
    assert clear.mean() > 0.95
    for i in np.flatnonzero(clear):
        assert set(idx[i]) == set(ii[i, :k]), i
    np.testing.assert_allclose(np.sqrt(d2[clear]), np.sort(dd[clear, :k], axis=1), rtol=1e-6, atol=1e-7)
    assert (idx[:, 0] == np.arange(n)).all() and (d2[:, 0] == 0).all()


def test_knn_ties_go_by_index():
    """Five copies of one point and three other points: every copy's neighbours are the copies in
    index order, then the others by distance."""
    p = np.zeros((3, 8), np.float32)
    p[:, [1, 3, 4, 6, 7]] = 0.5
    p[:, 0], p[:, 2], p[:, 5] = [0.6, 0.5, 0.5], [0.5, 0.8, 0.5], [0.5, 0.5, 0.2]
    idx, d2 = oracle.knn(p, 7)
    for i in (1, 3, 4, 6, 7):
        assert idx[i].tolist() == [1, 3, 4, 6, 7, 0, 2]


def test_symmetric_eigen_matches_numpy():
    g = np.random.default_rng(2)
    for _ in range(200):
        A = g.normal(size=(3, 3))
        A = A @ A.T if g.uniform() < 0.5 else A + A.T
        a6 = [A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]]
        ev, V = oracle.sym3_eigen(a6)
        np.testing.assert_allclose(np.sort(ev), np.linalg.eigvalsh(A), atol=1e-12 * np.abs(A).max())
        np.testing.assert_allclose(A @ V - V * ev, 0.0, atol=1e-12 * np.abs(A).max())
        np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-13)


def test_covariance_of_points_on_a_plane_is_the_plane_metric():
    """Points spread on a plane with unit normal n: the regularised covariance is I - (1 - eps) n n^T
    (eigenvalues 1, 1, eps with n the last), at every point."""
    g = np.random.default_rng(3)
    nrm = g.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    u = np.cross(nrm, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    v = np.cross(nrm, u)
    ab = g.uniform(-1, 1, (2, 600))
    p = (np.outer(u, ab[0]) + np.outer(v, ab[1]) + 0.3 * nrm[:, None]).astype(np.float32)
    eps = 1e-3
    cov = oracle.cloud_cov(p, 20, eps)
    want = np.eye(3) - (1 - eps) * np.outer(nrm, nrm)
    w6 = np.array([want[0, 0], want[0, 1], want[0, 2], want[1, 1], want[1, 2], want[2, 2]])
    # the binary32 points lie within 1e-7 of the plane: the normal is off by about 1e-6
    np.testing.assert_allclose(cov, np.repeat(w6[:, None], p.shape[1], 1), atol=2e-5)


def test_frame_points_reproject_to_their_pixels():
    room = synth.room_scene(4)
    cam = synth.Camera(160, 120, 131.25, 131.25, 80.0, 60.0)
    keys, cur = synth.tracking_cameras(4, n_key=1, width=160, height=120, f=131.25)
    d = synth.room_depth(room, cur, 5)
    d[7, 8] = np.nan
    d[10, 20] = 50.0
    s = 4
    pts = oracle.frame_points(d, cur, stride=s, dmin=0.1, dmax=10.0)
    ys, xs = np.mgrid[0:120:s, 0:160:s]
    dl = d[ys, xs]
    ok = np.isfinite(dl) & (dl >= 0.1) & (dl <= 10.0)
    assert pts.shape[1] == ok.sum()
    X, Y, Z = pts.astype(np.float64)
    np.testing.assert_allclose(Z, dl[ok])
    np.testing.assert_allclose(cur.fx * X / Z + cur.cx, xs[ok] + 0.5, atol=1e-4)
    np.testing.assert_allclose(cur.fy * Y / Z + cur.cy, ys[ok] + 0.5, atol=1e-4)
    R, t = synth.pose_wc(cur)
    pw = oracle.frame_points(d, cur, stride=s, pose_wc=(R, t))
    np.testing.assert_allclose(R.T @ (pw.astype(np.float64) - t[:, None]), pts, atol=1e-5)


def test_so3_exp_matches_rotation_vectors():
    spatial = pytest.importorskip("scipy.spatial.transform")
    g = np.random.default_rng(6)
    for ang in (0.0, 1e-9, 1e-6, 1e-4, 0.1, 1.0, 3.0):
        w = g.normal(size=3)
        w *= ang / np.linalg.norm(w)
        np.testing.assert_allclose(oracle.so3_exp(w), spatial.Rotation.from_rotvec(w).as_matrix(), atol=2e-15)


def spd(g, n):
    A = g.normal(size=(n, 3, 3)) * 0.3
    S = A @ A.transpose(0, 2, 1) + 0.05 * np.eye(3)
    return np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]])


def full(c6, i):
    a = c6[:, i]
    return np.array([[a[0], a[1], a[2]], [a[1], a[3], a[4]], [a[2], a[4], a[5]]])


def test_linearisation_against_differences_of_the_fixed_weight_cost():
    """With the correspondences and weights of the linearisation held fixed, cost(x) =
    sum d_i(x)^T W_i d_i(x) for the pose Exp(w) (R p + t) + v has gradient 2 b at x = 0, and the
    residuals' central differences give J, so H = sum J^T W J. Random SPD covariances stand in
    for the local ones, so W is independent of the neighbour search."""
    g = np.random.default_rng(7)
    tgt = g.uniform(-1, 1, (3, 400)).astype(np.float32)
    src = (tgt[:, :300] + g.normal(0, 0.01, (3, 300))).astype(np.float32)
    sc, tc = spd(g, 300), spd(g, 400)
    R = oracle.so3_exp([0.02, -0.01, 0.03])
    t = np.array([0.01, 0.02, -0.015])
    src = (R.T @ (src.astype(np.float64) - t[:, None])).astype(np.float32)  # so that T p lands near q
    lin = oracle.gicp_linearize(src, sc, tgt, tc, R, t, 0.2)
    corr = lin["corr"]
    assert lin["count"] == (corr >= 0).sum() > 250
    # the correspondences are the nearest targets within d_max (brute force in FP64, clear cases)
    P = R @ src.astype(np.float64) + t[:, None]
    D = ((P[:, :, None] - tgt.astype(np.float64)[:, None, :]) ** 2).sum(0)
    near = np.argmin(D, 1)
    srt = np.sort(D, 1)
    clear = (srt[:, 1] - srt[:, 0] > 1e-5) & (np.abs(srt[:, 0] - 0.04) > 1e-5)
    want = np.where(srt[:, 0] <= 0.04, near, -1)
    assert (corr[clear] == want[clear]).all()
    used = np.flatnonzero(corr >= 0)
    W = [np.linalg.inv(full(tc, corr[i]) + R @ full(sc, i) @ R.T) for i in used]
    q = tgt.astype(np.float64)[:, corr[used]]
    p = src.astype(np.float64)[:, used]

    def resid(x):
        E = oracle.so3_exp(x[:3])
        return q - (E @ (R @ p + t[:, None]) + x[3:, None])

    def cost(x):
        r = resid(x)
        return sum(r[:, k] @ W[k] @ r[:, k] for k in range(len(used)))

    assert cost(np.zeros(6)) == pytest.approx(lin["cost"], rel=1e-12)
    h = 1e-6
    grad = np.array([(cost(h * e) - cost(-h * e)) / (2 * h) for e in np.eye(6)])
    np.testing.assert_allclose(lin["b"], grad / 2, rtol=1e-6, atol=1e-9 * np.abs(grad).max())
    J = np.stack([(resid(h * e) - resid(-h * e)) / (2 * h) for e in np.eye(6)], -1)  # (3, m, 6)
    Hfd = sum(J[:, k, :].T @ W[k] @ J[:, k, :] for k in range(len(used)))
    np.testing.assert_allclose(lin["H"], Hfd, rtol=1e-6, atol=1e-9 * np.abs(Hfd).max())
    np.testing.assert_allclose(lin["H"], lin["H"].T, atol=0)


def room_clouds(seed, w=160, h=120, f=131.25, stride=2, n_key=3):
    room = synth.room_scene(seed)
    keys, cur = synth.tracking_cameras(seed, n_key=n_key, width=w, height=h, f=f)
    tgt = np.concatenate([oracle.frame_points(synth.room_depth(room, c, 100 + i), c, stride,
                                              pose_wc=synth.pose_wc(c)) for i, c in enumerate(keys)], 1)
    src = oracle.frame_points(synth.room_depth(room, cur, 99), cur, stride)
    return src, tgt, keys, cur


def test_align_recovers_a_known_rigid_motion():
    """Source = a target subset moved by a known motion (no noise beyond binary32 rounding): from
    keyframe 0's pose the alignment returns that motion."""
    _, tgt, keys, cur = room_clouds(8)
    g = np.random.default_rng(9)
    sel = np.sort(g.choice(tgt.shape[1], 2000, replace=False))
    R1, t1 = synth.pose_wc(cur)
    src = (R1.T @ (tgt[:, sel].astype(np.float64) - t1[:, None])).astype(np.float32)
    sc, tc = oracle.cloud_cov(src, 20, 1e-3), oracle.cloud_cov(tgt, 20, 1e-3)
    R0, t0 = synth.pose_wc(keys[0])
    r = oracle.gicp_align(src, sc, tgt, tc, R0, t0, 0.1, max_iter=40, eps_rot=1e-9, eps_trans=1e-9)
    assert r["status"] == 0 and r["iterations"] < 40
    ang = np.arccos(np.clip((np.trace(r["R"].T @ R1) - 1) / 2, -1, 1))
    assert ang < 1e-6 and np.linalg.norm(r["t"] - t1) < 1e-6, (ang, r["t"] - t1)
    assert r["cost"] < 1e-6 * r["count"]


def test_align_from_a_noisy_frame_lands_near_the_true_pose():
    src, tgt, keys, cur = room_clouds(10)
    sc, tc = oracle.cloud_cov(src, 20, 1e-3), oracle.cloud_cov(tgt, 20, 1e-3)
    R0, t0 = synth.pose_wc(keys[0])
    R1, t1 = synth.pose_wc(cur)
    r = oracle.gicp_align(src, sc, tgt, tc, R0, t0, 0.1, max_iter=40, eps_rot=1e-7, eps_trans=1e-7)
    ang = np.arccos(np.clip((np.trace(r["R"].T @ R1) - 1) / 2, -1, 1))
    a0 = np.arccos(np.clip((np.trace(R0.T @ R1) - 1) / 2, -1, 1))
    assert r["status"] == 0
    assert ang < 0.2 * a0 and np.linalg.norm(r["t"] - t1) < 0.01, (np.rad2deg(ang), np.linalg.norm(r["t"] - t1))


def test_align_with_too_few_correspondences_changes_nothing():
    src, tgt, keys, _ = room_clouds(11)
    sc, tc = oracle.cloud_cov(src, 20, 1e-3), oracle.cloud_cov(tgt, 20, 1e-3)
    R0, t0 = synth.pose_wc(keys[0])
    r = oracle.gicp_align(src, sc, tgt, tc, R0, t0 + 5.0, 0.01)
    assert r["status"] == 2 and r["iterations"] == 0 and r["count"] < 6
    np.testing.assert_array_equal(r["R"], R0)
    np.testing.assert_array_equal(r["t"], t0 + 5.0)
