"""Seeded synthetic inputs: gaussian scenes, pinhole cameras and RGB-D frames.

These stand in for the paper's evaluation data (Replica frames of 1200x680 and
TUM RGB-D frames of 640x480, Sec. IV-A), which are not available here. Nothing
in this module is part of the method: it only draws random numbers, places
cameras and paints frames. Both the HIP path's tests and the CPU oracle's tests
take their inputs from here; neither side's arithmetic lives here.

Every generator uses ``numpy.random.Generator(PCG64(seed))``, draws in float64
in the order documented per function, and returns float32 arrays.

Gaussian parameters are one SoA array of shape (14, N):
rows 0-2 mean (x, y, z), rows 3-5 log-scale, rows 6-9 quaternion (w, x, y, z),
row 10 opacity logit, rows 11-13 RGB.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ROW_MEAN = slice(0, 3)
ROW_LOG_SCALE = slice(3, 6)
ROW_QUAT = slice(6, 10)
ROW_OPACITY = 10
ROW_RGB = slice(11, 14)
N_PARAM_ROWS = 14


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Camera:
    """Pinhole camera; world -> camera is x_c = R @ x_w + t (row-major R)."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray = field(default_factory=lambda: np.eye(3, dtype=np.float32))
    t: np.ndarray = field(default_factory=lambda: np.zeros(3, dtype=np.float32))
    z_near: float = 0.2

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.ascontiguousarray(self.t, dtype=np.float32).reshape(3)

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


def centred_camera(width: int, height: int, f: float, z_near: float = 0.2) -> Camera:
    """Identity pose, principal point at the image centre (pixel (x, y) samples (x+.5, y+.5))."""
    return Camera(width, height, f, f, width / 2.0, height / 2.0, z_near=z_near)


def look_at_camera(width: int, height: int, f: float, centre, target,
                   z_near: float = 0.2) -> Camera:
    """Camera at ``centre`` looking at ``target`` with world +z up (x right, y down, z forward)."""
    c = np.asarray(centre, np.float64)
    fwd = np.asarray(target, np.float64) - c
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ c
    return Camera(width, height, f, f, width / 2.0, height / 2.0, R=R, t=t, z_near=z_near)


def _attributes(g: np.random.Generator, n: int) -> dict:
    """Draw order: log-scale (n,3) ~ N(-3, 0.5); quaternion (n,4) ~ normalise(N(0,1)^4);
    opacity logit (n,) ~ N(0,1); rgb (n,3) ~ U[0,1]."""
    log_scale = g.normal(-3.0, 0.5, size=(n, 3))
    q = g.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logit = g.normal(0.0, 1.0, size=n)
    rgb = g.uniform(0.0, 1.0, size=(n, 3))
    return dict(log_scale=log_scale, quat=q, logit=logit, rgb=rgb)


def _frustum_means(g: np.random.Generator, n: int, cam: Camera, z0: float, z1: float) -> np.ndarray:
    """Means uniform in the camera frustum's volume between depths z0 and z1 (identity pose).
    Draw order: U for z (n,), u ~ U[0,W) (n,), v ~ U[0,H) (n,)."""
    U = g.uniform(0.0, 1.0, size=n)
    z = np.cbrt(z0 ** 3 + U * (z1 ** 3 - z0 ** 3))
    u = g.uniform(0.0, cam.width, size=n)
    v = g.uniform(0.0, cam.height, size=n)
    X = (u - cam.cx) * z / cam.fx
    Y = (v - cam.cy) * z / cam.fy
    return np.stack([X, Y, z], axis=1)


def _pack(means: np.ndarray, attr: dict) -> np.ndarray:
    n = means.shape[0]
    out = np.empty((N_PARAM_ROWS, n), np.float32)
    out[ROW_MEAN] = means.T
    out[ROW_LOG_SCALE] = attr["log_scale"].T
    out[ROW_QUAT] = attr["quat"].T
    out[ROW_OPACITY] = attr["logit"]
    out[ROW_RGB] = attr["rgb"].T
    return out


def frustum_scene(seed: int, n: int, cam: Camera, z0: float, z1: float,
                  blob_frac: float = 0.0, n_blobs: int = 8, blob_sigma: float = 0.2) -> np.ndarray:
    """Random scene in an identity-pose camera's frustum.

    Draw order: frustum means for the n_uniform = n - n_blob free gaussians; then
    the n_blobs blob centres (frustum-uniform like the free means); then the blob
    members' offsets N(0, blob_sigma^2 I) (n_blob, 3); then attributes for all n.
    """
    g = rng(seed)
    n_blob = int(round(n * blob_frac))
    n_blob -= n_blob % max(n_blobs, 1)
    means = [_frustum_means(g, n - n_blob, cam, z0, z1)]
    if n_blob:
        centres = _frustum_means(g, n_blobs, cam, z0, z1)
        offs = g.normal(0.0, blob_sigma, size=(n_blob, 3))
        per = n_blob // n_blobs
        means.append(np.repeat(centres, per, axis=0) + offs)
    return _pack(np.concatenate(means, 0), _attributes(g, n))


def box_scene(seed: int, n: int, lo=(-3.0, -3.0, 0.0), hi=(3.0, 3.0, 4.0),
              blob_frac: float = 0.2, n_blobs: int = 8, blob_sigma: float = 0.2) -> np.ndarray:
    """Random scene in an axis-aligned box: uniform means, plus blobs with uniform centres.

    Draw order: free means U(box) (n_free, 3); blob centres U(box) (n_blobs, 3);
    member offsets N(0, blob_sigma^2 I); attributes for all n.
    """
    g = rng(seed)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    n_blob = int(round(n * blob_frac))
    n_blob -= n_blob % max(n_blobs, 1)
    means = [g.uniform(lo, hi, size=(n - n_blob, 3))]
    if n_blob:
        centres = g.uniform(lo, hi, size=(n_blobs, 3))
        offs = g.normal(0.0, blob_sigma, size=(n_blob, 3))
        means.append(np.repeat(centres, n_blob // n_blobs, axis=0) + offs)
    return _pack(np.concatenate(means, 0), _attributes(g, n))


# ----------------------------------------------------------------------------------------------
# Workloads.  "c0" .. "c4" follow the five benchmark configurations of this project.
# ----------------------------------------------------------------------------------------------

def camera_small() -> Camera:
    """64x48 pinhole, fx = fy = 60, principal point at the centre, identity pose."""
    return centred_camera(64, 48, 60.0)


def scene_small(seed: int = 0) -> np.ndarray:
    """2,000 gaussians, frustum-uniform at depth 1-5 m (the small plain-splat workload)."""
    return frustum_scene(seed, 2000, camera_small(), 1.0, 5.0)


def camera_replica() -> Camera:
    """1200x680 pinhole with fx = fy = 600 (Replica-sized frames)."""
    return centred_camera(1200, 680, 600.0)


def scene_replica(seed: int = 0, n: int = 300_000) -> np.ndarray:
    """300k gaussians at depth 0.5-8 m, 20% of them in 8 dense blobs (sigma 0.2 m)."""
    return frustum_scene(seed, n, camera_replica(), 0.5, 8.0, blob_frac=0.2)


def camera_tum() -> Camera:
    """640x480 pinhole with fx = fy = 525 (TUM-RGB-D-sized frames)."""
    return centred_camera(640, 480, 525.0)


def rgbd_frame(seed: int, width: int = 640, height: int = 480, n_rect: int = 40):
    """Synthetic RGB-D frame: smooth colour gradient plus rectangles of band-limited noise,
    planar depth with per-rectangle offsets and N(0, 5 mm^2) noise.

    Draw order: 3 corner colours U[0,1]^3 (3,3); depth plane z_c ~ U[2,3], g ~ U[-1,1]^2;
    then per rectangle: top-left x ~ U[0,W), y ~ U[0,H); w, h ~ U{16..128}; tint ~ U[0.2,0.8]^3;
    f0 ~ U[0.05,0.4]; 8 waves of (f ~ U[0.8,1.2] f0, theta ~ U[0,pi), phi ~ U[0,2pi));
    depth offset ~ U[-0.5,0.5]. Finally the depth noise (H, W).
    Returns rgb (3, H, W) float32 in [0,1] and depth (H, W) float32 in metres.
    """
    g = rng(seed)
    W, H = width, height
    xs = (np.arange(W) + 0.5) / W
    ys = (np.arange(H) + 0.5) / H
    corners = g.uniform(0.0, 1.0, size=(3, 3))
    X, Y = np.meshgrid(xs, ys)
    # bilinear blend between three corners (top-left, top-right, bottom-left)
    rgb = (corners[0][:, None, None] * (1 - X) * (1 - Y)
           + corners[1][:, None, None] * X * (1 - Y)
           + corners[2][:, None, None] * (1 - X) * Y
           + 0.5 * (corners[1] + corners[2])[:, None, None] * X * Y)
    zc = g.uniform(2.0, 3.0)
    gx, gy = g.uniform(-1.0, 1.0, size=2)
    px = np.arange(W)[None, :].astype(np.float64)
    py = np.arange(H)[:, None].astype(np.float64)
    depth = zc + gx * (px - W / 2) / W + gy * (py - H / 2) / H + 0.0 * px
    for _ in range(n_rect):
        x0 = int(g.uniform(0, W))
        y0 = int(g.uniform(0, H))
        w, h = g.integers(16, 129, size=2)
        tint = g.uniform(0.2, 0.8, size=3)
        f0 = g.uniform(0.05, 0.4)
        waves = np.zeros((h, w))
        yy = np.arange(y0, y0 + h)[:, None].astype(np.float64)
        xx = np.arange(x0, x0 + w)[None, :].astype(np.float64)
        for _k in range(8):
            f = g.uniform(0.8, 1.2) * f0
            th = g.uniform(0.0, np.pi)
            ph = g.uniform(0.0, 2 * np.pi)
            waves += np.cos(2 * np.pi * f * (xx * np.cos(th) + yy * np.sin(th)) + ph)
        dz = g.uniform(-0.5, 0.5)
        x1, y1 = min(x0 + w, W), min(y0 + h, H)
        patch = tint[:, None, None] + 0.2 * (waves / 8.0)[None]
        rgb[:, y0:y1, x0:x1] = patch[:, : y1 - y0, : x1 - x0]
        depth[y0:y1, x0:x1] += dz
    rgb = np.clip(rgb, 0.0, 1.0)
    depth = np.clip(depth, 1.0, 4.0) + g.normal(0.0, 0.005, size=(H, W))
    return rgb.astype(np.float32), depth.astype(np.float32)


def scene_window(seed: int = 0, n: int = 500_000) -> np.ndarray:
    """500k gaussians in the 6x6x4 m box [-3,3]x[-3,3]x[0,4], 20% in 8 blobs (sigma 0.2 m)."""
    return box_scene(seed, n)


def window_cameras(seed: int = 0):
    """Four 640x480 (f=525) and four 1200x680 (f=600) look-at cameras in the window scene.

    Per camera, in order: centre ~ U([-2,2]x[-2,2]x[1,3]); target ~ U([-1,1]x[-1,1]x[1,3]);
    redraw both while the target is closer than 1 m.
    """
    g = rng(seed)
    cams = []
    for k in range(8):
        while True:
            c = g.uniform([-2.0, -2.0, 1.0], [2.0, 2.0, 3.0])
            tgt = g.uniform([-1.0, -1.0, 1.0], [1.0, 1.0, 3.0])
            if np.linalg.norm(tgt - c) >= 1.0:
                break
        if k < 4:
            cams.append(look_at_camera(640, 480, 525.0, c, tgt))
        else:
            cams.append(look_at_camera(1200, 680, 600.0, c, tgt))
    return cams


def random_planes(seed: int, shape, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random float32 planes, e.g. upstream gradients or stand-in targets."""
    return rng(seed).uniform(lo, hi, size=shape).astype(np.float32)


# ----------------------------------- tracking frames -----------------------------------

@dataclass
class Room:
    """An axis-aligned room (interior box lo..hi) with axis-aligned boxes standing in it."""
    lo: np.ndarray
    hi: np.ndarray
    boxes: np.ndarray  # (n, 2, 3): lower and upper corner of each box


def room_scene(seed: int, n_boxes: int = 12) -> Room:
    """The 6x6x3 m room [-3,3]x[-3,3]x[0,3] with n_boxes boxes on the floor. Per box, in order:
    size ~ U([0.3, 0.3, 0.3], [1.0, 1.0, 1.5]); centre (x, y) ~ U within 0.3 m of the walls."""
    g = rng(seed)
    lo, hi = np.array([-3.0, -3.0, 0.0]), np.array([3.0, 3.0, 3.0])
    boxes = []
    for _ in range(n_boxes):
        size = g.uniform([0.3, 0.3, 0.3], [1.0, 1.0, 1.5])
        c = g.uniform(lo[:2] + 0.3 + size[:2] / 2, hi[:2] - 0.3 - size[:2] / 2)
        blo = np.array([c[0] - size[0] / 2, c[1] - size[1] / 2, 0.0])
        boxes.append([blo, blo + size])
    return Room(lo, hi, np.asarray(boxes, np.float64).reshape(-1, 2, 3))


def room_depth(room: Room, cam: Camera, seed: int, noise: float = 0.002) -> np.ndarray:
    """Depth frame (H, W) float32 of `room` seen by `cam`, ray-cast at pixel centres (camera z of
    the first surface hit: the walls from inside, the boxes from outside), plus N(0, noise^2)."""
    H, W = cam.height, cam.width
    R = np.asarray(cam.R, np.float64)
    o = -R.T @ np.asarray(cam.t, np.float64)
    ys, xs = np.mgrid[0:H, 0:W]
    dc = np.stack([(xs + 0.5 - cam.cx) / cam.fx, (ys + 0.5 - cam.cy) / cam.fy, np.ones((H, W))], -1)
    dw = dc @ R  # rows: R^T dc; the ray parameter is the camera depth (dc_z = 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        exit_t = np.where(dw > 0, (room.hi - o) / dw, np.where(dw < 0, (room.lo - o) / dw, np.inf))
        s = exit_t.min(-1)
        for blo, bhi in room.boxes:
            t1, t2 = (blo - o) / dw, (bhi - o) / dw
            tmin = np.nan_to_num(np.minimum(t1, t2), nan=-np.inf).max(-1)
            tmax = np.nan_to_num(np.maximum(t1, t2), nan=np.inf).min(-1)
            hit = (tmin <= tmax) & (tmin > 0)
            s = np.where(hit & (tmin < s), tmin, s)
    return (s + rng(seed).normal(0.0, noise, size=(H, W))).astype(np.float32)


def pose_wc(cam: Camera):
    """Camera-to-world pose (R_wc, t_wc) of `cam` in float64."""
    R = np.asarray(cam.R, np.float64)
    return R.T, -R.T @ np.asarray(cam.t, np.float64)


def camera_from_pose(R_wc, t_wc, like: Camera) -> Camera:
    """A camera with `like`'s intrinsics at the camera-to-world pose (R_wc, t_wc)."""
    R = np.asarray(R_wc, np.float64).T
    return Camera(like.width, like.height, like.fx, like.fy, like.cx, like.cy, R=R, t=-R @ np.asarray(t_wc),
                  z_near=like.z_near)


def tracking_cameras(seed: int, n_key: int = 8, width: int = 640, height: int = 480, f: float = 525.0,
                     rot_deg=(1.0, 3.0), trans_m=(0.03, 0.06)):
    """Keyframe cameras in the room and a current camera near the first one. Per keyframe, in order:
    centre ~ U([-2,-2,1.6], [2,2,2.2]), target ~ U([-2.5,-2.5,0.2], [2.5,2.5,1.5]), redrawn while
    closer than 1.5 m. Then the current camera: keyframe 0's camera-to-world pose moved by a rotation
    about a uniformly random axis by an angle ~ U(rot_deg) degrees (applied in the camera frame)
    and a translation of length ~ U(trans_m) along a uniformly random direction (world frame)."""
    from scipy.spatial.transform import Rotation
    g = rng(seed)
    keys = []
    for _ in range(n_key):
        while True:
            c = g.uniform([-2.0, -2.0, 1.6], [2.0, 2.0, 2.2])
            tg = g.uniform([-2.5, -2.5, 0.2], [2.5, 2.5, 1.5])
            if np.linalg.norm(tg - c) >= 1.5:
                break
        keys.append(look_at_camera(width, height, f, c, tg))
    axis = g.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = np.deg2rad(g.uniform(*rot_deg))
    tdir = g.normal(size=3)
    tdir /= np.linalg.norm(tdir)
    tlen = g.uniform(*trans_m)
    R0, t0 = pose_wc(keys[0])
    R1 = R0 @ Rotation.from_rotvec(axis * ang).as_matrix()
    t1 = t0 + tdir * tlen
    return keys, camera_from_pose(R1, t1, keys[0])
