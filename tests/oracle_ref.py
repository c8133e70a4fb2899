"""Oracle references for the mapping-step and keyframe-window parity tests: per view the oracle's
forward (Eq. 1), the L1 terms of Eq. 16 and the analytic backward, summed over the views. Targets
are nudged away from the L1 terms' sign changes, and the pixels the oracle flags as ambiguous (a
cutoff decision within rounding of its threshold, which an FP32 path may legitimately take the
other way) get a zero upstream gradient on both sides through the targets themselves."""
import numpy as np

import oracle

# the binary32 values of the default options, as the C ABI hands them to the kernels
F32_OPTS = oracle.RenderOpts(*(float(np.float32(v)) for v in (3.0, 1.0 / 255.0, 0.99, 1e-4, 0.3)))


def nudge_targets(rgb, depth, trgb, tdepth, eps=1e-3, step=0.01):
    """Targets moved by `step` wherever the residual is within eps of zero (both sides then take the
    same sign in the L1 gradient)."""
    trgb = np.array(trgb, np.float32, copy=True)
    tdepth = np.array(tdepth, np.float32, copy=True)
    trgb[np.abs(rgb - trgb) < eps] += step
    near = (np.abs(depth - tdepth) < eps) & (tdepth > 0)
    tdepth[near] += step
    return trgb, tdepth


def ambiguous_gaussians(p64, cam, amb, widen=2e-5, chunk=64):
    """Gaussians that reach a flagged pixel: Q <= sigma_cut^2 (1 + widen) at its centre (a superset
    of every pair whose cutoff decision there could go either way, and of its contributors)."""
    n = p64.shape[1]
    hit = np.zeros(n, bool)
    ys, xs = np.nonzero(amb)
    if xs.size == 0:
        return hit
    pr = oracle.project(p64, cam, F32_OPTS)
    idx = np.nonzero(pr[:, 0] > 0)[0]
    mx, my = pr[idx, 10], pr[idx, 11]
    a, b, c = pr[idx, 7], pr[idx, 8], pr[idx, 9]
    rx = 3.0 * np.sqrt(np.maximum(pr[idx, 4], 0)) * 1.01 + 1e-3
    ry = 3.0 * np.sqrt(np.maximum(pr[idx, 6], 0)) * 1.01 + 1e-3
    for k in range(0, xs.size, chunk):
        px = xs[k:k + chunk, None] + 0.5
        py = ys[k:k + chunk, None] + 0.5
        rows, cols = np.nonzero((np.abs(px - mx) <= rx) & (np.abs(py - my) <= ry))
        dx = px[rows, 0] - mx[cols]
        dy = py[rows, 0] - my[cols]
        Q = a[cols] * dx * dx + 2.0 * b[cols] * dx * dy + c[cols] * dy * dy
        hit[idx[cols[Q <= 9.0 * (1.0 + widen)]]] = True
    return hit


def mask_ambiguous(trgb, tdepth, amb):
    """Targets that give ambiguous pixels a zero upstream gradient on both sides: a NaN colour
    target (sign(NaN) = 0 in the L1 gradient of either implementation; the loss itself becomes NaN)
    and a depth target of 0 (no depth measurement: the pixel leaves the depth term)."""
    trgb = np.array(trgb, np.float32, copy=True)
    tdepth = np.array(tdepth, np.float32, copy=True)
    trgb[:, amb] = np.nan
    tdepth[amb] = 0.0
    return trgb, tdepth


def mapping_reference(p, cams, targets, lambda_rgb=1.0, lambda_depth=0.1, log=None):
    """Oracle mapping step over views. Returns dict(loss[v], psnr[v] on the nudged targets,
    targets: the nudged targets (float32), masked: the same with ambiguous pixels masked
    (mask_ambiguous), grad: the gradient (14, N) summed over views for the masked targets, mass: the
    absolute mass of each of its entries, amb[v]: the flagged pixels). targets: list of (rgb (3, H, W), depth (H, W)) host arrays."""
    p64 = np.asarray(p, np.float64)
    n = p64.shape[1]
    grad = np.zeros((14, n))
    mass = np.zeros((14, n))
    losses, psnrs, tg, masked, ambs = [], [], [], [], []
    for cam, (trgb, td) in zip(cams, targets):
        ref = oracle.render_fwd(p64, cam, F32_OPTS, amb_rel=1e-5)
        trgb = np.asarray(trgb, np.float32).reshape(3, cam.height, cam.width)
        td = np.asarray(td, np.float32).reshape(cam.height, cam.width)
        trgb, td = nudge_targets(ref["rgb"], ref["depth"], trgb, td)
        L, ps, _, _ = oracle.loss_l1(ref["rgb"], ref["depth"], trgb, td, lambda_rgb, lambda_depth)
        mr, md = mask_ambiguous(trgb, td, ref["amb"])
        _, _, gr, gd = oracle.loss_l1(ref["rgb"], ref["depth"], mr, md, lambda_rgb, lambda_depth)
        g, _, m = oracle.render_bwd(p64, cam, gr, gd, None, F32_OPTS, mass=True)
        grad += g
        mass += m
        losses.append(L)
        psnrs.append(ps)
        tg.append((trgb, td))
        masked.append((mr, md))
        ambs.append(ref["amb"])
        if log:
            log(f"oracle view {len(losses)}/{len(cams)}: {int(ref['amb'].sum())} ambiguous pixels")
    return dict(loss=np.array(losses), psnr=np.array(psnrs), grad=grad, mass=mass, targets=tg, masked=masked,
                amb=ambs)


def gradient_errors(gpu, ref, keep=None):
    """Per row group: max |gpu - ref| / max |ref|, and the largest elementwise relative error among
    elements with |ref| >= f max|ref| for f in (1e-1, 1e-2, 1e-3) (columns in `keep` only)."""
    rows = (("mean", slice(0, 3)), ("log_scale", slice(3, 6)), ("quat", slice(6, 10)),
            ("opacity", slice(10, 11)), ("rgb", slice(11, 14)))
    out = {}
    for name, sl in rows:
        g = np.asarray(gpu, np.float64)[sl]
        r = np.asarray(ref, np.float64)[sl]
        if keep is not None:
            g, r = g[:, keep], r[:, keep]
        scale = np.abs(r).max()
        err = np.abs(g - r)
        d = {"abs": float(err.max() / scale) if scale > 0 else float(err.max())}
        for f in (1e-1, 1e-2, 1e-3):
            big = np.abs(r) >= f * scale
            d[f"rel@{f:g}"] = float((err[big] / np.abs(r[big])).max()) if big.any() else 0.0
        out[name] = d
    return out
