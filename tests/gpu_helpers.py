"""Helpers shared by the GPU parity tests: device transfer, oracle comparison tolerances."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def have_gpu() -> bool:
    return torch.cuda.is_available()


def need_gpu():
    if not have_gpu():
        pytest.skip("no GPU")


def oracle_opts(o=None):
    """The oracle's render options for a GPU comparison: the binary32 values the C ABI hands the
    kernels (alpha_max = 0.99 arrives as 0.9900000095...), so that both sides clamp, skip and stop
    at the same thresholds. o: the binding's RenderOpts (default options when None)."""
    import oracle
    f = lambda v: float(np.float32(v))
    if o is None:
        o = oracle.RenderOpts()
    return oracle.RenderOpts(f(o.sigma_cut), f(o.alpha_min), f(o.alpha_max), f(o.T_min), f(o.lowpass),
                             tuple(f(b) for b in o.bg), f(o.bg_depth))


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda().contiguous()


def host(t):
    return t.detach().cpu().numpy()


def assert_close_rel(gpu, ref, tol, mask=None, what="", floor=1e-3):
    """Tolerance of the parity bar: per tensor max|gpu - ref| <= tol * max|ref|, and elementwise
    |gpu - ref| <= tol * |ref| wherever |ref| >= floor * max|ref|. mask selects compared elements.

    Used for rendered planes (floor = 1e-3); gradients use assert_grad_close."""
    g = np.asarray(gpu, np.float64)
    r = np.asarray(ref, np.float64)
    if mask is not None:
        g = g[..., mask] if g.ndim > mask.ndim else g[mask]
        r = r[..., mask] if r.ndim > mask.ndim else r[mask]
    scale = np.abs(r).max() if r.size else 0.0
    if scale == 0.0:
        assert np.abs(g).max(initial=0.0) == 0.0, f"{what}: reference is zero, gpu is not"
        return
    err = np.abs(g - r)
    assert err.max() <= tol * scale, f"{what}: max abs err {err.max():.3e} > {tol:.1e} * {scale:.3e}"
    big = np.abs(r) >= floor * scale
    rel = err[big] / np.abs(r[big])
    if rel.size:
        worst = rel.max()
        k = int(np.argmax(rel))
        assert worst <= tol, (f"{what}: max elementwise rel err {worst:.3e} > {tol:.1e} ({(rel > tol).sum()} elems; "
                              f"worst |ref|/max|ref| = {np.abs(r[big])[k] / scale:.2e}, max abs err/scale "
                              f"{err.max() / scale:.2e})")


U32 = 2.0 ** -24           # unit roundoff of binary32
MASS_C = 64.0              # rounding-error multiple allowed on a sum's absolute mass (measured up to 26)
NEAR_PLANE_FRAC = 2e-2     # near-plane splats: share of the absolute mass allowed (measured up to 0.72%)
GRAD_ROWS = (("mean", slice(0, 3)), ("log_scale", slice(3, 6)), ("quat", slice(6, 10)),
             ("opacity", slice(10, 11)), ("rgb", slice(11, 14)))


def assert_grad_close(gpu, ref, mass, what="", tol=1e-4, near=None, cols=None):
    """Gradient parity with the FP64 oracle. Every element: |gpu - ref| <= tol |ref| + MASS_C u mass,
    where mass (the oracle's render_bwd(..., mass=True)) is the absolute mass of the sum that
    defines the element, so u mass bounds what rounding to binary32 anywhere in that sum can cost
    (elements whose terms cancel get that allowance; a well-conditioned element, mass ~ |ref|, is
    held to about tol), plus 1e-12 of the row's largest entry for the FP64 residue of entries that
    vanish exactly. Per row group also max |gpu - ref| <= tol max |ref|. near (bool per gaussian,
    optional): splats just past the near plane, whose FP32 terms are dominated by the rounding of
    very elongated, far off-centre projections rather than by the sums; they are held to tol |ref| +
    NEAR_PLANE_FRAC mass and left out of the per-tensor bound. cols (optional) selects gaussians."""
    g = np.asarray(gpu, np.float64)
    r = np.asarray(ref, np.float64)
    m = np.asarray(mass, np.float64)
    if cols is not None:
        g, r, m = g[:, cols], r[:, cols], m[:, cols]
        near = None if near is None else np.asarray(near)[cols]
    reg = np.ones(g.shape[1], bool) if near is None else ~np.asarray(near, bool)
    for name, rows in GRAD_ROWS:
        e = np.abs(g[rows] - r[rows])
        # 1e-12 of the row's largest entry: the FP64 residue of entries that vanish exactly (the
        # rotation gradient of an isotropic gaussian), far below what binary32 resolves in the row
        bound = tol * np.abs(r[rows]) + np.where(reg[None, :], MASS_C * U32, NEAR_PLANE_FRAC) * m[rows] + \
            1e-12 * np.abs(r[rows]).max()
        bad = e > bound
        if bad.any():
            k = np.unravel_index(np.argmax(e / np.maximum(bound, 1e-300)), e.shape)
            raise AssertionError(
                f"{what} d{name}: {int(bad.sum())} elements beyond tol |ref| + c u mass; worst gaussian {k[1]}: "
                f"gpu {g[rows][k]:.6e} ref {r[rows][k]:.6e} mass {m[rows][k]:.3e} "
                f"({e[k] / max(bound[k], 1e-300):.2f} x bound, near plane {not reg[k[1]]})")
        if reg.any():
            scale = np.abs(r[rows][:, reg]).max()
            assert e[:, reg].max() <= tol * scale + 1e-300, (
                f"{what} d{name}: max abs err {e[:, reg].max():.3e} > {tol:.0e} * {scale:.3e}")


def near_plane_splats(p, cams, frac=1.25):
    """Gaussians whose camera depth is within frac * z_near in some view where they project."""
    import oracle
    near = np.zeros(np.asarray(p).shape[1], bool)
    for c in cams:
        pr = oracle.project(np.asarray(p, np.float64), c, oracle_opts())
        near |= (pr[:, 0] > 0) & (pr[:, 3] <= frac * c.z_near)
    return near
