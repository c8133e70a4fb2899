"""Helpers shared by the GPU parity tests: device transfer, oracle comparison tolerances."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def have_gpu() -> bool:
    return torch.cuda.is_available()


def need_gpu():
    if not have_gpu():
        pytest.skip("no GPU")


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda().contiguous()


def host(t):
    return t.detach().cpu().numpy()


def assert_close_rel(gpu, ref, tol, mask=None, what="", floor=1e-3):
    """Tolerance of the parity bar: per tensor max|gpu - ref| <= tol * max|ref|, and elementwise
    |gpu - ref| <= tol * |ref| wherever |ref| >= floor * max|ref|. mask selects compared elements.

    Rendered planes use floor = 1e-3. Gradients are sums over many pixels with cancelling signs;
    their FP32 absolute error floor is a few 1e-7 of max|ref| on the small scenes (measured), so
    they use floor = 1e-2, where that floor is at most a tenth of the 1e-4 bar; the full-size
    sampled test measures up to 1.2e-6 and uses 2e-2."""
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
