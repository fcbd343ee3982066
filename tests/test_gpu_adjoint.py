"""GPU adjoint (bn_normals_vjp / torch.autograd) against the FP64 oracle's
adjoint and against FP64 central finite differences."""
import numpy as np
import pytest

import oracle
import paper_2209_08241_amd as bn
from gpu_util import log, to_gpu
from synth import scenes

pytestmark = pytest.mark.gpu

VALID = 0


def vjp_tol(ref):
    """Elementwise bound: binary32 evaluation of about 60 operations per
    pixel, with cancellation in the tangential projection."""
    return 1e-4 * np.abs(ref).max() + 1e-3 * np.abs(ref)


def check_vjp(depth, fx, fy, cx, cy, alpha, g, mode="rel", tau=4.0, stride_pad=0, what=""):
    import torch
    o = oracle.default()
    codes = o.normals_f32(depth, fx, fy, cx, cy, alpha, mode, tau)["mask"]
    ref = o.normals_vjp_f64(depth, fx, fy, cx, cy, alpha, codes, g)
    d = to_gpu(depth, stride_pad)
    gt = torch.from_numpy(g.astype(np.float32)).cuda()
    got = bn.normals_vjp(d, fx, fy, cx, cy, gt, alpha, mode, tau).cpu().numpy()
    err = np.abs(got - ref)
    bad = err > vjp_tol(ref)
    if bad.any():
        y, x = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {bad.sum()} gradients off; at ({x},{y}) gpu {got[y, x]} "
                             f"oracle {ref[y, x]} (max |ref| {np.abs(ref).max():.3g})")
    return float(err.max() / max(np.abs(ref).max(), 1e-30))


@pytest.mark.parametrize("alpha", [1, 2, 3, 8])
def test_vjp_random_cotangent(alpha):
    s = scenes.frame_640x480(seed=2000 + alpha)
    rng = np.random.default_rng(alpha)
    g = rng.standard_normal((480, 640, 3))
    e = check_vjp(s.depth, *s.intrinsics, alpha, g, what=f"640x480 alpha={alpha}")
    log(f"alpha={alpha}: max |gpu - oracle| / max|grad| = {e:.2e}")


@pytest.mark.parametrize("alpha", [1, 2, 5])
def test_vjp_large_frame_tiles(alpha):
    """Frames of 2^20 pixels and more take the 64 x 16 tiles."""
    s = scenes.frame_1920x1080(seed=2100 + alpha)
    rng = np.random.default_rng(100 + alpha)
    g = rng.standard_normal((1080, 1920, 3))
    check_vjp(s.depth, *s.intrinsics, alpha, g, what=f"1920x1080 alpha={alpha}")


@pytest.mark.parametrize("H,W,pad", [(1, 1, 0), (5, 7, 0), (33, 65, 3), (17, 130, 0), (70, 90, 5),
                                     (1024, 1024, 0), (1023, 1025, 2)])
def test_vjp_shapes(H, W, pad):
    rng = np.random.default_rng(H * W)
    d = rng.uniform(1.0, 1.3, size=(H, W)).astype(np.float32)
    d[rng.random((H, W)) < 0.03] = 0.0
    g = rng.standard_normal((H, W, 3))
    for alpha in (1, 2):
        check_vjp(d, 150.0, 160.0, (W - 1) / 2, (H - 1) / 2, alpha, g, "rel", 1.1, pad,
                  what=f"{H}x{W} pad {pad}")


def test_vjp_ignores_masked_cotangents():
    import torch
    s = scenes.frame_640x480(seed=2010)
    d = to_gpu(s.depth)
    n, m, _ = bn.estimate_normals(d, *s.intrinsics, 2)
    g = torch.randn((480, 640, 3), device="cuda")
    a = bn.normals_vjp(d, *s.intrinsics, g, 2)
    g2 = g.clone()
    g2[m != VALID] = float("nan")
    b = bn.normals_vjp(d, *s.intrinsics, g2, 2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    c = bn.normals_vjp(d, *s.intrinsics, g, 2)
    assert torch.equal(a, c)      # deterministic


def _loss_fd(o, depth, fx, fy, cx, cy, codes, t, U, pts, h=1e-6):
    dd = depth.astype(np.float64)

    def loss(x):
        nn = o.normals_frozen_f64(x, fx, fy, cx, cy, 2, codes)
        return np.sum((1.0 - np.sum(nn * t, axis=-1))[U]) / U.sum()
    out = []
    for (y, x) in pts:
        e = np.zeros_like(dd)
        e[y, x] = h
        out.append((loss(dd + e) - loss(dd - e)) / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("seed,x0,y0", [(2000, 300, 200), (2005, 100, 80), (2011, 500, 300)])
def test_autograd_loss_vs_finite_differences(seed, x0, y0):
    """Differentiation workload on a 32x32 crop: loss = mean over pixels
    valid in prediction and noise-free target of (1 - cos angle); the GPU
    gradient (autograd through the adjoint kernel) against FP64 central
    differences with h = 1e-6 m."""
    import torch
    o = oracle.default()
    s = scenes.frame_640x480(seed=seed)
    n = 32
    d = np.ascontiguousarray(s.depth[y0:y0 + n, x0:x0 + n])
    dc = np.ascontiguousarray(s.depth_clean[y0:y0 + n, x0:x0 + n]).astype(np.float32)
    fx, fy, cx, cy = s.fx, s.fy, s.cx - x0, s.cy - y0
    dt = torch.from_numpy(d).cuda().requires_grad_(True)
    tn, tm, _ = bn.estimate_normals(torch.from_numpy(dc).cuda(), fx, fy, cx, cy, 2)
    pn, pm = bn.normals_with_grad(dt, fx, fy, cx, cy, 2)
    loss = bn.cosine_loss(pn, tn, pm, tm)
    loss.backward()
    torch.cuda.synchronize()
    g = dt.grad.cpu().numpy().astype(np.float64)
    codes = pm.cpu().numpy()
    U = (codes == VALID) & (tm.cpu().numpy() == VALID)
    t = tn.cpu().numpy().astype(np.float64)
    pts = [(y, x) for y in range(0, n, 3) for x in range(0, n, 3)]
    fd = _loss_fd(o, d, fx, fy, cx, cy, codes, t, U, pts)
    got = np.array([g[y, x] for (y, x) in pts])
    tol = 1e-4 * np.abs(fd).max() + 1e-3 * np.abs(fd)
    assert np.all(np.abs(got - fd) <= tol), (np.abs(got - fd).max(), np.abs(fd).max())


def test_differentiation_batch_16():
    """16 x 640x480: per-frame autograd gradient of the cosine loss against
    the oracle's FP64 adjoint of the same cotangent."""
    import torch
    o = oracle.default()
    worst = 0.0
    for i in range(16):
        s = scenes.frame_640x480(seed=2000 + i)
        dt = torch.from_numpy(s.depth).cuda().requires_grad_(True)
        tn, tm, _ = bn.estimate_normals(torch.from_numpy(s.depth_clean.astype(np.float32)).cuda(),
                                        *s.intrinsics, 2)
        pn, pm = bn.normals_with_grad(dt, *s.intrinsics, 2)
        loss = bn.cosine_loss(pn, tn, pm, tm)
        loss.backward()
        torch.cuda.synchronize()
        codes = pm.cpu().numpy()
        U = (codes == VALID) & (tm.cpu().numpy() == VALID)
        gcot = np.where(U[..., None], -tn.cpu().numpy().astype(np.float64) / U.sum(), 0.0)
        ref = o.normals_vjp_f64(s.depth, *s.intrinsics, 2, codes, gcot)
        got = dt.grad.cpu().numpy()
        err = np.abs(got - ref)
        assert np.all(err <= vjp_tol(ref)), f"frame {i}: {err.max():.3g} vs {np.abs(ref).max():.3g}"
        worst = max(worst, float(err.max() / np.abs(ref).max()))
    log(f"differentiation batch: worst max|err|/max|grad| = {worst:.2e}")


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
@pytest.mark.parametrize("H,W", [(1, 4), (3, 8), (5, 4), (9, 12), (31, 224), (32, 228),
                                 (33, 252), (64, 448), (65, 8), (70, 256), (97, 500),
                                 (130, 996), (480, 640), (257, 1992)])
def test_vjp_vector_layout_equals_scalar_layout(alpha, H, W):
    """Rows of whole float4 groups take the vector kernels (bands of rows
    rolled per wavefront); a row stride that is not a multiple of 4 takes the
    scalar tiles.  Both sum the same four contributions in the same order,
    so the gradients agree bit for bit, at widths on and off the 224-column
    strips and heights on and off the 16- and 32-row bands."""
    import torch
    rng = np.random.default_rng(H * 7919 + W + alpha)
    d = rng.uniform(1.0, 1.3, size=(H, W)).astype(np.float32)
    d[rng.random((H, W)) < 0.02] = 0.0
    g = torch.from_numpy(rng.standard_normal((H, W, 3)).astype(np.float32)).cuda()
    fx, fy, cx, cy = 150.0, 160.0, (W - 1) / 2, (H - 1) / 2
    vec = bn.normals_vjp(to_gpu(d), fx, fy, cx, cy, g, alpha, "rel", 1.1)
    sca = bn.normals_vjp(to_gpu(d, 1), fx, fy, cx, cy, g, alpha, "rel", 1.1)
    # an output 4 bytes off 16-byte alignment also takes the scalar tiles
    buf = torch.empty(H * W + 1, dtype=torch.float32, device="cuda")
    off = bn.normals_vjp(to_gpu(d), fx, fy, cx, cy, g, alpha, "rel", 1.1,
                         grad_depth=buf[1:].view(H, W))
    torch.cuda.synchronize()
    assert torch.equal(vec.view(torch.int32), sca.view(torch.int32))
    assert torch.equal(vec.view(torch.int32), off.view(torch.int32))
    if H * W <= 70 * 256:
        o = oracle.default()
        codes = o.normals_f32(d, fx, fy, cx, cy, alpha, "rel", 1.1)["mask"]
        ref = o.normals_vjp_f64(d, fx, fy, cx, cy, alpha, codes, g.cpu().numpy().astype(np.float64))
        assert np.all(np.abs(vec.cpu().numpy() - ref) <= vjp_tol(ref))


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
@pytest.mark.parametrize("n,H,W", [(1, 480, 640), (3, 61, 252), (16, 480, 640), (40, 120, 160),
                                   (64, 240, 320)])
def test_vjp_stack_vector_layout_equals_scalar_layout(alpha, n, H, W):
    """The stack adjoint, vector kernels (frame stride a multiple of 4; bands
    of four or eight wavefronts by the size of the stack) against scalar
    tiles (row stride W + 1), bit for bit."""
    import torch
    rng = np.random.default_rng(n * 1000 + H + alpha)
    d = rng.uniform(1.0, 1.3, size=(n, H, W)).astype(np.float32)
    g = torch.from_numpy(rng.standard_normal((n, H, W, 3)).astype(np.float32)).cuda()
    intr = [(150.0 + 3 * k, 160.0, (W - 1) / 2, (H - 1) / 2) for k in range(n)]
    dv = torch.from_numpy(d).cuda()
    pad = torch.full((n, H, W + 1), float("nan"), device="cuda")
    pad[:, :, :W] = dv
    vec = bn.normals_vjp_stack(dv, intr, g, alpha, "rel", 1.1)
    sca = bn.normals_vjp_stack(pad[:, :, :W], intr, g, alpha, "rel", 1.1)
    torch.cuda.synchronize()
    assert torch.equal(vec.view(torch.int32), sca.view(torch.int32))
