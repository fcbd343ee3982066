"""The oracle's adjoint (vector-Jacobian product of the frozen normal map)
against FP64 central finite differences of the oracle's own forward map."""
import numpy as np
import pytest

import oracle
from synth import scenes

VALID = 0


def fd_vjp(o, depth, fx, fy, cx, cy, alpha, codes, gn, h=1e-6):
    """Central differences of L(d) = sum(normals(d) . gn), codes frozen."""
    d = depth.astype(np.float64).copy()
    H, W = d.shape
    out = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            keep = d[y, x]
            d[y, x] = keep + h
            lp = np.sum(o.normals_frozen_f64(d, fx, fy, cx, cy, alpha, codes) * gn)
            d[y, x] = keep - h
            lm = np.sum(o.normals_frozen_f64(d, fx, fy, cx, cy, alpha, codes) * gn)
            d[y, x] = keep
            out[y, x] = (lp - lm) / (2 * h)
    return out


def crop(seed, x0, y0, size, alpha):
    s = scenes.frame_640x480(seed=seed)
    d = np.ascontiguousarray(s.depth[y0:y0 + size, x0:x0 + size])
    return d, s.fx, s.fy, s.cx - x0, s.cy - y0


@pytest.mark.parametrize("alpha", [1, 2])
@pytest.mark.parametrize("seed,x0,y0", [(2000, 300, 200), (2003, 40, 60)])
def test_vjp_matches_finite_differences(alpha, seed, x0, y0):
    o = oracle.default()
    d, fx, fy, cx, cy = crop(seed, x0, y0, 32, alpha)
    codes = o.normals_f32(d, fx, fy, cx, cy, alpha, "rel", 4.0)["mask"]
    assert (codes == VALID).sum() > 300
    rng = np.random.default_rng(seed + alpha)
    gn = rng.standard_normal((32, 32, 3))
    g = o.normals_vjp_f64(d, fx, fy, cx, cy, alpha, codes, gn)
    g_fd = fd_vjp(o, d, fx, fy, cx, cy, alpha, codes, gn)
    scale = np.abs(g_fd).max()
    assert scale > 0
    assert np.abs(g - g_fd).max() <= 1e-7 * scale


def test_loss_gradient_against_finite_differences():
    """The differentiation workload's loss: mean over U of (1 - n.t), U =
    pixels valid in the prediction and in the noise-free target."""
    o = oracle.default()
    s = scenes.frame_640x480(seed=2001)
    x0, y0, n = 200, 150, 32
    d = np.ascontiguousarray(s.depth[y0:y0 + n, x0:x0 + n])
    dc = np.ascontiguousarray(s.depth_clean[y0:y0 + n, x0:x0 + n]).astype(np.float32)
    fx, fy, cx, cy = s.fx, s.fy, s.cx - x0, s.cy - y0
    pred = o.normals_f32(d, fx, fy, cx, cy, 2, "rel", 4.0)
    tgt = o.normals_f32(dc, fx, fy, cx, cy, 2, "rel", 4.0)
    U = (pred["mask"] == VALID) & (tgt["mask"] == VALID)
    t = tgt["normals"]

    def loss(dd):
        nn = o.normals_frozen_f64(dd, fx, fy, cx, cy, 2, pred["mask"])
        return np.sum((1.0 - np.sum(nn * t, axis=-1))[U]) / U.sum()
    gn = np.where(U[..., None], -t / U.sum(), 0.0)
    g = o.normals_vjp_f64(d, fx, fy, cx, cy, 2, pred["mask"], gn)
    dd = d.astype(np.float64)
    h = 1e-6
    for (y, x) in [(10, 10), (16, 5), (3, 20), (27, 27), (15, 16)]:
        e = np.zeros_like(dd)
        e[y, x] = h
        fd = (loss(dd + e) - loss(dd - e)) / (2 * h)
        assert abs(g[y, x] - fd) <= 1e-6 * max(abs(fd), 1e-3)
