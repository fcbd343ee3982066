"""GPU evaluation tools against the evaluation oracle: angle images
(Eqs. 14-15), their MSE, and the local plane fit (25-neighbour ground
truth of Section 4)."""
import numpy as np
import pytest

import paper_2209_08241_amd as bn
from gpu_util import log
from oracle import evaluation as oev
from synth import scenes

pytestmark = pytest.mark.gpu


def random_normals(H, W, seed):
    rng = np.random.default_rng(seed)
    n = rng.normal(size=(H, W, 3))
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    n = n.astype(np.float32)
    # axis directions, signed zeros and zero vectors in the first row
    special = [(0, 0, 1), (0, 0, -1), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 0),
               (-0.0, -0.0, -1), (-1, -0.0, 0), (1, -0.0, 0), (0.6, 0.8, 0), (-0.6, -0.8, 0)]
    for k, v in enumerate(special[:W]):
        n[0, k] = v
    return n


def circ(a, b):
    d = np.abs(a - b)
    return np.minimum(d, 2 * np.pi - d)


@pytest.mark.parametrize("H,W", [(1, 12), (37, 61), (480, 640)])
def test_angles(H, W):
    import torch
    n = random_normals(H, W, H * 31 + W)
    t, p = bn.normal_angles(torch.from_numpy(n).cuda())
    torch.cuda.synchronize()
    rt, rp = oev.angle_images(n.astype(np.float64))
    assert np.abs(t.cpu().numpy() - rt).max() <= 1e-6
    assert circ(p.cpu().numpy().astype(np.float64), rp).max() <= 1e-6
    assert float(p.min()) >= 0.0


@pytest.mark.parametrize("H,W", [(1, 1), (13, 29), (480, 640), (1080, 1920)])
def test_angle_mse(H, W):
    import torch
    rng = np.random.default_rng(H + W)
    a = random_normals(H, W, 1 + H)
    b = (a + rng.normal(scale=0.05, size=a.shape)).astype(np.float32)
    b /= np.linalg.norm(b, axis=-1, keepdims=True).clip(1e-12)
    ma = rng.choice([0, 0, 0, 1, 2], size=(H, W)).astype(np.uint8)
    mb = rng.choice([0, 0, 0, 1, 2], size=(H, W)).astype(np.uint8)
    cu = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    got = bn.angle_mse(cu(a), cu(ma), cu(b), cu(mb))
    want = oev.angle_mse(a.astype(np.float64), ma, b.astype(np.float64), mb)
    assert got[2] == want[2]
    assert abs(got[0] - want[0]) <= 1e-10 * max(want[0], 1e-300)
    assert abs(got[1] - want[1]) <= 1e-10 * max(want[1], 1e-300)
    got = bn.angle_mse(cu(a), None, cu(b), None)
    want = oev.angle_mse(a.astype(np.float64), np.zeros((H, W), np.uint8), b.astype(np.float64),
                         np.zeros((H, W), np.uint8))
    assert got[2] == want[2] == H * W
    assert abs(got[0] - want[0]) <= 1e-10 * max(want[0], 1e-300)


def _fit_compare(depth, fx, fy, cx, cy, r, pixels=None):
    import torch
    n, m = bn.plane_fit_normals(torch.from_numpy(np.ascontiguousarray(depth)).cuda(), fx, fy,
                                cx, cy, r)
    torch.cuda.synchronize()
    n, m = n.cpu().numpy(), m.cpu().numpy()
    rn, rm, eigs = oev.plane_fit(depth.astype(np.float64), fx, fy, cx, cy, r, pixels=pixels)
    if pixels is None:
        assert np.array_equal(m, rm)
        sel = rm == 0
    else:
        xs = np.array([x for x, _ in pixels])
        ys = np.array([y for _, y in pixels])
        assert np.array_equal(m[ys, xs], rm[ys, xs])
        sel = np.zeros(rm.shape, bool)
        sel[ys, xs] = rm[ys, xs] == 0
    e = eigs[sel]
    gap = (e[:, 1] - e[:, 0]) / e[:, 2]
    tol = 2e-6 + 1e-13 / np.maximum(gap, 1e-300)
    err = np.abs(n[sel].astype(np.float64) - rn[sel]).max(axis=-1)
    assert np.all(err <= tol), f"plane fit error {err.max():.3g}"
    return int(sel.sum())


@pytest.mark.parametrize("r", [1, 2, 3])
def test_plane_fit_small_scene(r):
    log(f"plane fit r={r}")
    s = scenes.make_scene(60, 80, fx=70.0, fy=74.0, cx=39.5, cy=29.0, seed=51)
    k = _fit_compare(s.depth, s.fx, s.fy, s.cx, s.cy, r)
    assert k > 1000


def test_plane_fit_640_sampled():
    s = scenes.frame_640x480(seed=1)
    pts = [(x, y) for y in range(0, 480, 9) for x in range(0, 640, 7)]
    k = _fit_compare(s.depth, *s.intrinsics, 2, pixels=pts)
    assert k > 2500


def test_plane_fit_exact_plane():
    import torch
    from pins import camera_facing_plane
    n0 = camera_facing_plane(40.0, 130.0)
    d = scenes.plane_depth(48, 64, 300.0, 320.0, 31.5, 23.5, n0, -1.8).astype(np.float32)
    n, m = bn.plane_fit_normals(torch.from_numpy(d).cuda(), 300.0, 320.0, 31.5, 23.5, 2)
    torch.cuda.synchronize()
    v = m.cpu().numpy() == 0
    assert v.sum() == (48 - 4) * (64 - 4)
    # binary32 depth: a few ulps of tilt over a 5-pixel window
    assert np.abs(n.cpu().numpy()[v] - n0).max() < 1e-4


def test_accuracy_table_small():
    """The sweep runs end to end; on noise-free depth the four-pair estimate
    is far closer to the analytic normals than on noisy depth."""
    from paper_2209_08241_amd import evaluate
    rows = evaluate.accuracy_table(frames=1, noise_levels=(0.0, 0.002),
                                   configs=[("four_pair", 2, 0), ("pair_removal", 2, 0),
                                            ("multiscale", 1, 2)], H=96, W=128)
    assert len(rows) == 6
    by = {(r["noise_k"], r["method"]): r for r in rows}
    assert by[(0.0, "four_pair")]["mse_theta"] < 0.1 * by[(0.002, "four_pair")]["mse_theta"]
    for r in rows:
        assert 0.5 < r["coverage"] <= 1.0
        assert r["mse_theta"] >= 0 and r["mse_phi_fit"] >= 0
