"""GPU parity of the pair-removal and multi-scale methods against the
oracle (masks and counts bit-exact, normals within 1e-5 per component), the
batched form of each against its plain form (bit for bit), and the
store / accumulate semantics of the counts."""
import numpy as np
import pytest

import oracle
import paper_2209_08241_amd as bn
from gpu_util import NORMAL_TOL, assert_parity, log, to_gpu
from synth import scenes

pytestmark = pytest.mark.gpu

PR, MS = "pair_removal", "multiscale"


@pytest.fixture(scope="module")
def f640():
    return scenes.frame_640x480(seed=1)


@pytest.fixture(scope="module")
def f1080():
    return scenes.frame_1920x1080(seed=2)


def run(depth, fx, fy, cx, cy, alpha, mode, tau, method, scales=0, variant=0, stride_pad=0):
    import torch
    d = to_gpu(depth, stride_pad)
    n, m, st = bn.estimate_normals(d, fx, fy, cx, cy, alpha, mode, tau, variant=variant,
                                   method=method, scales=scales)
    torch.cuda.synchronize()
    return n.cpu().numpy(), m.cpu().numpy(), st.cpu().numpy()


def check(depth, fx, fy, cx, cy, alpha, mode, tau, method, scales=0, variant=0, stride_pad=0,
          what=""):
    ref = oracle.variant_f32(depth, fx, fy, cx, cy, alpha, mode, tau, method=method,
                             scales=scales)
    n, m, st = run(depth, fx, fy, cx, cy, alpha, mode, tau, method, scales, variant, stride_pad)
    return assert_parity(ref, n, m, st, what=what)


@pytest.mark.parametrize("alpha", [1, 2, 3, 8])
@pytest.mark.parametrize("mode,tau", [("rel", 4.0), ("rel", 1.5), ("abs", 1e-3), ("none", 1.0)])
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_pair_removal_640(f640, alpha, mode, tau, variant):
    log(f"pair removal 640x480 alpha={alpha} {mode} {tau} variant={variant}")
    s = f640
    check(s.depth, *s.intrinsics, alpha, mode, tau, PR, 0, variant, what="pair removal")


@pytest.mark.parametrize("alpha,K", [(1, 1), (1, 3), (2, 2), (2, 4), (3, 2), (4, 2), (8, 1),
                                     (1, 8), (2, 5), (2, 8), (3, 3), (3, 5), (4, 4), (5, 3),
                                     (7, 2), (8, 2), (3, 6), (8, 8)])
@pytest.mark.parametrize("mode,tau", [("rel", 4.0), ("abs", 5e-3), ("none", 1.0)])
def test_multiscale_640(f640, alpha, K, mode, tau):
    """Every variant the offsets allow against the oracle, and the vector
    tiles against the scalar tiles bit for bit."""
    log(f"multiscale 640x480 alpha={alpha} K={K} {mode}")
    s = f640
    variants = (0, 1, 2, 3, 4) if alpha * K <= 16 else (0, 1)
    scalar = run(s.depth, *s.intrinsics, alpha, mode, tau, MS, K, 1)
    for variant in variants:
        check(s.depth, *s.intrinsics, alpha, mode, tau, MS, K, variant,
              what=f"multiscale a={alpha} K={K} v={variant}")
        got = run(s.depth, *s.intrinsics, alpha, mode, tau, MS, K, variant)
        for a, b in zip(got, scalar):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"v={variant}"
    # the pipelined pair of tiles and the small workgroups serve the five-tap
    # methods only
    for v in (5, 6, 7):
        with pytest.raises(bn.BnError) as e:
            run(s.depth, *s.intrinsics, alpha, mode, tau, MS, K, v)
        assert e.value.status == bn.BN_ERR_UNSUPPORTED


@pytest.mark.parametrize("alpha,K", [(3, 3), (2, 5), (8, 2), (1, 8), (3, 6), (8, 3), (5, 4)])
def test_multiscale_vector_variants_need_short_reach(f640, alpha, K):
    """Vector tiles serve alpha * K <= 16 only; beyond it the request for one
    is refused and the automatic choice is the scalar tile."""
    import torch
    s = f640
    d = to_gpu(s.depth)
    for v in (2, 3, 4):
        if alpha * K <= 16:
            bn.estimate_normals(d, *s.intrinsics, alpha, method=MS, scales=K, variant=v)
            continue
        with pytest.raises(bn.BnError) as e:
            bn.estimate_normals(d, *s.intrinsics, alpha, method=MS, scales=K, variant=v)
        assert e.value.status == bn.BN_ERR_UNSUPPORTED
    torch.cuda.synchronize()


@pytest.mark.parametrize("method,alpha,K", [(PR, 2, 0), (PR, 1, 0), (MS, 1, 3), (MS, 2, 2)])
def test_1920x1080_sampled_rows(f1080, method, alpha, K):
    """Full frame on the GPU, row bands of it against the oracle's row entry."""
    log(f"1080p {method} alpha={alpha} K={K}")
    s = f1080
    n, m, st = run(s.depth, *s.intrinsics, alpha, "rel", 4.0, method, K)
    H = s.depth.shape[0]
    full = oracle.variant_f32(s.depth, *s.intrinsics, alpha, "rel", 4.0, method=method, scales=K)
    assert [int(c) for c in st[:3]] == [int(c) for c in full["counts"]]
    for (rb, re) in ((0, 24), (H // 2 - 8, H // 2 + 8), (H - 24, H)):
        ref = oracle.variant_f32(s.depth, *s.intrinsics, alpha, "rel", 4.0, method=method,
                                 scales=K, rows=(rb, re))
        assert_parity(ref, n[rb:re], m[rb:re], what=f"rows {rb}..{re}")


@pytest.mark.parametrize("H,W", [(1, 1), (3, 5), (5, 3), (17, 33), (33, 17), (9, 1025),
                                 (31, 129), (2, 2048), (64, 4), (11, 12), (19, 260), (7, 1028)])
def test_ragged_and_strided(H, W):
    rng = np.random.default_rng(H * 7919 + W)
    d = rng.uniform(0.8, 1.3, size=(H, W)).astype(np.float32)
    d[rng.random((H, W)) < 0.04] = 0.0
    fx, fy, cx, cy = 280.0, 300.0, (W - 1) / 2, (H - 1) / 2
    for pad in (0, 3):
        for alpha in (1, 2):
            check(d, fx, fy, cx, cy, alpha, "rel", 1.05, PR, 0, 0, pad,
                  what=f"pairs {H}x{W} a={alpha} pad={pad}")
            check(d, fx, fy, cx, cy, alpha, "rel", 1.05, MS, 2, 0, pad,
                  what=f"ms {H}x{W} a={alpha} pad={pad}")


def test_special_values():
    rng = np.random.default_rng(5)
    H, W = 40, 64
    d = rng.uniform(0.5, 3.0, size=(H, W)).astype(np.float32)
    specials = [0.0, -0.0, -1.0, np.nan, np.inf, -np.inf, 1e-40, 1e30,
                np.finfo(np.float32).max, 1e-20]
    for k, v in enumerate(specials):
        d[rng.integers(H), rng.integers(W)] = v
        d[rng.integers(H), rng.integers(W)] = v
    d[5, :] *= 1e6
    d[9, :] *= 1e-6
    for method, K in ((PR, 0), (MS, 1), (MS, 3)):
        for mode, tau in (("rel", 4.0), ("abs", 1e-4), ("none", 1.0)):
            check(d, 120.0, 125.0, 31.5, 19.5, 1, mode, tau, method, K,
                  what=f"special {method} K={K} {mode}")


def test_step_scene_pairs_keep_own_plane():
    """Next to a step the pair-removal normal is the exact normal of the
    pixel's own plane (to binary32 rounding), where the four-pair method
    removes the pixel."""
    import pins_variants as pv
    H, W = 30, 34
    fx, fy, cx, cy = 250.0, 270.0, 15.5, 13.0
    d, lab, nrm = pv._step_scene(H, W, fx, fy, cx, cy)
    f = d.astype(np.float32)
    n, m, _ = run(f, fx, fy, cx, cy, 1, "rel", 4.0, PR)
    n4, m4, _ = run(f, fx, fy, cx, cy, 1, "rel", 4.0, "four_pair")
    v = m == 0
    assert (v & (m4 == 1)).sum() > 30
    err = np.abs(n[v].astype(np.float64) - nrm[lab[v]]).max()
    assert err <= 4 * 2.0 ** -24 * max(fx, fy) + NORMAL_TOL


@pytest.mark.parametrize("method,alpha,K", [(PR, 2, 0), (MS, 1, 3), (MS, 3, 3), ("four_pair", 2, 0)])
def test_batch_equals_plain(method, alpha, K):
    import torch
    frames_h = [scenes.sized_frame(H, W, 40 + k) for k, (H, W) in
                enumerate([(240, 320), (480, 640), (120, 160), (97, 131), (480, 640)])]
    dev = torch.device("cuda")
    frames = [bn.BatchFrame(torch.from_numpy(s.depth).to(dev), s.fx, s.fy, s.cx, s.cy)
              for s in frames_h]
    with bn.BatchPlan(frames, alpha, "rel", 4.0, method=method, scales=K) as plan:
        plan.run()
        torch.cuda.synchronize()
        for s, fr in zip(frames_h, frames):
            n, m, st = run(s.depth, s.fx, s.fy, s.cx, s.cy, alpha, "rel", 4.0, method, K)
            assert np.array_equal(fr.mask.cpu().numpy(), m)
            assert np.array_equal(fr.normals.cpu().numpy(), n)
            assert fr.stats[:3].cpu().tolist() == st[:3].tolist()
        ref = oracle.variant_f32(frames_h[1].depth, *frames_h[1].intrinsics, alpha, "rel", 4.0,
                                 method=method, scales=K)
        assert_parity(ref, frames[1].normals.cpu().numpy(), frames[1].mask.cpu().numpy(),
                      frames[1].stats.cpu().numpy(), what="batch frame 1")


@pytest.mark.parametrize("method,K", [("four_pair", 0), (PR, 0), (MS, 2)])
def test_counts_store_and_accumulate_flag(f640, method, K):
    """Stored by default, added with BN_FLAG_COUNTS_ACCUMULATE (plain and
    batched)."""
    import torch
    s = f640
    d = to_gpu(s.depth)
    ref = oracle.variant_f32(s.depth, *s.intrinsics, 2, "rel", 4.0, method=method, scales=K)
    want = [int(c) for c in ref["counts"]]
    st = bn.new_stats(device="cuda")
    for _ in range(3):
        bn.estimate_normals(d, *s.intrinsics, 2, method=method, scales=K, stats=st,
                            accumulate_counts=True)
    torch.cuda.synchronize()
    assert st[:3].cpu().tolist() == [3 * c for c in want]
    for _ in range(3):
        bn.estimate_normals(d, *s.intrinsics, 2, method=method, scales=K, stats=st)
    torch.cuda.synchronize()
    assert st[:3].cpu().tolist() == want
    fr = bn.BatchFrame(d, *s.intrinsics)
    with bn.BatchPlan([fr], 2, "rel", 4.0, method=method, scales=K) as plan:
        for _ in range(3):
            plan.run()
        torch.cuda.synchronize()
        assert fr.stats[:3].cpu().tolist() == want


def _median_rho_sphere(H, W, fx, fy, cx, cy, scale=1.0):
    """A sphere filling the frame (binary32 depth, scaled), and the median
    four-pair rho of its interior pixels: at that tau many pair and
    multi-scale decisions sit near the threshold."""
    depth, _ = scenes.sphere_depth(H, W, fx, fy, cx, cy, (0.05, -0.04, 1.2), 0.7)
    assert np.all(np.isfinite(depth))
    d32 = (depth * scale).astype(np.float32)
    rho = oracle.variant_f64(d32.astype(np.float64), fx, fy, cx, cy, 2, "rel", 1e6,
                             method="four_pair", want_rho=True)["rho"]
    return d32, float(np.median(rho[2:H - 2, 2:W - 2]))


@pytest.mark.parametrize("variant", [0, 1, 2, 5])
@pytest.mark.parametrize("method,alpha,K", [(PR, 1, 0), (PR, 2, 0), (MS, 1, 3), (MS, 2, 2)])
def test_fused_sequences_near_threshold(method, alpha, K, variant):
    """The fused binary32 sequences of pair removal and multi-scale decide
    exactly as the oracle's where many decisions sit near tau (a sphere with
    tau at its median rho, and tau 1e-3 either side of it)."""
    H, W, fx, fy, cx, cy = 96, 128, 140.0, 128.0, 63.5, 47.0
    d, tau = _median_rho_sphere(H, W, fx, fy, cx, cy)
    for t in (tau, tau * (1 - 1e-3), tau * (1 + 1e-3)):
        log(f"near threshold {method} alpha={alpha} K={K} variant={variant} tau={t:.6g}")
        v = variant if (method == PR or variant in (0, 1, 2)) else 0
        check(d, fx, fy, cx, cy, alpha, "rel", t, method, K, v, what="near threshold")


@pytest.mark.parametrize("method,alpha,K,scales", [(PR, 1, 0, (3e9, 4e9, 4.5e9, 7e9)),
                                                   (MS, 1, 2, (3e9, 3.5e9))])
def test_fused_sequences_at_overflow(method, alpha, K, scales):
    """Depths scaled (|m|^2 grows as depth^4) so that the squared lengths of
    the pairs and of the kept vectors straddle FLT_MAX: the INVALID pixels
    (binary32 overflow) and the decisions beside them are the oracle's."""
    H, W, fx, fy, cx, cy = 64, 80, 90.0, 84.0, 39.5, 31.0
    d, tau = _median_rho_sphere(H, W, fx, fy, cx, cy)
    for scale in scales:
        ds = (d.astype(np.float64) * scale).astype(np.float32)
        ref = oracle.variant_f32(ds, fx, fy, cx, cy, alpha, "rel", tau, method=method,
                                 scales=K)
        log(f"overflow {method} alpha={alpha} scale={scale:g} "
            f"invalid={int((ref['mask'] == 2).sum())}")
        n, m, st = run(ds, fx, fy, cx, cy, alpha, "rel", tau, method, K)
        assert np.array_equal(m, ref["mask"]), f"masks differ at scale {scale:g}"
        assert st[:3].tolist() == [int(c) for c in ref["counts"]]
