"""GPU parity of the plain entry point (bn_estimate_normals) against the
oracle: masks and counts bit-exact, normals within 1e-5 per component."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2209_08241_amd as bn
from gpu_util import assert_parity, check_frame, gpu_normals, log, to_gpu
from synth import scenes

pytestmark = pytest.mark.gpu

ALL_VARIANTS = [1, 2, 3, 4, 5, 6, 7]


@pytest.fixture(scope="module")
def f640():
    return scenes.frame_640x480(seed=1)


@pytest.fixture(scope="module")
def f1080():
    return scenes.frame_1920x1080(seed=2)


def test_library_is_native():
    import torch
    assert torch.cuda.is_available()
    assert bn.lib().bn_version() == 3
    names = dict(bn.variants())
    assert names[1] == "scalar" and names[2] == "vec4"


@pytest.mark.parametrize("alpha", [1, 2, 3])
@pytest.mark.parametrize("mode,tau", [("rel", 4.0), ("abs", 2e-4), ("none", 1.0)])
@pytest.mark.parametrize("variant", [0] + ALL_VARIANTS)
def test_640x480(f640, alpha, mode, tau, variant):
    log(f"640x480 alpha={alpha} mode={mode} variant={variant}")
    s = f640
    check_frame(s.depth, *s.intrinsics, alpha, mode, tau, variant, what="640x480")


@pytest.mark.parametrize("alpha", [1, 2, 8])
@pytest.mark.parametrize("variant", [0] + ALL_VARIANTS)
def test_1920x1080(f1080, alpha, variant):
    log(f"1920x1080 alpha={alpha} variant={variant}")
    s = f1080
    check_frame(s.depth, *s.intrinsics, alpha, "rel", 4.0, variant, what="1920x1080")


@pytest.mark.parametrize("alpha", range(1, 9))
def test_every_alpha(f640, alpha):
    log(f"alpha sweep {alpha}")
    s = f640
    check_frame(s.depth, *s.intrinsics, alpha, "rel", 3.0, 0, what=f"alpha={alpha}")



def test_count_parts_around_the_direct_root():
    """The count reduction sends the last 31 parts of a frame (in dispatch
    order) straight to the root word and the others through 32 slot words:
    frames whose part counts sit on either side of those boundaries (1, 31,
    32, 33, 62, 63, 64 and 95 tiles of 1024 pixels, and so 4 times as many
    scalar parts) give the oracle's counts in every tile shape."""
    rng = np.random.default_rng(11)
    for H in (1, 31, 32, 33, 62, 63, 64, 95):
        W = 1024
        d = (1.0 + 0.01 * np.arange(W, dtype=np.float32)[None, :]
             + 0.05 * rng.standard_normal((H, W)).astype(np.float32)).astype(np.float32)
        d[rng.random((H, W)) < 0.03] = 0.0
        for variant in [0] + ALL_VARIANTS:
            log(f"count parts: {H}x{W} v={variant}")
            check_frame(d, 800.0, 800.0, 511.5, H / 2.0, 1, "rel", 2.0, variant,
                        what=f"parts {H}x{W} v={variant}")

@pytest.mark.parametrize("W", [1, 2, 3, 4, 5, 7, 8, 9, 12, 13, 17, 31, 33, 64, 65, 127, 129,
                               255, 257, 1023, 1025, 1028])
@pytest.mark.parametrize("H", [1, 2, 3, 5, 17, 33])
def test_ragged_shapes(H, W):
    rng = np.random.default_rng(H * 10007 + W)
    d = rng.uniform(0.8, 1.2, size=(H, W)).astype(np.float32)
    d[rng.random((H, W)) < 0.05] = 0.0
    fx, fy, cx, cy = 300.0, 310.0, (W - 1) / 2, (H - 1) / 2
    for alpha in (1, 2, 3):
        for variant in [0] + ALL_VARIANTS:
            if variant and not _supported(variant, W):
                continue
            check_frame(d, fx, fy, cx, cy, alpha, "rel", 1.02, variant,
                        what=f"{H}x{W} a={alpha} v={variant}")


def _supported(variant, W, stride=None):
    import torch
    stride = W if stride is None else stride
    d = torch.empty(max(stride, 4) * 2, dtype=torch.float32, device="cuda")
    n = torch.empty(max(W, 4) * 3 * 2, dtype=torch.float32, device="cuda")
    m = torch.empty(max(W, 4) * 2, dtype=torch.uint8, device="cuda")
    return bool(bn.lib().bn_variant_supported(variant, ctypes.c_void_p(d.data_ptr()), 2, W,
                                              stride, ctypes.c_void_p(n.data_ptr()),
                                              ctypes.c_void_p(m.data_ptr())))


@pytest.mark.parametrize("pad", [1, 3, 4, 64])
def test_strided_rows(f640, pad):
    s = f640
    for variant in [0] + ALL_VARIANTS:
        if variant and not _supported(variant, 640, 640 + pad):
            continue
        check_frame(s.depth, *s.intrinsics, 2, "rel", 4.0, variant, stride_pad=pad,
                    what=f"stride pad {pad} v={variant}")


SPECIALS = np.array([0.0, -0.0, -1.0, np.nan, np.inf, -np.inf, 1e-40, 1e-45, 1e30, 1e-30, 1e8,
                     3.4e38, 1e-20, 1e12], dtype=np.float32)


@pytest.mark.parametrize("alpha", [1, 2, 5])
@pytest.mark.parametrize("mode,tau", [("rel", 4.0), ("abs", 1e-3), ("none", 1.0)])
def test_special_values(alpha, mode, tau):
    rng = np.random.default_rng(alpha)
    H, W = 37, 68
    d = rng.uniform(0.5, 4.0, size=(H, W)).astype(np.float32)
    idx = rng.random((H, W)) < 0.15
    d[idx] = rng.choice(SPECIALS, size=int(idx.sum()))
    for variant in [0] + ALL_VARIANTS:
        check_frame(d, 200.0, 210.0, 33.5, 18.0, alpha, mode, tau, variant,
                    what=f"specials a={alpha} {mode} v={variant}")


def test_uniform_special_frames():
    for v in SPECIALS:
        d = np.full((9, 12), v, dtype=np.float32)
        for variant in [0] + ALL_VARIANTS:
            check_frame(d, 100.0, 100.0, 5.5, 4.0, 1, "rel", 4.0, variant, what=f"all {v}")


def test_wide_dynamic_range():
    """Log-uniform depths over 7 decades (REL and ABS)."""
    rng = np.random.default_rng(99)
    d = (10.0 ** rng.uniform(-3, 4, size=(64, 96))).astype(np.float32)
    # smooth patches so that some pixels are VALID
    d[10:40, 20:60] = np.float32(2.5)
    d[45:60, 5:90] = (1.0 + 0.001 * np.arange(85, dtype=np.float32))[None, :]
    for mode, tau in (("rel", 4.0), ("abs", 0.5)):
        for variant in [0] + ALL_VARIANTS:
            check_frame(d, 400.0, 380.0, 47.5, 31.5, 2, mode, tau, variant,
                        what=f"wide range {mode} v={variant}")


def test_empty_frames():
    import torch
    for H, W in ((0, 0), (0, 16), (16, 0)):
        d = torch.empty((H, W), dtype=torch.float32, device="cuda")
        n, m, st = bn.estimate_normals(d, 500.0, 500.0, 1.0, 1.0)
        torch.cuda.synchronize()
        assert n.shape == (H, W, 3) and m.shape == (H, W)
        assert not st.cpu().any()


def test_deterministic_and_variant_invariant(f1080):
    s = f1080
    outs = []
    for variant in ALL_VARIANTS + [0, 0]:
        n, m, st = gpu_normals(s.depth, *s.intrinsics, 2, "rel", 4.0, variant)
        outs.append((n, m, st))
    n0, m0, s0 = outs[0]
    for n, m, st in outs[1:]:
        assert np.array_equal(n.view(np.uint32), n0.view(np.uint32))
        assert np.array_equal(m, m0)
        assert np.array_equal(st, s0)


def test_stats_store_and_accumulate(f640):
    """Counts are stored by default (over whatever the 16 bytes held, the
    reserved word included) and added with the accumulate flag; every
    variant, repeated calls on one stream (whose work area each call leaves
    zero) and a second stream give the same counts."""
    import torch
    s = f640
    d = to_gpu(s.depth)
    ref = [int(c) for c in oracle.normals_f32(s.depth, *s.intrinsics, 2)["counts"]]
    side = torch.cuda.Stream()
    for variant in [0] + ALL_VARIANTS:
        st = torch.full((4,), -5, dtype=torch.int32, device="cuda")
        for _ in range(3):
            bn.estimate_normals(d, *s.intrinsics, 2, stats=st, variant=variant)
        torch.cuda.synchronize()
        assert st.cpu().tolist() == ref + [0], f"variant {variant}: stored counts"
        acc = bn.new_stats()
        for _ in range(3):
            bn.estimate_normals(d, *s.intrinsics, 2, stats=acc, variant=variant,
                                accumulate_counts=True)
        with torch.cuda.stream(side):
            bn.estimate_normals(d, *s.intrinsics, 2, stats=acc, variant=variant,
                                accumulate_counts=True, stream=side)
        torch.cuda.synchronize()
        assert acc.cpu().tolist() == [4 * c for c in ref] + [0], f"variant {variant}: added"


def test_argument_errors():
    import torch
    d = torch.ones((8, 8), dtype=torch.float32, device="cuda")
    n = torch.zeros((8, 8, 3), dtype=torch.float32, device="cuda")
    m = torch.full((8, 8), 7, dtype=torch.uint8, device="cuda")
    dp, np_, mp = d.data_ptr(), n.data_ptr(), m.data_ptr()
    P = bn.make_params
    cases = [
        (P(alpha=0), (dp, 8, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(alpha=9), (dp, 8, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_UNSUPPORTED),
        (P(tau=0.0), (dp, 8, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(tau=float("nan")), (dp, 8, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(mode=7), (dp, 8, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(variant=99), (dp, 8, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(), (dp, 8, 8, 7, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(), (dp, 8, 8, 8, 0.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(), (dp, 8, 8, 8, 500.0, float("inf"), 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(), (dp, 8, 8, 8, 500.0, 500.0, float("nan"), 3.5), bn.BN_ERR_INVALID_ARG),
        (P(), (0, 8, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(), (dp, -1, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_INVALID_ARG),
        (P(), (dp, 8, 70000, 70000, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_UNSUPPORTED),
        (P(variant=2), (dp + 4, 7, 8, 8, 500.0, 500.0, 3.5, 3.5), bn.BN_ERR_UNSUPPORTED),
    ]
    for params, (ptr, H, W, stride, fx, fy, cx, cy), want in cases:
        rc = bn.raw_estimate_normals(ptr, H, W, stride, fx, fy, cx, cy, params, np_, mp, 0)
        assert rc == want, (params.alpha, params.mask_mode, params.tau, params.variant, H, W, rc)
    torch.cuda.synchronize()
    # nothing was written by any rejected call
    assert torch.all(m == 7) and torch.all(n == 0)


def test_max_pixels_sampled():
    """The largest frame the entry point accepts (2^28 pixels, width 65536),
    checked against the oracle on sampled row bands."""
    import torch
    H, W = 4096, 65536
    rng = np.random.default_rng(5)
    log("max-size frame: generating")
    base = rng.uniform(1.0, 3.0, size=(1, W)).astype(np.float32)
    d = torch.from_numpy(base).cuda().repeat(H, 1)
    d += torch.linspace(0, 1, H, device="cuda")[:, None]
    holes = torch.rand((H, W), device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    d[holes < 0.02] = 0.0
    fx, fy, cx, cy = 20000.0, 20000.0, 32767.5, 2047.5
    n, m, st = bn.estimate_normals(d, fx, fy, cx, cy, 2, "rel", 4.0)
    torch.cuda.synchronize()
    total = [int(v) for v in st.cpu()[:3]]
    assert sum(total) == H * W
    for (y0, y1) in ((0, 6), (2045, 2052), (4090, 4096)):
        r0, r1 = max(0, y0 - 2), min(H, y1 + 2)
        band = d[r0:r1].cpu().numpy()
        # the band carries the alpha rows the sampled rows read; shifting cy by
        # the integer r0 keeps every binary32 y - cy bit-identical
        ref = oracle.default().normals_f32_rows(
            np.ascontiguousarray(band), fx, fy, cx, cy - r0, 2, "rel", 4.0,
            y0 - r0, y1 - r0)
        got_n = n[y0:y1].cpu().numpy()
        got_m = m[y0:y1].cpu().numpy()
        assert_parity(ref, got_n, got_m, what=f"rows {y0}:{y1}")


def test_max_pixels_counts_and_variants():
    """The 2^28-pixel frame, a smooth surface with steps and holes: the
    four-pair counts equal the oracle's exactly (the oracle's row entry band by
    band over the whole frame), and pair removal and multi-scale (alpha 2, K 2)
    match the oracle on sampled row bands.  The surface is smooth at the pixel
    spacing, so the per-scale normals of multi-scale point the same way; where
    noise dominates instead, their sum can cancel and the binary32 error grows
    with the cancellation, which the boundary test does not bound."""
    import torch
    H, W = 4096, 65536
    log("max-size frame (counts, variants): generating")
    x = torch.arange(W, device="cuda", dtype=torch.float64)[None, :]
    y = torch.arange(H, device="cuda", dtype=torch.float64)[:, None]
    d = (1.5 + x / W + 0.5 * y / H
         + 0.1 * torch.sin(2 * np.pi * x / 6000) * torch.sin(2 * np.pi * y / 700)
         + 0.4 * (torch.div(x, 5000, rounding_mode="floor")
                  + torch.div(y, 600, rounding_mode="floor")).remainder(2)).float()
    del x, y
    holes = torch.rand((H, W), device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    d[holes < 0.02] = 0.0
    del holes
    fx, fy, cx, cy = 20000.0, 20000.0, 32767.5, 2047.5
    normals = torch.empty((H, W, 3), device="cuda")
    mask = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    st = bn.new_stats(device="cuda")
    bn.estimate_normals(d, fx, fy, cx, cy, 2, "rel", 4.0, normals=normals, mask=mask, stats=st)
    torch.cuda.synchronize()
    got = [int(v) for v in st.cpu()[:3]]
    want = np.zeros(3, dtype=np.uint64)
    step = 512
    for y0 in range(0, H, step):
        y1 = min(H, y0 + step)
        r0, r1 = max(0, y0 - 2), min(H, y1 + 2)
        band = np.ascontiguousarray(d[r0:r1].cpu().numpy())
        ref = oracle.default().normals_f32_rows(band, fx, fy, cx, cy - r0, 2, "rel", 4.0,
                                                y0 - r0, y1 - r0)
        want += ref["counts"]
    log(f"max-size counts: gpu {got}, oracle {[int(c) for c in want]}")
    assert got == [int(c) for c in want]
    assert min(got) > H * W // 20, "the frame should mix all three codes"
    for method, K, reach in (("pair_removal", 0, 2), ("multiscale", 2, 4)):
        log(f"max-size {method}")
        bn.estimate_normals(d, fx, fy, cx, cy, 2, "rel", 4.0, method=method, scales=K,
                            normals=normals, mask=mask, stats=st)
        torch.cuda.synchronize()
        for (y0, y1) in ((0, 6), (2045, 2052), (4088, 4096)):
            r0, r1 = max(0, y0 - reach), min(H, y1 + reach)
            band = np.ascontiguousarray(d[r0:r1].cpu().numpy())
            ref = oracle.variant_f32(band, fx, fy, cx, cy - r0, 2, "rel", 4.0, method=method,
                                     scales=K, rows=(y0 - r0, y1 - r0))
            assert_parity(ref, normals[y0:y1].cpu().numpy(), mask[y0:y1].cpu().numpy(),
                          what=f"{method} rows {y0}:{y1}")
