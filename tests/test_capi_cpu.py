"""The C-ABI library on the CPU: it loads, exports every function that
include/bnormals.h declares, and rejects bad arguments before any HIP call
(so no GPU is needed for these)."""
import ctypes
import os
import re

import pytest

import paper_2209_08241_amd as bn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bnormals.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w ]*?\**\s*\b(bn_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for want in ("bn_estimate_normals", "bn_batch_plan_create", "bn_batch_plan_update",
                 "bn_batch_run", "bn_batch_launch", "bn_batch_plan_destroy", "bn_status_string", "bn_version"):
        assert want in names


def test_library_exports_every_declared_symbol():
    L = bn.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"


def test_struct_sizes_match_header():
    assert ctypes.sizeof(bn.Params) == 32
    assert ctypes.sizeof(bn.FrameStats) == bn.STATS_BYTES == 16 and bn.STATS_WORDS == 4
    assert ctypes.sizeof(bn.Frame) == 64


def test_version_and_status_strings():
    L = bn.lib()
    assert L.bn_version() == 3
    for s in range(5):
        assert L.bn_status_string(s)
    assert L.bn_status_string(99) == b"unknown status"
    assert L.bn_variant_count() >= 2
    assert L.bn_variant_name(0) is None and L.bn_variant_name(1) == b"scalar"


@pytest.mark.parametrize("kw,dims,want", [
    (dict(alpha=0), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(alpha=9), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_UNSUPPORTED),
    (dict(tau=0.0), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(tau=float("inf")), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(mode=3), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(variant=17), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(method=3), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(method=-1), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(method="four_pair", scales=2), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(method="pair_removal", scales=3), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(method="multiscale", scales=0), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(method="multiscale", scales=9), (8, 8, 8, 500.0, 500.0), bn.BN_ERR_UNSUPPORTED),
    (dict(method="multiscale", alpha=3, scales=6, variant=2), (8, 8, 8, 500.0, 500.0),
     bn.BN_ERR_UNSUPPORTED),
    (dict(method="multiscale", alpha=5, scales=4, variant=4), (8, 8, 8, 500.0, 500.0),
     bn.BN_ERR_UNSUPPORTED),
    (dict(), (8, 8, 7, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(), (-1, 8, 8, 500.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(), (8, 8, 8, -5.0, 500.0), bn.BN_ERR_INVALID_ARG),
    (dict(), (8, 8, 8, 500.0, float("nan")), bn.BN_ERR_INVALID_ARG),
    (dict(), (8, 65537, 65537, 500.0, 500.0), bn.BN_ERR_UNSUPPORTED),
    (dict(), (1 << 15, 1 << 14, 1 << 14, 500.0, 500.0), bn.BN_ERR_UNSUPPORTED),
])
def test_argument_errors_before_launch(kw, dims, want):
    H, W, stride, fx, fy = dims
    p = bn.make_params(**kw)
    # fake, never-dereferenced addresses: validation fails before any HIP call
    rc = bn.raw_estimate_normals(0x10000, H, W, stride, fx, fy, 3.5, 3.5, p, 0x20000, 0x30000, 0)
    assert rc == want


def test_flags_and_reserved_checked():
    p = bn.make_params()
    p.flags = 2
    assert bn.raw_estimate_normals(0x10000, 8, 8, 8, 500.0, 500.0, 3.5, 3.5, p, 0x20000,
                                   0x30000, 0) == bn.BN_ERR_INVALID_ARG
    p = bn.make_params(accumulate_counts=True)
    assert p.flags == bn.FLAG_COUNTS_ACCUMULATE
    p.reserved = 1
    assert bn.raw_estimate_normals(0x10000, 8, 8, 8, 500.0, 500.0, 3.5, 3.5, p, 0x20000,
                                   0x30000, 0) == bn.BN_ERR_INVALID_ARG


def test_adjoint_only_for_the_four_pair_method():
    L = bn.lib()
    for method, scales in (("pair_removal", 0), ("multiscale", 2)):
        p = bn.make_params(method=method, scales=scales)
        rc = L.bn_normals_vjp(ctypes.c_void_p(0x10000), 8, 8, 8, ctypes.c_float(500.0),
                              ctypes.c_float(500.0), ctypes.c_float(3.5), ctypes.c_float(3.5),
                              ctypes.byref(p), ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000),
                              None)
        assert rc == bn.BN_ERR_UNSUPPORTED


def test_adjoint_alignment_checked_before_launch():
    L = bn.lib()
    p = bn.make_params()
    for depth, gn, gd in ((0x10002, 0x20000, 0x30000), (0x10000, 0x20002, 0x30000),
                          (0x10000, 0x20000, 0x30002)):
        rc = L.bn_normals_vjp(ctypes.c_void_p(depth), 8, 8, 8, ctypes.c_float(500.0),
                              ctypes.c_float(500.0), ctypes.c_float(3.5), ctypes.c_float(3.5),
                              ctypes.byref(p), ctypes.c_void_p(gn), ctypes.c_void_p(gd), None)
        assert rc == bn.BN_ERR_INVALID_ARG, (hex(depth), hex(gn), hex(gd))


def test_null_pointers_rejected():
    p = bn.make_params()
    assert bn.raw_estimate_normals(0, 8, 8, 8, 500.0, 500.0, 1.0, 1.0, p, 0x20000, 0x30000, 0) \
        == bn.BN_ERR_INVALID_ARG
    assert bn.raw_estimate_normals(0x10000, 8, 8, 8, 500.0, 500.0, 1.0, 1.0, p, 0, 0x30000, 0) \
        == bn.BN_ERR_INVALID_ARG
    assert bn.raw_estimate_normals(0x10000, 8, 8, 8, 500.0, 500.0, 1.0, 1.0, p, 0x20000, 0, 0) \
        == bn.BN_ERR_INVALID_ARG
    assert bn.lib().bn_estimate_normals(0x10000, 8, 8, 8, 500.0, 500.0, 1.0, 1.0, None,
                                        0x20000, 0x30000, 0, 0) == bn.BN_ERR_INVALID_ARG


def test_empty_frame_is_a_no_op():
    p = bn.make_params()
    assert bn.raw_estimate_normals(0, 0, 0, 0, 500.0, 500.0, 1.0, 1.0, p, 0, 0, 0) == bn.BN_OK


def test_batch_plan_argument_errors():
    L = bn.lib()
    h = ctypes.c_void_p()
    p = bn.make_params()
    assert L.bn_batch_plan_create(None, 1, ctypes.byref(p), ctypes.byref(h)) == bn.BN_ERR_INVALID_ARG
    assert h.value is None
    fr = (bn.Frame * 1)(bn.Frame(0x10000, 8, 8, 8, 500.0, 500.0, 3.5, 3.5, 0x20000, 0x30000, 0))
    assert L.bn_batch_plan_create(fr, 0, ctypes.byref(p), ctypes.byref(h)) == bn.BN_ERR_INVALID_ARG
    bad = bn.make_params(alpha=0)
    assert L.bn_batch_plan_create(fr, 1, ctypes.byref(bad), ctypes.byref(h)) == bn.BN_ERR_INVALID_ARG
    forced = bn.make_params(variant=2)
    assert L.bn_batch_plan_create(fr, 1, ctypes.byref(forced), ctypes.byref(h)) == bn.BN_ERR_UNSUPPORTED
    assert L.bn_batch_run(None, None) == bn.BN_ERR_INVALID_ARG
    assert L.bn_batch_launch(None, None) == bn.BN_ERR_INVALID_ARG
    L.bn_batch_plan_destroy(None)


def test_eval_argument_errors():
    L = bn.lib()
    assert L.bn_plane_fit_normals(ctypes.c_void_p(0x10000), 8, 8, 8, 500.0, 500.0, 3.5, 3.5, 4,
                                  ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000),
                                  None) == bn.BN_ERR_UNSUPPORTED
    assert L.bn_plane_fit_normals(ctypes.c_void_p(0x10000), 8, 8, 8, 500.0, 500.0, 3.5, 3.5, 0,
                                  ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000),
                                  None) == bn.BN_ERR_INVALID_ARG
    assert L.bn_angle_mse(None, None, None, None, 4, 4, None, None, None) == bn.BN_ERR_INVALID_ARG
    assert L.bn_normal_angles(None, 4, 4, None, None, None) == bn.BN_ERR_INVALID_ARG


def test_probe_argument_errors():
    L = bn.lib()
    assert L.bn_stream_copy(0x20000, 0x10000, 24, None) == bn.BN_ERR_INVALID_ARG
    assert L.bn_stream_copy(0x20008, 0x10000, 32, None) == bn.BN_ERR_INVALID_ARG
    assert L.bn_stream_copy(0x20000, 0x10000, 0, None) == bn.BN_OK
    assert L.bn_stream_pattern(0x10000, 0x20000, 0x30000, 1000, None) == bn.BN_ERR_INVALID_ARG
    assert L.bn_stream_pattern(0x10004, 0x20000, 0x30000, 1024, None) == bn.BN_ERR_INVALID_ARG
    assert L.bn_alu_probe(None, 0, 16, 1.0, None) == bn.BN_OK
    assert L.bn_alu_probe(None, 4, 16, 1.0, None) == bn.BN_ERR_INVALID_ARG
    assert L.bn_alu_probe(0x10002, 4, 16, 1.0, None) == bn.BN_ERR_INVALID_ARG


def test_alignment_checked_before_launch():
    p = bn.make_params()
    # misaligned depth / normals / stats: rejected before any HIP call
    assert bn.raw_estimate_normals(0x10002, 8, 8, 8, 500.0, 500.0, 3.5, 3.5, p, 0x20000, 0x30000,
                                   0) == bn.BN_ERR_INVALID_ARG
    assert bn.raw_estimate_normals(0x10000, 8, 8, 8, 500.0, 500.0, 3.5, 3.5, p, 0x20001, 0x30000,
                                   0) == bn.BN_ERR_INVALID_ARG
    assert bn.raw_estimate_normals(0x10000, 8, 8, 8, 500.0, 500.0, 3.5, 3.5, p, 0x20000, 0x30000,
                                   0x40042) == bn.BN_ERR_INVALID_ARG


def test_stack_argument_errors():
    """Rejected before any launch (the addresses are never dereferenced)."""
    L = bn.lib()
    p = bn.make_params()
    good = (bn.Intrinsics * 3)(*[bn.Intrinsics(500.0, 500.0, 3.5, 3.5)] * 3)
    bad = (bn.Intrinsics * 3)(bn.Intrinsics(500.0, 500.0, 3.5, 3.5),
                              bn.Intrinsics(500.0, -1.0, 3.5, 3.5),
                              bn.Intrinsics(500.0, 500.0, 3.5, 3.5))
    big = (bn.Intrinsics * 65)(*[bn.Intrinsics(500.0, 500.0, 3.5, 3.5)] * 65)
    D, N, M = 0x10000, 0x20000, 0x30000

    def fwd(n, H, W, row, frame, intr, params=p, stats=0, normals=N):
        return L.bn_estimate_normals_stack(D, n, H, W, row, frame, intr, ctypes.byref(params),
                                           normals, M, stats, None)

    def adj(n, H, W, row, frame, intr, params=p, gd=M):
        return L.bn_normals_vjp_stack(D, n, H, W, row, frame, intr, ctypes.byref(params), N,
                                      gd, None)

    for f in (fwd, adj):
        assert f(-1, 8, 8, 8, 64, good) == bn.BN_ERR_INVALID_ARG
        assert f(65, 8, 8, 8, 64, big) == bn.BN_ERR_UNSUPPORTED
        assert f(3, 8, 8, 8, 64, None) == bn.BN_ERR_INVALID_ARG
        assert f(3, 8, 8, 8, 64, bad) == bn.BN_ERR_INVALID_ARG       # frame 1's fy
        assert f(3, 8, 8, 8, 63, good) == bn.BN_ERR_INVALID_ARG      # frames overlap
        assert f(3, 8, 8, 7, 64, good) == bn.BN_ERR_INVALID_ARG      # row stride < width
        assert f(3, 8, 8, 8, -64, good) == bn.BN_ERR_INVALID_ARG
        assert f(3, 8, 65537, 65537, 1 << 20, good) == bn.BN_ERR_UNSUPPORTED
        assert f(3, 8, 8, 8, 64, good, params=bn.make_params(alpha=0)) == bn.BN_ERR_INVALID_ARG
        assert f(0, 8, 8, 8, 64, None) == bn.BN_OK                   # nothing to do
        assert f(3, 0, 8, 8, 0, good) == bn.BN_OK
    assert fwd(3, 8, 8, 8, 64, good, stats=0x40001) == bn.BN_ERR_INVALID_ARG
    assert fwd(3, 8, 8, 8, 64, good, params=bn.make_params(variant=3)) == bn.BN_ERR_UNSUPPORTED
    assert fwd(3, 8, 8, 8, 64, good, params=bn.make_params(variant=17)) == bn.BN_ERR_INVALID_ARG
    assert fwd(3, 8, 8, 8, 64, good, normals=0x20002) == bn.BN_ERR_INVALID_ARG
    assert adj(3, 8, 8, 8, 64, good, params=bn.make_params(method="pair_removal")) == \
        bn.BN_ERR_UNSUPPORTED
    assert adj(3, 8, 8, 8, 64, good, params=bn.make_params(variant=1)) == bn.BN_ERR_UNSUPPORTED
    assert adj(3, 8, 8, 8, 64, good, gd=0x30002) == bn.BN_ERR_INVALID_ARG


def test_binding_refuses_short_or_wrong_stats():
    """bn_frame_stats is 4 words; the binding refuses any tensor the C ABI
    could write past (shorter, strided, wrong type) before any call."""
    import torch
    cpu = torch.device("cpu")
    bn._check_stats(torch.zeros(4, dtype=torch.int32), (4,), cpu)
    bn._check_stats(torch.zeros(3, 4, dtype=torch.int32), (3, 4), cpu)
    for bad, shape in ((torch.zeros(3, dtype=torch.int32), (4,)),
                       (torch.zeros(8, dtype=torch.int32)[::2], (4,)),
                       (torch.zeros(4, dtype=torch.int64), (4,)),
                       (torch.zeros(2, 4, dtype=torch.int32), (3, 4)),
                       (torch.zeros(12, dtype=torch.int32), (3, 4)),
                       (torch.zeros(4, 8, dtype=torch.int32)[:, :4], (4, 4))):
        with pytest.raises(ValueError):
            bn._check_stats(bad, shape, cpu)


def test_binding_refuses_bad_grad_depth():
    """The adjoint writes H*W dense floats: the binding refuses a gradient
    buffer of another shape, type or layout before any call."""
    import torch
    cpu = torch.device("cpu")
    bn._check_grad_depth(torch.zeros(6, 8), (6, 8), cpu)
    for bad in (torch.zeros(5, 8), torch.zeros(6, 8, dtype=torch.float64),
                torch.zeros(8, 6).t(), torch.zeros(48), None):
        with pytest.raises(ValueError):
            bn._check_grad_depth(bad, (6, 8), cpu)


def test_noalloc_argument_errors_before_launch():
    """bn_estimate_normals_batch_noalloc validates before any HIP call."""
    L = bn.lib()
    p = bn.make_params()
    fr = (bn.Frame * 17)(*[bn.Frame(0x10000, 8, 8, 8, 500.0, 500.0, 3.5, 3.5, 0x20000,
                                    0x30000, 0)] * 17)
    call = L.bn_estimate_normals_batch_noalloc
    assert call(None, 1, ctypes.byref(p), None) == bn.BN_ERR_INVALID_ARG
    assert call(fr, 0, ctypes.byref(p), None) == bn.BN_ERR_INVALID_ARG
    assert call(fr, 17, ctypes.byref(p), None) == bn.BN_ERR_UNSUPPORTED
    assert call(fr, 2, ctypes.byref(bn.make_params(alpha=0)), None) == bn.BN_ERR_INVALID_ARG
    assert call(fr, 2, ctypes.byref(bn.make_params(variant=2)), None) == bn.BN_ERR_UNSUPPORTED
    bad = (bn.Frame * 1)(bn.Frame(0x10000, 8, 8, 7, 500.0, 500.0, 3.5, 3.5, 0x20000, 0x30000, 0))
    assert call(bad, 1, ctypes.byref(p), None) == bn.BN_ERR_INVALID_ARG
