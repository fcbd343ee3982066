"""Counted launches on many streams: each stream gets a count work area of
its own, more streams than the pool holds recycle the work areas after the
device is idle, and streams created one after another's destruction (once
its launch has completed) count correctly whatever handle values they get.
Every launch's counts must equal the oracle's."""
import ctypes

import pytest

import oracle
import paper_2209_08241_amd as bn
from gpu_util import log, to_gpu
from synth import scenes

pytestmark = pytest.mark.gpu

MAX_STREAMS = 64


def _hip():
    L = ctypes.CDLL("libamdhip64.so")
    L.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    L.hipStreamCreate.restype = ctypes.c_int
    L.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    L.hipStreamDestroy.restype = ctypes.c_int
    return L


def _create(L):
    h = ctypes.c_void_p()
    assert L.hipStreamCreate(ctypes.byref(h)) == 0
    return h.value


def test_more_streams_than_the_pool():
    import torch
    s = scenes.sized_frame(96, 128, seed=77)
    want = [int(c) for c in oracle.normals_f32(s.depth, *s.intrinsics, 2, "rel", 4.0)["counts"]]
    d = to_gpu(s.depth)
    n = MAX_STREAMS + 8
    st = bn.new_stats(n, device="cuda")
    st.fill_(-1)
    normals = torch.empty((n, 96, 128, 3), device="cuda")
    masks = torch.empty((n, 96, 128), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    L = _hip()
    streams = [_create(L) for _ in range(n)]
    try:
        log(f"{n} streams, one counted launch each, then again in reverse order")
        for rnd in range(2):
            order = range(n) if rnd == 0 else reversed(range(n))
            for k in order:
                bn.estimate_normals(d, *s.intrinsics, 2, normals=normals[k], mask=masks[k],
                                    stats=st[k], stream=streams[k])
            torch.cuda.synchronize()
            got = st[:, :3].cpu().tolist()
            assert all(g == want for g in got), f"round {rnd}"
            assert not st[:, 3].any()
    finally:
        for h in streams:
            L.hipStreamDestroy(h)


def test_stream_created_after_a_destroyed_one():
    import torch
    s = scenes.sized_frame(480, 640, seed=78)
    want = [int(c) for c in oracle.normals_f32(s.depth, *s.intrinsics, 2, "rel", 4.0)["counts"]]
    d = to_gpu(s.depth)
    st = bn.new_stats(8, device="cuda")
    normals = torch.empty((8, 480, 640, 3), device="cuda")
    masks = torch.empty((8, 480, 640), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    L = _hip()
    for k in range(8):
        h = _create(L)
        bn.estimate_normals(d, *s.intrinsics, 2, normals=normals[k], mask=masks[k], stats=st[k],
                            stream=h)
        torch.cuda.synchronize()
        # the next stream may take over the handle value
        assert L.hipStreamDestroy(h) == 0
    torch.cuda.synchronize()
    assert all(g == want for g in st[:, :3].cpu().tolist())
