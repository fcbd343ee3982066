"""Python binding of libbnormals.so, the gfx950 HIP implementation of the
boundary-aware surface normal estimator (include/bnormals.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch provides device memory and the current
stream.  There is no CPU fallback: if the library is not built, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbnormals.so")

BN_OK, BN_ERR_INVALID_ARG, BN_ERR_UNSUPPORTED, BN_ERR_DEVICE, BN_ERR_OOM = 0, 1, 2, 3, 4
MASK_REL, MASK_ABS, MASK_NONE = 0, 1, 2
VALID, BOUNDARY, INVALID = 0, 1, 2
MODES = {"rel": MASK_REL, "abs": MASK_ABS, "none": MASK_NONE}
MAX_ALPHA = 8


class BnError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _status_string(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("mask_mode", ctypes.c_int32),
                ("tau", ctypes.c_float), ("variant", ctypes.c_uint32),
                ("method", ctypes.c_int32), ("scales", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


METHODS = {"four_pair": 0, "pair_removal": 1, "multiscale": 2}
FLAG_COUNTS_ACCUMULATE = 1


STATS_BYTES = 16                 # sizeof(bn_frame_stats)
STATS_WORDS = STATS_BYTES // 4   # n_valid, n_boundary, n_invalid, reserved


class FrameStats(ctypes.Structure):
    _fields_ = [("n_valid", ctypes.c_uint32), ("n_boundary", ctypes.c_uint32),
                ("n_invalid", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


def new_stats(n: Optional[int] = None, device="cuda"):
    """bn_frame_stats storage: int32 [STATS_WORDS] (or [n, STATS_WORDS]),
    zeroed.  Words 0..2 are the VALID / BOUNDARY / INVALID counts."""
    import torch
    shape = (STATS_WORDS,) if n is None else (n, STATS_WORDS)
    return torch.zeros(shape, dtype=torch.int32, device=device)


def _check_stats(stats, shape, device):
    """A stats tensor the C ABI can write: int32, contiguous, on the depth's
    device, of exactly `shape` (so no write lands past its end)."""
    import torch
    if not isinstance(stats, torch.Tensor) or stats.dtype != torch.int32 or \
            tuple(stats.shape) != tuple(shape) or not stats.is_contiguous() or \
            stats.device != device:
        raise ValueError(f"stats must be a contiguous int32 tensor of shape {tuple(shape)} on "
                         f"{device} (bn_frame_stats is {STATS_WORDS} words)")


class Frame(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("depth_stride", ctypes.c_int64),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("normals", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("stats", ctypes.c_void_p)]


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


MAX_STACK = 64


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2209_08241_amd.build`")
        # PyTorch brings up its GPU runtime first: when the library's own calls
        # come first in a process (an autotuning call before any tensor is on
        # the device, say), PyTorch's later initialisation finds no GPU
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        L.bn_estimate_normals.argtypes = [vp, i32, i32, i64, f32, f32, f32, f32,
                                          ctypes.POINTER(Params), vp, vp, vp, vp]
        L.bn_estimate_normals.restype = ctypes.c_int
        L.bn_variant_count.argtypes = []
        L.bn_variant_count.restype = ctypes.c_int
        L.bn_variant_name.argtypes = [ctypes.c_int]
        L.bn_variant_name.restype = ctypes.c_char_p
        L.bn_variant_supported.argtypes = [ctypes.c_int, vp, i32, i32, i64, vp, vp]
        L.bn_variant_supported.restype = ctypes.c_int
        L.bn_status_string.argtypes = [ctypes.c_int]
        L.bn_status_string.restype = ctypes.c_char_p
        L.bn_normals_vjp.argtypes = [vp, i32, i32, i64, f32, f32, f32, f32,
                                     ctypes.POINTER(Params), vp, vp, vp]
        L.bn_normals_vjp.restype = ctypes.c_int
        L.bn_version.argtypes = []
        L.bn_version.restype = ctypes.c_int
        L.bn_estimate_normals_stack.argtypes = [vp, i32, i32, i32, i64, i64,
                                                ctypes.POINTER(Intrinsics),
                                                ctypes.POINTER(Params), vp, vp, vp, vp]
        L.bn_estimate_normals_stack.restype = ctypes.c_int
        L.bn_normals_vjp_stack.argtypes = [vp, i32, i32, i32, i64, i64,
                                           ctypes.POINTER(Intrinsics), ctypes.POINTER(Params),
                                           vp, vp, vp]
        L.bn_normals_vjp_stack.restype = ctypes.c_int
        _bind_batch(L)
        _bind_eval(L)
        _lib = L
    return _lib


MSE_WORKSPACE_DOUBLES = 3 * 2048   # BN_MSE_WORKSPACE_DOUBLES


def _bind_eval(L) -> None:
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.bn_normal_angles.argtypes = [vp, i32, i32, vp, vp, vp]
    L.bn_normal_angles.restype = ctypes.c_int
    L.bn_angle_mse.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, vp]
    L.bn_angle_mse.restype = ctypes.c_int
    L.bn_plane_fit_normals.argtypes = [vp, i32, i32, i64, f32, f32, f32, f32, i32, vp, vp, vp]
    L.bn_plane_fit_normals.restype = ctypes.c_int
    u64 = ctypes.c_uint64
    L.bn_stream_copy.argtypes = [vp, vp, u64, vp]
    L.bn_stream_copy.restype = ctypes.c_int
    L.bn_stream_pattern.argtypes = [vp, vp, vp, u64, vp]
    L.bn_stream_pattern.restype = ctypes.c_int
    L.bn_alu_probe.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, f32, vp]
    L.bn_alu_probe.restype = ctypes.c_int


def _bind_batch(L) -> None:
    if not hasattr(L, "bn_batch_plan_create"):
        return
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    L.bn_batch_plan_create.argtypes = [ctypes.POINTER(Frame), i32, ctypes.POINTER(Params),
                                       ctypes.POINTER(vp)]
    L.bn_batch_plan_create.restype = ctypes.c_int
    L.bn_batch_plan_update.argtypes = [vp, ctypes.POINTER(Frame), i32, vp]
    L.bn_batch_plan_update.restype = ctypes.c_int
    L.bn_batch_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32)]
    L.bn_batch_plan_info.restype = ctypes.c_int
    L.bn_batch_run.argtypes = [vp, vp]
    L.bn_batch_run.restype = ctypes.c_int
    L.bn_batch_launch.argtypes = [vp, vp]
    L.bn_batch_launch.restype = ctypes.c_int
    L.bn_batch_plan_destroy.argtypes = [vp]
    L.bn_batch_plan_destroy.restype = None
    L.bn_estimate_normals_batch_noalloc.argtypes = [ctypes.POINTER(Frame), i32,
                                                    ctypes.POINTER(Params), vp]
    L.bn_estimate_normals_batch_noalloc.restype = ctypes.c_int
    L.bn_batch_plan_autotune.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    L.bn_batch_plan_autotune.restype = ctypes.c_int
    L.bn_autotune_plain.argtypes = [i32, i32, ctypes.POINTER(Params), ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_float)]
    L.bn_autotune_plain.restype = ctypes.c_int
    L.bn_autotune_save.argtypes = [ctypes.c_char_p]
    L.bn_autotune_save.restype = ctypes.c_int
    L.bn_autotune_load.argtypes = [ctypes.c_char_p]
    L.bn_autotune_load.restype = ctypes.c_int
    L.bn_autotune_reset.argtypes = []
    L.bn_autotune_reset.restype = None
    L.bn_autotune_entries.argtypes = []
    L.bn_autotune_entries.restype = ctypes.c_int


def _status_string(status: int) -> str:
    try:
        return lib().bn_status_string(int(status)).decode()
    except Exception:
        return "unknown status"


def default_variant(height: int, width: int, method="four_pair", alpha: int = 2,
                    scales: int = 0) -> int:
    """The variant the library takes with no autotuning entry, for dense
    frames of this size (vector tiles when the method and the layout allow
    them, except four-pair frames of at most 2^19 pixels: scalar tiles)."""
    me = METHODS[method] if isinstance(method, str) else int(method)
    vec_method = me != METHODS["multiscale"] or alpha * max(scales, 1) <= 16
    if not (vec_method and width % 4 == 0):
        return 1
    return 1 if (me == METHODS["four_pair"] and height * width <= (1 << 19)) else 2


def variants() -> Sequence[Tuple[int, str]]:
    """(id, name) of every kernel variant of the plain entry point."""
    L = lib()
    return [(i, L.bn_variant_name(i).decode()) for i in range(1, L.bn_variant_count() + 1)]


def make_params(alpha: int = 2, mode="rel", tau: float = 4.0, variant: int = 0,
                method="four_pair", scales: int = 0, accumulate_counts: bool = False) -> Params:
    """bn_params: method is "four_pair" (the paper's estimator), "pair_removal"
    or "multiscale" (with `scales` = K offsets alpha, 2 alpha, .., K alpha);
    accumulate_counts adds each call's counts to the stats instead of
    storing them."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    me = METHODS[method] if isinstance(method, str) else int(method)
    return Params(int(alpha), m, float(tau), int(variant), me, int(scales),
                  FLAG_COUNTS_ACCUMULATE if accumulate_counts else 0, 0)


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _check_depth(depth):
    import torch
    if not isinstance(depth, torch.Tensor) or not depth.is_cuda:
        raise TypeError("depth must be a CUDA (HIP) torch tensor")
    if depth.dtype != torch.float32 or depth.dim() != 2:
        raise TypeError("depth must be a 2-D float32 tensor")
    if depth.numel() > 0 and depth.shape[1] > 1 and depth.stride(1) != 1:
        raise ValueError("depth rows must be contiguous (stride(1) == 1)")


def estimate_normals(depth, fx: float, fy: float, cx: float, cy: float, alpha: int = 2,
                     mode="rel", tau: float = 4.0, *, variant: int = 0, method="four_pair",
                     scales: int = 0, accumulate_counts: bool = False,
                     normals=None, mask=None, stats=None, want_stats: bool = True,
                     stream=None):
    """Normals [H,W,3] float32, codes [H,W] uint8 and counts for one frame.

    `stats` (an int32 tensor of STATS_WORDS, a bn_frame_stats; words 0..2
    are the VALID / BOUNDARY / INVALID counts) receives the frame's counts
    (added to it with accumulate_counts); without one, one is allocated when
    want_stats.  Returns (normals, mask, stats_or_None).
    """
    import torch
    _check_depth(depth)
    H, W = depth.shape
    dev = depth.device
    if normals is None:
        normals = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    if mask is None:
        mask = torch.empty((H, W), dtype=torch.uint8, device=dev)
    if stats is None and want_stats:
        stats = new_stats(device=dev)
    if not (normals.is_contiguous() and normals.shape == (H, W, 3)
            and normals.dtype == torch.float32):
        raise ValueError("normals must be a contiguous float32 [H, W, 3] tensor")
    if not (mask.is_contiguous() and mask.shape == (H, W) and mask.dtype == torch.uint8):
        raise ValueError("mask must be a contiguous uint8 [H, W] tensor")
    if stats is not None:
        _check_stats(stats, (STATS_WORDS,), dev)
    p = make_params(alpha, mode, tau, variant, method, scales, accumulate_counts)
    stride = depth.stride(0) if H > 0 else W
    rc = lib().bn_estimate_normals(
        ctypes.c_void_p(depth.data_ptr()), H, W, stride, fx, fy, cx, cy, ctypes.byref(p),
        ctypes.c_void_p(normals.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
        ctypes.c_void_p(stats.data_ptr() if stats is not None else 0),
        ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_estimate_normals")
    return normals, mask, stats


def _check_stack(depth):
    import torch
    if not isinstance(depth, torch.Tensor) or not depth.is_cuda:
        raise TypeError("depth must be a CUDA (HIP) torch tensor")
    if depth.dtype != torch.float32 or depth.dim() != 3:
        raise TypeError("a stack's depth must be a 3-D float32 tensor [n, H, W]")
    if depth.numel() > 0 and depth.shape[2] > 1 and depth.stride(2) != 1:
        raise ValueError("depth rows must be contiguous (stride(2) == 1)")


def _intrinsics_array(intrinsics, n: int):
    """bn_intrinsics[n] from one (fx, fy, cx, cy) for every frame or from a
    sequence of n of them."""
    vals = list(intrinsics)
    if len(vals) == 4 and all(isinstance(v, (int, float)) for v in vals):
        vals = [tuple(vals)] * n
    if len(vals) != n:
        raise ValueError(f"{len(vals)} intrinsics for {n} frames")
    return (Intrinsics * max(n, 1))(*[Intrinsics(*map(float, v)) for v in vals])


def _stack_strides(depth):
    n, H, W = depth.shape
    row = depth.stride(1) if H > 0 else W
    frame = depth.stride(0) if n > 1 else H * row
    return row, frame


def estimate_normals_stack(depth, intrinsics, alpha: int = 2, mode="rel", tau: float = 4.0, *,
                           variant: int = 0, method="four_pair", scales: int = 0,
                           accumulate_counts: bool = False, normals=None, mask=None, stats=None,
                           want_stats: bool = True, stream=None):
    """n frames of one size in one launch (bn_estimate_normals_stack).

    `depth` is [n, H, W] float32 on the device; `intrinsics` one (fx, fy, cx,
    cy) for all frames or n of them.  Returns normals [n, H, W, 3], mask
    [n, H, W] and stats [n, STATS_WORDS] (or None); frame k equals
    estimate_normals on depth[k] bit for bit."""
    import torch
    _check_stack(depth)
    n, H, W = depth.shape
    dev = depth.device
    arr = _intrinsics_array(intrinsics, n)
    if normals is None:
        normals = torch.empty((n, H, W, 3), dtype=torch.float32, device=dev)
    if mask is None:
        mask = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    if stats is None and want_stats:
        stats = new_stats(n, device=dev)
    if not (normals.is_contiguous() and normals.shape == (n, H, W, 3)
            and normals.dtype == torch.float32):
        raise ValueError("normals must be a contiguous float32 [n, H, W, 3] tensor")
    if not (mask.is_contiguous() and mask.shape == (n, H, W) and mask.dtype == torch.uint8):
        raise ValueError("mask must be a contiguous uint8 [n, H, W] tensor")
    if stats is not None:
        _check_stats(stats, (n, STATS_WORDS), dev)
    p = make_params(alpha, mode, tau, variant, method, scales, accumulate_counts)
    row, frame = _stack_strides(depth)
    rc = lib().bn_estimate_normals_stack(
        ctypes.c_void_p(depth.data_ptr()), n, H, W, row, frame, arr, ctypes.byref(p),
        ctypes.c_void_p(normals.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
        ctypes.c_void_p(stats.data_ptr() if stats is not None else 0),
        ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_estimate_normals_stack")
    return normals, mask, stats


def raw_estimate_normals(depth_ptr: int, H: int, W: int, stride: int, fx, fy, cx, cy,
                         params: Params, normals_ptr: int, mask_ptr: int, stats_ptr: int,
                         stream: int = 0) -> int:
    """Direct C-ABI call with raw device addresses; returns the status code."""
    return lib().bn_estimate_normals(ctypes.c_void_p(depth_ptr), H, W, stride, fx, fy, cx, cy,
                                     ctypes.byref(params), ctypes.c_void_p(normals_ptr),
                                     ctypes.c_void_p(mask_ptr), ctypes.c_void_p(stats_ptr),
                                     ctypes.c_void_p(stream))


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

class BatchFrame:
    """One frame of a batch: device depth plus intrinsics; outputs are
    allocated when not given."""

    def __init__(self, depth, fx, fy, cx, cy, normals=None, mask=None, stats=None,
                 want_stats: bool = True):
        import torch
        _check_depth(depth)
        H, W = depth.shape
        dev = depth.device
        self.depth = depth
        self.fx, self.fy, self.cx, self.cy = float(fx), float(fy), float(cx), float(cy)
        self.normals = normals if normals is not None else torch.empty(
            (H, W, 3), dtype=torch.float32, device=dev)
        self.mask = mask if mask is not None else torch.empty((H, W), dtype=torch.uint8,
                                                              device=dev)
        if stats is None and want_stats:
            stats = new_stats(device=dev)
        if stats is not None:
            _check_stats(stats, (STATS_WORDS,), dev)
        if not (self.normals.is_contiguous() and tuple(self.normals.shape) == (H, W, 3) and
                self.normals.dtype == torch.float32 and self.normals.device == dev):
            raise ValueError("normals must be a contiguous float32 [H, W, 3] tensor on the "
                             "depth's device")
        if not (self.mask.is_contiguous() and tuple(self.mask.shape) == (H, W) and
                self.mask.dtype == torch.uint8 and self.mask.device == dev):
            raise ValueError("mask must be a contiguous uint8 [H, W] tensor on the depth's "
                             "device")
        self.stats = stats

    def _c(self) -> Frame:
        H, W = self.depth.shape
        return Frame(self.depth.data_ptr(), H, W, self.depth.stride(0) if H > 0 else W,
                     self.fx, self.fy, self.cx, self.cy, self.normals.data_ptr(),
                     self.mask.data_ptr(), self.stats.data_ptr() if self.stats is not None else 0)


class BatchPlan:
    """A bn_batch_plan: every frame of the list in one graph launch."""

    def __init__(self, frames, alpha: int = 2, mode="rel", tau: float = 4.0, *,
                 method="four_pair", scales: int = 0, accumulate_counts: bool = False):
        L = lib()
        self._frames = list(frames)
        arr = (Frame * len(self._frames))(*[f._c() for f in self._frames])
        self.params = make_params(alpha, mode, tau, 0, method, scales, accumulate_counts)
        h = ctypes.c_void_p()
        rc = L.bn_batch_plan_create(arr, len(self._frames), ctypes.byref(self.params),
                                    ctypes.byref(h))
        if rc != BN_OK:
            raise BnError(rc, "bn_batch_plan_create")
        self._h = h

    @property
    def frames(self):
        return self._frames

    def run(self, stream=None) -> None:
        """Replay the plan's graph on `stream`."""
        rc = lib().bn_batch_run(self._h, ctypes.c_void_p(_stream_handle(stream)))
        if rc != BN_OK:
            raise BnError(rc, "bn_batch_run")

    def launch(self, stream=None) -> None:
        """The same kernels as plain launches (one kernel for lists of at most
        16 frames, two otherwise): less host time per call than a replay."""
        rc = lib().bn_batch_launch(self._h, ctypes.c_void_p(_stream_handle(stream)))
        if rc != BN_OK:
            raise BnError(rc, "bn_batch_launch")

    def update(self, frames, stream=None) -> None:
        frames = list(frames)
        arr = (Frame * len(frames))(*[f._c() for f in frames])
        rc = lib().bn_batch_plan_update(self._h, arr, len(frames),
                                        ctypes.c_void_p(_stream_handle(stream)))
        if rc != BN_OK:
            raise BnError(rc, "bn_batch_plan_update")
        self._frames = frames

    def autotune(self, stream=None):
        """Time the plan's grid shapes - a flat grid of 1, 2 or 4 tiles per
        workgroup (shape 0, -2, -4) or 2, 4, 8 persistent workgroups per CU
        (shape 2, 4, 8) - and keep the fastest (runs the plan).  Returns
        (shape, microseconds)."""
        best, us = ctypes.c_int32(), ctypes.c_float()
        rc = lib().bn_batch_plan_autotune(self._h, ctypes.c_void_p(_stream_handle(stream)),
                                          ctypes.byref(best), ctypes.byref(us))
        if rc != BN_OK:
            raise BnError(rc, "bn_batch_plan_autotune")
        return best.value, us.value

    def info(self):
        px, tiles, wg = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        rc = lib().bn_batch_plan_info(self._h, ctypes.byref(px), ctypes.byref(tiles),
                                      ctypes.byref(wg))
        if rc != BN_OK:
            raise BnError(rc, "bn_batch_plan_info")
        return {"pixels": px.value, "tiles": tiles.value, "workgroups": wg.value}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().bn_batch_plan_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        import torch
        torch.cuda.synchronize()
        self.close()


NOALLOC_MAX_FRAMES = 16   # BN_NOALLOC_MAX_FRAMES


def estimate_normals_batch_noalloc(frames, alpha: int = 2, mode="rel", tau: float = 4.0, *,
                                   method="four_pair", scales: int = 0,
                                   accumulate_counts: bool = False, stream=None) -> None:
    """At most NOALLOC_MAX_FRAMES BatchFrames in one launch through
    bn_estimate_normals_batch_noalloc, which allocates nothing (its count
    work areas are a fixed device array shared by every call on the GPU:
    calls must not overlap in time)."""
    frames = list(frames)
    arr = (Frame * max(len(frames), 1))(*[f._c() for f in frames])
    p = make_params(alpha, mode, tau, 0, method, scales, accumulate_counts)
    rc = lib().bn_estimate_normals_batch_noalloc(arr, len(frames), ctypes.byref(p),
                                                 ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_estimate_normals_batch_noalloc")


# ---------------------------------------------------------------------------
# autotuning table
# ---------------------------------------------------------------------------

def autotune_plain(height: int, width: int, alpha: int = 2, mode="rel", tau: float = 4.0, *,
                   method="four_pair", scales: int = 0):
    """Time every plain variant on frames of this size; returns (variant, us)."""
    p = make_params(alpha, mode, tau, 0, method, scales)
    best, us = ctypes.c_int32(), ctypes.c_float()
    rc = lib().bn_autotune_plain(int(height), int(width), ctypes.byref(p), ctypes.byref(best),
                                 ctypes.byref(us))
    if rc != BN_OK:
        raise BnError(rc, "bn_autotune_plain")
    return best.value, us.value


def autotune_save(path: str) -> None:
    rc = lib().bn_autotune_save(os.fsencode(path))
    if rc != BN_OK:
        raise BnError(rc, "bn_autotune_save")


def autotune_load(path: str) -> None:
    rc = lib().bn_autotune_load(os.fsencode(path))
    if rc != BN_OK:
        raise BnError(rc, "bn_autotune_load")


def autotune_reset() -> None:
    lib().bn_autotune_reset()


def autotune_entries() -> int:
    return int(lib().bn_autotune_entries())


# ---------------------------------------------------------------------------
# differentiation
# ---------------------------------------------------------------------------

def _check_grad_depth(grad_depth, shape, device):
    """The adjoint writes prod(shape) dense floats: refuse anything else."""
    import torch
    if not (isinstance(grad_depth, torch.Tensor) and grad_depth.is_contiguous() and
            tuple(grad_depth.shape) == tuple(shape) and grad_depth.dtype == torch.float32 and
            grad_depth.device == device):
        raise ValueError(f"grad_depth must be a contiguous float32 tensor of shape "
                         f"{tuple(shape)} on {device}")


def normals_vjp(depth, fx, fy, cx, cy, grad_normals, alpha: int = 2, mode="rel",
                tau: float = 4.0, grad_depth=None, stream=None):
    """d(sum normals . grad_normals)/d depth with every pixel's code held
    fixed (bn_normals_vjp).  Returns grad_depth [H, W] float32."""
    import torch
    _check_depth(depth)
    H, W = depth.shape
    g = grad_normals
    if not (g.is_cuda and g.dtype == torch.float32 and g.shape == (H, W, 3)):
        raise ValueError("grad_normals must be a float32 [H, W, 3] device tensor")
    g = g.contiguous()
    if grad_depth is None:
        grad_depth = torch.empty((H, W), dtype=torch.float32, device=depth.device)
    _check_grad_depth(grad_depth, (H, W), depth.device)
    p = make_params(alpha, mode, tau, 0)
    stride = depth.stride(0) if H > 0 else W
    rc = lib().bn_normals_vjp(ctypes.c_void_p(depth.data_ptr()), H, W, stride, fx, fy, cx, cy,
                              ctypes.byref(p), ctypes.c_void_p(g.data_ptr()),
                              ctypes.c_void_p(grad_depth.data_ptr()),
                              ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_normals_vjp")
    return grad_depth


def normals_vjp_stack(depth, intrinsics, grad_normals, alpha: int = 2, mode="rel",
                      tau: float = 4.0, grad_depth=None, stream=None):
    """The adjoint of estimate_normals_stack (bn_normals_vjp_stack): grad
    [n, H, W] from the cotangent [n, H, W, 3], every frame in one launch."""
    import torch
    _check_stack(depth)
    n, H, W = depth.shape
    g = grad_normals
    if not (g.is_cuda and g.dtype == torch.float32 and g.shape == (n, H, W, 3)):
        raise ValueError("grad_normals must be a float32 [n, H, W, 3] device tensor")
    g = g.contiguous()
    if grad_depth is None:
        grad_depth = torch.empty((n, H, W), dtype=torch.float32, device=depth.device)
    _check_grad_depth(grad_depth, (n, H, W), depth.device)
    arr = _intrinsics_array(intrinsics, n)
    p = make_params(alpha, mode, tau, 0)
    row, frame = _stack_strides(depth)
    rc = lib().bn_normals_vjp_stack(ctypes.c_void_p(depth.data_ptr()), n, H, W, row, frame, arr,
                                    ctypes.byref(p), ctypes.c_void_p(g.data_ptr()),
                                    ctypes.c_void_p(grad_depth.data_ptr()),
                                    ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_normals_vjp_stack")
    return grad_depth


def _normals_function():
    import torch

    class NormalsFunction(torch.autograd.Function):
        """normals, mask = f(depth); backward through the hand-written
        adjoint kernel (codes frozen; the mask output is not differentiable)."""

        @staticmethod
        def forward(ctx, depth, fx, fy, cx, cy, alpha, mode, tau):
            n, m, _ = estimate_normals(depth, fx, fy, cx, cy, alpha, mode, tau, want_stats=False)
            ctx.save_for_backward(depth)
            ctx.args = (fx, fy, cx, cy, alpha, mode, tau)
            ctx.mark_non_differentiable(m)
            return n, m

        @staticmethod
        def backward(ctx, grad_n, grad_m):
            (depth,) = ctx.saved_tensors
            fx, fy, cx, cy, alpha, mode, tau = ctx.args
            gd = None
            if ctx.needs_input_grad[0]:
                gd = normals_vjp(depth, fx, fy, cx, cy, grad_n.float(), alpha, mode, tau)
            return gd, None, None, None, None, None, None, None

    class StackFunction(torch.autograd.Function):
        """The same over a stack [n, H, W]: one launch each way."""

        @staticmethod
        def forward(ctx, depth, intrinsics, alpha, mode, tau):
            n, m, _ = estimate_normals_stack(depth, intrinsics, alpha, mode, tau,
                                             want_stats=False)
            ctx.save_for_backward(depth)
            ctx.args = (intrinsics, alpha, mode, tau)
            ctx.mark_non_differentiable(m)
            return n, m

        @staticmethod
        def backward(ctx, grad_n, grad_m):
            (depth,) = ctx.saved_tensors
            intrinsics, alpha, mode, tau = ctx.args
            gd = None
            if ctx.needs_input_grad[0]:
                gd = normals_vjp_stack(depth, intrinsics, grad_n.float(), alpha, mode, tau)
            return gd, None, None, None, None

    return NormalsFunction, StackFunction


_NormalsFunction = None
_StackFunction = None


def normals_with_grad(depth, fx, fy, cx, cy, alpha: int = 2, mode="rel", tau: float = 4.0):
    """Differentiable estimate_normals: returns (normals, mask); gradients
    flow to `depth` through bn_normals_vjp."""
    global _NormalsFunction, _StackFunction
    if _NormalsFunction is None:
        _NormalsFunction, _StackFunction = _normals_function()
    return _NormalsFunction.apply(depth, float(fx), float(fy), float(cx), float(cy), int(alpha),
                                  mode, float(tau))


def normals_with_grad_stack(depth, intrinsics, alpha: int = 2, mode="rel", tau: float = 4.0):
    """Differentiable estimate_normals_stack over depth [n, H, W]: returns
    (normals, mask); gradients flow through bn_normals_vjp_stack."""
    global _NormalsFunction, _StackFunction
    if _StackFunction is None:
        _NormalsFunction, _StackFunction = _normals_function()
    n = depth.shape[0]
    arr = _intrinsics_array(intrinsics, n)
    key = tuple((c.fx, c.fy, c.cx, c.cy) for c in arr[:n])
    return _StackFunction.apply(depth, key, int(alpha), mode, float(tau))


def cosine_loss(normals, target, mask, target_mask):
    """mean over pixels valid in both of (1 - normals . target); any leading
    shape (one frame or a stack).  No host synchronisation."""
    import torch
    U = (mask == VALID) & (target_mask == VALID)
    cos = (normals * target).sum(-1)
    return torch.where(U, 1.0 - cos, torch.zeros_like(cos)).sum() / U.sum().clamp(min=1)


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

BACKEND_HIP, BACKEND_FAKE = 0, 1
REQ_PENDING, REQ_ADMITTED, REQ_READY, REQ_RUNNING, REQ_DONE, REQ_FAILED = range(6)
BN_ERR_TIMEOUT = 5


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("max_batches_in_flight", ctypes.c_int32), ("params", Params),
                ("backend", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("fake_ns_per_pixel", ctypes.c_double), ("fake_launch_ns", ctypes.c_double),
                ("fake_copy_gbs", ctypes.c_double)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32),
                ("batch_size", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("batch", ctypes.c_uint64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double), ("normals", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("stats", ctypes.c_void_p)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("submitted", "completed", "failed", "released", "batches", "pending",
                 "in_flight_batches", "bytes_in_use", "peak_bytes_in_use", "max_batch_seen")]


def _bind_server(L) -> None:
    if getattr(L, "_server_bound", False):
        return
    vp, i32, i64, f32, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                              ctypes.c_double)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.bn_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    L.bn_server_submit.argtypes = [vp, vp, i32, i32, i32, i64, f32, f32, f32, f32, u64p]
    L.bn_server_query.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(RequestInfo)]
    L.bn_server_wait.argtypes = [vp, ctypes.c_uint64, dbl, ctypes.POINTER(RequestInfo)]
    L.bn_server_release.argtypes = [vp, ctypes.c_uint64]
    L.bn_server_progress.argtypes = [vp]
    L.bn_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.bn_server_fake_advance.argtypes = [vp, dbl]
    L.bn_server_fake_fail.argtypes = [vp, ctypes.c_uint64]
    L.bn_server_destroy.argtypes = [vp]
    L.bn_server_destroy.restype = None
    L.bn_server_run_poisson.argtypes = [vp, ctypes.POINTER(Frame), i32, dbl, i32, ctypes.c_uint64,
                                        ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                        ctypes.POINTER(i64)]
    for name in ("bn_server_create", "bn_server_submit", "bn_server_query", "bn_server_wait",
                 "bn_server_release", "bn_server_progress", "bn_server_get_stats",
                 "bn_server_fake_advance", "bn_server_fake_fail", "bn_server_run_poisson"):
        getattr(L, name).restype = ctypes.c_int
    L._server_bound = True


class Server:
    """bn_server: continuous batching of mixed-size frames under an HBM budget."""

    def __init__(self, budget_bytes: int, max_batch: int = 16, max_batches_in_flight: int = 2,
                 alpha: int = 2, mode="rel", tau: float = 4.0, backend: str = "hip",
                 fake_ns_per_pixel: float = 0.004, fake_launch_ns: float = 5000.0,
                 fake_copy_gbs: float = 25.0, *, method="four_pair", scales: int = 0):
        L = lib()
        _bind_server(L)
        cfg = ServerConfig(int(budget_bytes), int(max_batch), int(max_batches_in_flight),
                           make_params(alpha, mode, tau, 0, method, scales),
                           BACKEND_FAKE if backend == "fake" else BACKEND_HIP, 0,
                           float(fake_ns_per_pixel), float(fake_launch_ns), float(fake_copy_gbs))
        h = ctypes.c_void_p()
        rc = L.bn_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != BN_OK:
            raise BnError(rc, "bn_server_create")
        self._h = h
        self._keep = {}

    def submit(self, depth, fx, fy, cx, cy, *, host: Optional[bool] = None, height=None,
               width=None, stride=None) -> int:
        """Queue a frame; `depth` is a torch tensor (device or host), or a raw
        address with height/width/stride and `host` given.  Returns its id."""
        L = lib()
        if isinstance(depth, int):
            ptr, H, W = depth, int(height), int(width)
            st = int(stride if stride is not None else W)
            on_host = bool(host)
        else:
            H, W = depth.shape
            ptr = depth.data_ptr()
            st = depth.stride(0) if H > 0 else W
            on_host = not depth.is_cuda if host is None else bool(host)
        rid = ctypes.c_uint64()
        rc = L.bn_server_submit(self._h, ctypes.c_void_p(ptr), 1 if on_host else 0, H, W, st,
                                fx, fy, cx, cy, ctypes.byref(rid))
        if rc != BN_OK:
            raise BnError(rc, "bn_server_submit")
        if not isinstance(depth, int):
            self._keep[rid.value] = depth       # the input must outlive the request
        return rid.value

    def query(self, rid: int) -> dict:
        info = RequestInfo()
        rc = lib().bn_server_query(self._h, rid, ctypes.byref(info))
        if rc != BN_OK:
            raise BnError(rc, "bn_server_query")
        return info.as_dict()

    def wait(self, rid: int, timeout: float = 60.0) -> dict:
        info = RequestInfo()
        rc = lib().bn_server_wait(self._h, rid, float(timeout), ctypes.byref(info))
        if rc != BN_OK:
            raise BnError(rc, "bn_server_wait")
        return info.as_dict()

    def release(self, rid: int) -> None:
        rc = lib().bn_server_release(self._h, rid)
        if rc != BN_OK:
            raise BnError(rc, "bn_server_release")
        self._keep.pop(rid, None)

    def progress(self) -> int:
        rc = lib().bn_server_progress(self._h)
        if rc < 0:
            raise BnError(-rc, "bn_server_progress")
        return rc

    def stats(self) -> dict:
        s = ServerStats()
        rc = lib().bn_server_get_stats(self._h, ctypes.byref(s))
        if rc != BN_OK:
            raise BnError(rc, "bn_server_get_stats")
        return {k: getattr(s, k) for k, _ in s._fields_}

    def fake_advance(self, seconds: float) -> None:
        rc = lib().bn_server_fake_advance(self._h, float(seconds))
        if rc != BN_OK:
            raise BnError(rc, "bn_server_fake_advance")

    def fake_fail(self, rid: int) -> None:
        rc = lib().bn_server_fake_fail(self._h, rid)
        if rc != BN_OK:
            raise BnError(rc, "bn_server_fake_fail")

    def run_poisson(self, pool, rate_hz: float, n_requests: int, seed: int = 3000):
        """Open-loop Poisson load over `pool` (BatchFrame list of device
        frames); returns latencies (s), wall time (s) and pixels."""
        import numpy as np
        arr = (Frame * len(pool))(*[f._c() for f in pool])
        lat = (ctypes.c_double * n_requests)()
        wall = ctypes.c_double()
        px = ctypes.c_int64()
        rc = lib().bn_server_run_poisson(self._h, arr, len(pool), float(rate_hz), int(n_requests),
                                         int(seed), lat, ctypes.byref(wall), ctypes.byref(px))
        if rc != BN_OK:
            raise BnError(rc, "bn_server_run_poisson")
        return {"latency_s": np.frombuffer(lat, dtype=np.float64).copy(), "wall_s": wall.value,
                "pixels": px.value}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().bn_server_destroy(self._h)
        self._h = None
        self._keep = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def device_to_host(ptr: int, nbytes: int):
    """Copy device memory at `ptr` into a new numpy uint8 array (tests)."""
    import numpy as np
    import torch
    out = np.empty(nbytes, dtype=np.uint8)
    if nbytes:
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        torch.cuda.synchronize()
        rc = hip.hipMemcpy(out.ctypes.data, ctypes.c_void_p(ptr), nbytes, 2)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed: {rc}")
    return out


# ---------------------------------------------------------------------------
# evaluation tools (Section 4)
# ---------------------------------------------------------------------------

def _check_normals(n, what="normals"):
    import torch
    if not (isinstance(n, torch.Tensor) and n.is_cuda and n.dtype == torch.float32
            and n.dim() == 3 and n.shape[2] == 3 and n.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous CUDA float32 [H, W, 3] tensor")


def normal_angles(normals, stream=None):
    """(theta, phi) images [H, W] float32 of a normal map (Eqs. 14-15):
    phi = atan2(ny, nx) in [0, 2 pi), theta = atan2(|(nx, ny)|, nz)."""
    import torch
    _check_normals(normals)
    H, W = normals.shape[:2]
    theta = torch.empty((H, W), dtype=torch.float32, device=normals.device)
    phi = torch.empty_like(theta)
    rc = lib().bn_normal_angles(ctypes.c_void_p(normals.data_ptr()), H, W,
                                ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_normal_angles")
    return theta, phi


def angle_mse(normals_a, mask_a, normals_b, mask_b=None, stream=None, sync: bool = True):
    """(MSE theta, MSE phi, pixel count) over the pixels VALID in both maps
    (a None mask counts as all valid).  Returns a device tensor of 3 doubles
    when sync is False."""
    import torch
    _check_normals(normals_a, "normals_a")
    _check_normals(normals_b, "normals_b")
    H, W = normals_a.shape[:2]
    if normals_b.shape[:2] != (H, W):
        raise ValueError("the two normal maps differ in size")
    for m in (mask_a, mask_b):
        if m is not None and not (m.is_cuda and m.dtype == torch.uint8 and m.shape == (H, W)
                                  and m.is_contiguous()):
            raise ValueError("masks must be contiguous CUDA uint8 [H, W] tensors")
    dev = normals_a.device
    ws = torch.empty(MSE_WORKSPACE_DOUBLES, dtype=torch.float64, device=dev)
    out = torch.empty(3, dtype=torch.float64, device=dev)
    rc = lib().bn_angle_mse(ctypes.c_void_p(normals_a.data_ptr()),
                            ctypes.c_void_p(mask_a.data_ptr() if mask_a is not None else 0),
                            ctypes.c_void_p(normals_b.data_ptr()),
                            ctypes.c_void_p(mask_b.data_ptr() if mask_b is not None else 0),
                            H, W, ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                            ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_angle_mse")
    if not sync:
        return out
    t, p, k = out.cpu().tolist()
    return t, p, int(k)


def plane_fit_normals(depth, fx, fy, cx, cy, radius: int = 2, stream=None):
    """Plane-fit normals [H, W, 3] float32 and codes [H, W] uint8 over the
    (2 radius + 1)^2 window (radius 2: the 25-neighbour fit)."""
    import torch
    _check_depth(depth)
    H, W = depth.shape
    normals = torch.empty((H, W, 3), dtype=torch.float32, device=depth.device)
    mask = torch.empty((H, W), dtype=torch.uint8, device=depth.device)
    stride = depth.stride(0) if H > 0 else W
    rc = lib().bn_plane_fit_normals(ctypes.c_void_p(depth.data_ptr()), H, W, stride, fx, fy, cx,
                                    cy, int(radius), ctypes.c_void_p(normals.data_ptr()),
                                    ctypes.c_void_p(mask.data_ptr()),
                                    ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_plane_fit_normals")
    return normals, mask


# ---------------------------------------------------------------------------
# bandwidth probes
# ---------------------------------------------------------------------------

def stream_copy(dst, src, stream=None) -> None:
    """Copy src into dst (same byte size, a multiple of 16) with 16-byte
    non-temporal loads and stores."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("dst and src differ in size")
    rc = lib().bn_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), n,
                              ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_stream_copy")


def stream_pattern(depth, normals, mask, stream=None) -> None:
    """The estimator's traffic shape without its arithmetic (see the header)."""
    n = depth.numel()
    rc = lib().bn_stream_pattern(ctypes.c_void_p(depth.data_ptr()),
                                 ctypes.c_void_p(normals.data_ptr()),
                                 ctypes.c_void_p(mask.data_ptr()), n,
                                 ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_stream_pattern")


def alu_probe(out, iters: int, m: float = 1.0000001, stream=None) -> int:
    """Independent binary32 multiply chains, 8 per thread, `iters` steps each,
    over out.numel() / 256 workgroups; writes each thread's sum of chains to
    `out` and returns the number of multiplies (lane operations) issued."""
    import torch
    if (not isinstance(out, torch.Tensor) or out.dtype != torch.float32 or not out.is_cuda
            or not out.is_contiguous() or out.numel() % 256):
        raise ValueError("out must be a contiguous float32 device tensor of a multiple of 256")
    wgs = out.numel() // 256
    rc = lib().bn_alu_probe(ctypes.c_void_p(out.data_ptr()), wgs, int(iters), float(m),
                            ctypes.c_void_p(_stream_handle(stream)))
    if rc != BN_OK:
        raise BnError(rc, "bn_alu_probe")
    return wgs * 256 * 8 * int(iters)
