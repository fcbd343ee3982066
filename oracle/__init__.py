"""FP64 CPU oracle of the boundary-aware normal estimator -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never imports it and shares no code with it.

`liboracle.so` is built from bn_oracle.c (plain C, FP64, no FMA contraction);
this module is its ctypes front end.  The PCA brute force lives in
oracle/pca.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bn_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

VALID, BOUNDARY, INVALID = 0, 1, 2
MODES = {"rel": 0, "abs": 1, "none": 2}
METHODS = {"four_pair": 0, "pair_removal": 1, "multiscale": 2}

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
             "-fexcess-precision=standard", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (always when force=True)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def load(path: str = LIB):
    """ctypes handle on an oracle library built from bn_oracle.c."""
    if path == LIB and not os.path.exists(LIB):
        build()
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    up = ctypes.POINTER(ctypes.c_uint8)
    qp = ctypes.POINTER(ctypes.c_uint64)
    L.bno_normals_f32.argtypes = [fp, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                  ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_float, dp, up, qp, dp, dp, dp]
    L.bno_normals_f32.restype = ctypes.c_int
    L.bno_normals_f32_rows.argtypes = [fp, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_float, ctypes.c_int, ctypes.c_int,
                                       dp, up, qp, dp, dp, dp]
    L.bno_normals_f32_rows.restype = ctypes.c_int
    L.bno_normals_f64.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, dp, up, qp, dp, dp, dp]
    L.bno_normals_f64.restype = ctypes.c_int
    L.bno_normals_frozen_f64.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, up, dp]
    L.bno_normals_frozen_f64.restype = ctypes.c_int
    L.bno_normals_vjp_f64.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, up, dp, dp]
    L.bno_normals_vjp_f64.restype = ctypes.c_int
    L.bno_variant_f32_rows.argtypes = [ctypes.c_int, ctypes.c_int, fp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_float, ctypes.c_int, ctypes.c_int, dp, up, qp,
                                       dp, dp, up, dp]
    L.bno_variant_f32_rows.restype = ctypes.c_int
    L.bno_variant_f64.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, dp, up, qp, dp, dp, up, dp]
    L.bno_variant_f64.restype = ctypes.c_int
    L.bno_variant_abs_threshold_f32.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                                ctypes.c_float, ctypes.c_float, ctypes.c_int]
    L.bno_variant_abs_threshold_f32.restype = ctypes.c_float
    L.bno_abs_threshold_f32.argtypes = [ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, ctypes.c_int]
    L.bno_abs_threshold_f32.restype = ctypes.c_float
    return L


def _ptr(a: Optional[np.ndarray], ct):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ct))
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _mode(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


def _method(method) -> int:
    return METHODS[method] if isinstance(method, str) else int(method)


def _run(fn, depth, dt, ct, fx, fy, cx, cy, alpha, mode, tau, want_r, want_rho, eq7):
    depth = np.asarray(depth)
    if depth.ndim != 2 or depth.dtype != dt:
        raise TypeError(f"depth must be a 2-D {np.dtype(dt).name} array")
    if depth.strides[1] != depth.itemsize or depth.strides[0] % depth.itemsize:
        depth = np.ascontiguousarray(depth)
    H, W = depth.shape
    stride = depth.strides[0] // depth.itemsize if H > 0 else W
    normals = np.zeros((H, W, 3), dtype=np.float64)
    mask = np.zeros((H, W), dtype=np.uint8)
    counts = np.zeros(3, dtype=np.uint64)
    r = np.empty((H, W), dtype=np.float64) if want_r else None
    rho = np.empty((H, W), dtype=np.float64) if want_rho else None
    gap = np.zeros(1, dtype=np.float64) if eq7 else None
    rc = fn(_ptr(depth, ct), H, W, stride, fx, fy, cx, cy, int(alpha), _mode(mode),
            tau, _ptr(normals, ctypes.c_double), _ptr(mask, ctypes.c_uint8),
            _ptr(counts, ctypes.c_uint64), _ptr(r, ctypes.c_double),
            _ptr(rho, ctypes.c_double), _ptr(gap, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out: Dict[str, np.ndarray] = {"normals": normals, "mask": mask, "counts": counts}
    if want_r:
        out["r"] = r
    if want_rho:
        out["rho"] = rho
    if eq7:
        out["eq7_gap"] = float(gap[0])
    return out


def _band_buffers(out, n, W):
    """Output buffers of a band of n rows: fresh ones, or the caller's (which
    must be C-contiguous and large enough)."""
    if out is None:
        return np.zeros((n, W, 3), dtype=np.float64), np.zeros((n, W), dtype=np.uint8)
    normals, mask = out
    if (normals.dtype != np.float64 or mask.dtype != np.uint8 or
            not normals.flags.c_contiguous or not mask.flags.c_contiguous or
            normals.size < 3 * n * W or mask.size < n * W):
        raise ValueError("band buffers too small or of the wrong type")
    return normals, mask


class Oracle:
    """The oracle entry points bound to one library file."""

    def __init__(self, path: str = LIB):
        self.path = path
        self.L = load(path)

    def normals_f32(self, depth, fx, fy, cx, cy, alpha=2, mode="rel", tau=4.0, *,
                    want_r=False, want_rho=False, eq7=False):
        """Binary32 depth -> FP64 camera-facing normals, codes and counts.

        The validity and boundary decisions are the binary32 ones the GPU
        path must reproduce bit for bit.
        """
        return _run(self.L.bno_normals_f32, depth, np.float32, ctypes.c_float,
                    fx, fy, cx, cy, alpha, mode, tau, want_r, want_rho, eq7)

    def normals_f32_rows(self, depth, fx, fy, cx, cy, alpha, mode, tau, row_begin, row_end,
                         out=None):
        """Rows [row_begin, row_end) of normals_f32 on the full frame.  out:
        optional (normals, mask) buffers (C-contiguous float64 and uint8 of at
        least (row_end - row_begin) * W * 3 and * W elements) to write into;
        the band occupies their first elements."""
        depth = np.asarray(depth)
        if depth.ndim != 2 or depth.dtype != np.float32:
            raise TypeError("depth must be a 2-D float32 array")
        if depth.strides[1] != 4 or depth.strides[0] % 4:
            depth = np.ascontiguousarray(depth)
        H, W = depth.shape
        stride = depth.strides[0] // 4 if H > 0 else W
        n = row_end - row_begin
        normals, mask = _band_buffers(out, n, W)
        counts = np.zeros(3, dtype=np.uint64)
        none = ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
        rc = self.L.bno_normals_f32_rows(
            _ptr(depth, ctypes.c_float), H, W, stride, fx, fy, cx, cy, int(alpha),
            _mode(mode), tau, int(row_begin), int(row_end), _ptr(normals, ctypes.c_double),
            _ptr(mask, ctypes.c_uint8), _ptr(counts, ctypes.c_uint64), none, none, none)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        return {"normals": normals, "mask": mask, "counts": counts}

    def normals_f64(self, depth, fx, fy, cx, cy, alpha=2, mode="rel", tau=4.0, *,
                    want_r=False, want_rho=False, eq7=False):
        """FP64 depth -> FP64 normals; boundary decided in FP64 on r or rho."""
        return _run(self.L.bno_normals_f64, depth, np.float64, ctypes.c_double,
                    fx, fy, cx, cy, alpha, mode, tau, want_r, want_rho, eq7)

    def normals_frozen_f64(self, depth, fx, fy, cx, cy, alpha, codes):
        """FP64 normals of the pixels whose code is VALID, codes held fixed."""
        depth = np.ascontiguousarray(depth, dtype=np.float64)
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        H, W = depth.shape
        out = np.zeros((H, W, 3), dtype=np.float64)
        rc = self.L.bno_normals_frozen_f64(_ptr(depth, ctypes.c_double), H, W, W, fx, fy, cx, cy,
                                           int(alpha), _ptr(codes, ctypes.c_uint8),
                                           _ptr(out, ctypes.c_double))
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        return out

    def normals_vjp_f64(self, depth, fx, fy, cx, cy, alpha, codes, grad_normals):
        """FP64 d(sum normals . grad_normals)/d depth with the codes frozen."""
        depth = np.ascontiguousarray(depth, dtype=np.float64)
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        g = np.ascontiguousarray(grad_normals, dtype=np.float64)
        H, W = depth.shape
        out = np.zeros((H, W), dtype=np.float64)
        rc = self.L.bno_normals_vjp_f64(_ptr(depth, ctypes.c_double), H, W, W, fx, fy, cx, cy,
                                        int(alpha), _ptr(codes, ctypes.c_uint8),
                                        _ptr(g, ctypes.c_double), _ptr(out, ctypes.c_double))
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        return out

    def variant_f32(self, depth, fx, fy, cx, cy, alpha=2, mode="rel", tau=4.0, *,
                    method="four_pair", scales=0, rows=None, want_r=False, want_rho=False,
                    want_keep=False, gap=False, out=None):
        """Any method (four_pair, pair_removal, multiscale), binary32 depth in,
        FP64 normals out, binary32 decisions; rows=(begin, end) evaluates
        those rows of the frame only (out: as for normals_f32_rows)."""
        depth = np.asarray(depth)
        if depth.ndim != 2 or depth.dtype != np.float32:
            raise TypeError("depth must be a 2-D float32 array")
        if depth.strides[1] != 4 or depth.strides[0] % 4:
            depth = np.ascontiguousarray(depth)
        H, W = depth.shape
        stride = depth.strides[0] // 4 if H > 0 else W
        rb, re = (0, H) if rows is None else rows
        n = re - rb
        normals, mask = _band_buffers(out, n, W)
        counts = np.zeros(3, dtype=np.uint64)
        r = np.empty((n, W)) if want_r else None
        rho = np.empty((n, W)) if want_rho else None
        keep = np.zeros((n, W), dtype=np.uint8) if want_keep else None
        g = np.zeros(1) if gap else None
        rc = self.L.bno_variant_f32_rows(
            _method(method), int(scales), _ptr(depth, ctypes.c_float), H, W, stride, fx, fy,
            cx, cy, int(alpha), _mode(mode), tau, int(rb), int(re),
            _ptr(normals, ctypes.c_double), _ptr(mask, ctypes.c_uint8),
            _ptr(counts, ctypes.c_uint64), _ptr(r, ctypes.c_double), _ptr(rho, ctypes.c_double),
            _ptr(keep, ctypes.c_uint8), _ptr(g, ctypes.c_double))
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        out = {"normals": normals, "mask": mask, "counts": counts}
        if want_r:
            out["r"] = r
        if want_rho:
            out["rho"] = rho
        if want_keep:
            out["keep"] = keep
        if gap:
            out["gap"] = float(g[0])
        return out

    def variant_f64(self, depth, fx, fy, cx, cy, alpha=2, mode="rel", tau=4.0, *,
                    method="four_pair", scales=0, want_r=False, want_rho=False,
                    want_keep=False, gap=False):
        """Any method, FP64 depth in, FP64 normals and FP64 decisions."""
        depth = np.ascontiguousarray(depth, dtype=np.float64)
        H, W = depth.shape
        normals = np.zeros((H, W, 3), dtype=np.float64)
        mask = np.zeros((H, W), dtype=np.uint8)
        counts = np.zeros(3, dtype=np.uint64)
        r = np.empty((H, W)) if want_r else None
        rho = np.empty((H, W)) if want_rho else None
        keep = np.zeros((H, W), dtype=np.uint8) if want_keep else None
        g = np.zeros(1) if gap else None
        rc = self.L.bno_variant_f64(
            _method(method), int(scales), _ptr(depth, ctypes.c_double), H, W, W, fx, fy, cx, cy,
            int(alpha), _mode(mode), tau, _ptr(normals, ctypes.c_double),
            _ptr(mask, ctypes.c_uint8), _ptr(counts, ctypes.c_uint64), _ptr(r, ctypes.c_double),
            _ptr(rho, ctypes.c_double), _ptr(keep, ctypes.c_uint8), _ptr(g, ctypes.c_double))
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        out = {"normals": normals, "mask": mask, "counts": counts}
        if want_r:
            out["r"] = r
        if want_rho:
            out["rho"] = rho
        if want_keep:
            out["keep"] = keep
        if gap:
            out["gap"] = float(g[0])
        return out

    def variant_abs_threshold_f32(self, method, scales, fx, fy, tau, alpha) -> float:
        """Binary32 ABS threshold on |m|^2 of a method."""
        return float(self.L.bno_variant_abs_threshold_f32(_method(method), int(scales), fx, fy,
                                                          tau, int(alpha)))

    def abs_threshold_f32(self, fx, fy, tau, alpha) -> float:
        """Binary32 threshold on |m|^2 that ABS mode compares against."""
        return float(self.L.bno_abs_threshold_f32(fx, fy, tau, int(alpha)))


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(LIB)
    return _default


def normals_f32(*args, **kw):
    return default().normals_f32(*args, **kw)


def normals_f64(*args, **kw):
    return default().normals_f64(*args, **kw)


def normals_f32_rows(*args, **kw):
    return default().normals_f32_rows(*args, **kw)


def abs_threshold_f32(*args, **kw):
    return default().abs_threshold_f32(*args, **kw)


def variant_f32(*args, **kw):
    return default().variant_f32(*args, **kw)


def variant_f64(*args, **kw):
    return default().variant_f64(*args, **kw)


def normals_frozen_f64(*args, **kw):
    return default().normals_frozen_f64(*args, **kw)


def normals_vjp_f64(*args, **kw):
    return default().normals_vjp_f64(*args, **kw)
