"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle element by element."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import paper_2209_08241_amd as bn

# Per-component tolerance of the binary32 normal against the FP64 oracle.
NORMAL_TOL = 1e-5


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_gpu(depth: np.ndarray, stride_pad: int = 0):
    import torch
    H, W = depth.shape
    if stride_pad:
        buf = torch.full((H, W + stride_pad), float("nan"), dtype=torch.float32, device="cuda")
        buf[:, :W] = torch.from_numpy(np.ascontiguousarray(depth)).cuda()
        return buf[:, :W]
    return torch.from_numpy(np.ascontiguousarray(depth)).cuda()


def gpu_normals(depth: np.ndarray, fx, fy, cx, cy, alpha=2, mode="rel", tau=4.0, variant=0,
                stride_pad: int = 0):
    import torch
    d = to_gpu(depth, stride_pad)
    n, m, st = bn.estimate_normals(d, fx, fy, cx, cy, alpha, mode, tau, variant=variant)
    torch.cuda.synchronize()
    return n.cpu().numpy(), m.cpu().numpy(), st.cpu().numpy()


def assert_parity(ref: dict, normals: np.ndarray, mask: np.ndarray, stats=None,
                  tol: float = NORMAL_TOL, what: str = "") -> float:
    """Mask and counts bit-exact, normals within tol per component."""
    om = ref["mask"]
    if not np.array_equal(mask, om):
        bad = np.argwhere(mask != om)
        y, x = bad[0][:2]
        raise AssertionError(f"{what}: {len(bad)} mask mismatches; first at (x={x}, y={y}): "
                             f"gpu {mask[y, x]} oracle {om[y, x]}")
    err = np.abs(normals.astype(np.float64) - ref["normals"])
    e = float(err.max()) if err.size else 0.0
    if e > tol:
        y, x = np.unravel_index(np.argmax(err.max(axis=-1)), err.shape[:2])
        raise AssertionError(f"{what}: normal error {e:.3g} > {tol} at (x={x}, y={y}): gpu "
                             f"{normals[y, x]} oracle {ref['normals'][y, x]}")
    if stats is not None:
        cnt = [int(c) for c in ref["counts"]]
        got = [int(c) for c in stats[:3]]
        if got != cnt:
            raise AssertionError(f"{what}: counts {got} != oracle {cnt}")
    return e


def check_frame(depth, fx, fy, cx, cy, alpha=2, mode="rel", tau=4.0, variant=0,
                stride_pad=0, what=""):
    ref = oracle.normals_f32(depth, fx, fy, cx, cy, alpha, mode, tau)
    n, m, st = gpu_normals(depth, fx, fy, cx, cy, alpha, mode, tau, variant, stride_pad)
    return assert_parity(ref, n, m, st, what=what)
