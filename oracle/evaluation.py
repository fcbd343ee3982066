"""Evaluation quantities of Section 4 -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy definitions, checked by tests/pins_eval.py:
  * the spherical angle images of a normal map (Eqs. 14-15), with the
    quadrant-aware arctangent and I_phi wrapped into [0, 2 pi) (the paper
    writes tan^-1 of a ratio and states that the images lie in [0, 2 pi]);
  * the mean squared error of two angle images over the pixels that are
    VALID in both (the accuracy metric of Section 4);
  * the local plane fit over a (2r+1) x (2r+1) window (r = 2: the
    25-neighbour fit the paper uses as ground truth on real data), from the
    brute-force plane-PCA in oracle/pca.py.
Only the test-suite may import this module.
"""
from __future__ import annotations

import numpy as np

from oracle import pca

VALID, BOUNDARY, INVALID = 0, 1, 2


def angle_images(normals: np.ndarray):
    """(I_theta, I_phi) of an [H, W, 3] normal map, FP64.

    I_phi = atan2(ny, nx) taken into [0, 2 pi)   (Eq. 14)
    I_theta = atan2(sqrt(nx^2 + ny^2), nz)       (Eq. 15), in [0, pi]
    A zero vector gives (0, 0)."""
    n = np.asarray(normals, dtype=np.float64)
    nx, ny, nz = n[..., 0], n[..., 1], n[..., 2]
    phi = np.arctan2(ny, nx)
    phi = np.where(phi < 0.0, phi + 2.0 * np.pi, phi)
    theta = np.arctan2(np.sqrt(nx * nx + ny * ny), nz)
    return theta, phi


def angle_mse(normals_a, mask_a, normals_b, mask_b):
    """(MSE of I_theta, MSE of I_phi, pixel count) over the pixels whose code
    is VALID in both maps; (0, 0, 0) when there are none."""
    ta, pa = angle_images(normals_a)
    tb, pb = angle_images(normals_b)
    both = (np.asarray(mask_a) == VALID) & (np.asarray(mask_b) == VALID)
    k = int(both.sum())
    if k == 0:
        return 0.0, 0.0, 0
    return float(np.mean((ta[both] - tb[both]) ** 2)), float(np.mean((pa[both] - pb[both]) ** 2)), k


def plane_fit(depth, fx, fy, cx, cy, radius: int = 2, pixels=None):
    """Plane-fit normals over the (2 radius + 1)^2 window: the camera-facing
    eigenvector of the smallest eigenvalue of the window's scatter matrix.
    Returns (normals [H, W, 3] (0 where INVALID), codes (VALID / INVALID),
    eigenvalues [H, W, 3] ascending (NaN where INVALID)).  INVALID when the
    window leaves the image or holds a depth that is not finite and > 0.
    `pixels`: evaluate only these (x, y); the rest stay INVALID."""
    depth = np.asarray(depth, dtype=np.float64)
    H, W = depth.shape
    offs = pca.window_offsets(radius)
    normals = np.zeros((H, W, 3))
    codes = np.full((H, W), INVALID, dtype=np.uint8)
    eigs = np.full((H, W, 3), np.nan)
    if pixels is None:
        pixels = [(x, y) for y in range(H) for x in range(W)]
    for x, y in pixels:
        pts = []
        ok = True
        for dx, dy in offs:
            xx, yy = x + dx, y + dy
            if not (0 <= xx < W and 0 <= yy < H):
                ok = False
                break
            d = depth[yy, xx]
            if not (np.isfinite(d) and d > 0):
                ok = False
                break
            pts.append(pca.backproject(xx, yy, d, fx, fy, cx, cy))
        if not ok:
            continue
        P = np.array(pts)
        D = P - P.mean(axis=0)
        w = np.linalg.eigvalsh(D.T @ D)
        q = pca.backproject(x, y, depth[y, x], fx, fy, cx, cy)
        normals[y, x] = pca.pca_normal(P, q)
        codes[y, x] = VALID
        eigs[y, x] = w
    return normals, codes, eigs
