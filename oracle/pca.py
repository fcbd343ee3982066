"""Brute-force plane-PCA normals -- TEST INFRASTRUCTURE ONLY.

Plane-PCA (the classical estimator the paper reviews in its introduction,
and, with a 5x5 window of 25 neighbours, the ground truth it uses for real
depth maps in Section 4): back-project the neighbourhood of a pixel, form the
3x3 scatter matrix about the centroid and take the eigenvector of the
smallest eigenvalue as the surface normal.  Orientation: the side facing the
camera (n . X < 0 at the query point X).

Used on tiny frames only, pixel by pixel, with numpy's symmetric
eigensolver as the one library step.
"""
from __future__ import annotations

from typing import Iterable, Optional, Tuple

import numpy as np


def backproject(col: float, row: float, d: float, fx: float, fy: float,
                cx: float, cy: float) -> np.ndarray:
    """X = (u d, v d, d), u = (col - cx)/fx, v = (row - cy)/fy (Eqs. 8-9)."""
    return np.array([(col - cx) / fx * d, (row - cy) / fy * d, d], dtype=np.float64)


def pca_normal(points: np.ndarray, query: np.ndarray) -> np.ndarray:
    """Smallest-eigenvalue eigenvector of the scatter matrix, camera-facing."""
    P = np.asarray(points, dtype=np.float64)
    c = P.mean(axis=0)
    D = P - c
    M = D.T @ D
    w, V = np.linalg.eigh(M)
    n = V[:, 0]
    if n @ query > 0:
        n = -n
    return n / np.linalg.norm(n)


def stencil_offsets(alpha: int) -> Tuple[Tuple[int, int], ...]:
    """(dx, dy) of taps 1..5: centre, +x, +y, -x, -y at distance alpha."""
    a = int(alpha)
    return ((0, 0), (a, 0), (0, a), (-a, 0), (0, -a))


def window_offsets(half: int = 2) -> Tuple[Tuple[int, int], ...]:
    """The (2*half+1)^2 window; half=2 gives the 25-neighbour fit."""
    return tuple((dx, dy) for dy in range(-half, half + 1) for dx in range(-half, half + 1))


def pca_normals(depth: np.ndarray, fx: float, fy: float, cx: float, cy: float,
                offsets: Iterable[Tuple[int, int]],
                pixels: Optional[Iterable[Tuple[int, int]]] = None) -> np.ndarray:
    """Plane-PCA normal at each pixel whose whole neighbourhood is inside the
    image with finite positive depth; NaN elsewhere.  Pure Python loop: tiny
    frames or a short pixel list only."""
    depth = np.asarray(depth, dtype=np.float64)
    H, W = depth.shape
    offs = list(offsets)
    out = np.full((H, W, 3), np.nan)
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
            pts.append(backproject(xx, yy, d, fx, fy, cx, cy))
        if not ok:
            continue
        q = backproject(x, y, depth[y, x], fx, fy, cx, cy)
        out[y, x] = pca_normal(np.array(pts), q)
    return out
