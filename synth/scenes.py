"""Seeded synthetic depth scenes for tests and benchmarks.

This module only builds inputs: it ray-casts simple primitives in FP64, adds
the depth-sensor noise and hole model, and reports the analytic geometry
(clean depth, face labels and the true camera-facing surface normal) that the
oracle's closed-form tests compare against.  It contains none of the normal
estimator's arithmetic, and both the oracle and the GPU path consume its
output unchanged.

Camera model: pinhole with z-depth.  Pixel (x, y) -- x the column, y the row --
looks along ray (u, v, 1) with u = (x - cx)/fx and v = (y - cy)/fy, and a hit
at ray parameter t is the point t*(u, v, 1) whose depth is z = t.  This is
the back-projection X = (u d, v d, d) of the paper's Section 3.1 (Eqs. 8-9).

Scene recipe (one frame):
  * a fronto-parallel wall at z = 4.0 m behind everything;
  * tilted finite planes: sides 0.6-1.5 m, normal 15-50 degrees off the
    optical axis, centre depth 1-3 m;
  * spheres: radius 0.2-0.5 m, centre depth 1-3.5 m;
  * boxes: edges 0.3-0.8 m, yaw -45..45 degrees, front depth 0.8-2.5 m;
  * every object stays at least 0.3 m in front of the wall, so every
    silhouette is a depth step;
  * noisy depth = float32(clean + N(0,1) * 0.001 * clean^2), i.e. a
    quadratic-in-range noise model of a time-of-flight / structured-light
    sensor (0.25 mm at 0.5 m, 16 mm at 4 m);
  * holes: each pixel independently set to 0.0 with probability 0.02.

The random stream is numpy's PCG64 seeded with the frame seed and drawn in a
fixed order (objects, then noise, then holes), so a seed fixes the frame
byte for byte.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

WALL_Z = 4.0
NOISE_K = 0.001
HOLE_P = 0.02


@dataclasses.dataclass
class Scene:
    depth: np.ndarray          # float32 [H, W]: noisy depth with holes (0.0)
    depth_clean: np.ndarray    # float64 [H, W]: exact ray-cast z-depth
    labels: np.ndarray         # uint16 [H, W]: 0 = wall, one id per primitive face
    normals: np.ndarray        # float64 [H, W, 3]: analytic camera-facing unit normals
    fx: float
    fy: float
    cx: float
    cy: float
    seed: int
    prims: list                # primitive descriptions (dicts)

    @property
    def shape(self) -> Tuple[int, int]:
        return self.depth.shape

    @property
    def intrinsics(self) -> Tuple[float, float, float, float]:
        return (self.fx, self.fy, self.cx, self.cy)


# ----------------------------------------------------------------------------
# camera helpers
# ----------------------------------------------------------------------------

def pixel_rays(H: int, W: int, fx: float, fy: float, cx: float, cy: float,
               x0: int = 0, x1: Optional[int] = None,
               y0: int = 0, y1: Optional[int] = None) -> np.ndarray:
    """Unnormalised rays (u, v, 1) for the pixel rectangle [y0,y1) x [x0,x1)."""
    x1 = W if x1 is None else x1
    y1 = H if y1 is None else y1
    xs = (np.arange(x0, x1, dtype=np.float64) - cx) / fx
    ys = (np.arange(y0, y1, dtype=np.float64) - cy) / fy
    r = np.empty((y1 - y0, x1 - x0, 3), dtype=np.float64)
    r[..., 0] = xs[None, :]
    r[..., 1] = ys[:, None]
    r[..., 2] = 1.0
    return r


def _bbox(center: np.ndarray, radius: float, H: int, W: int,
          fx: float, fy: float, cx: float, cy: float):
    """Conservative pixel rectangle covering the ball (center, radius).

    For a point P of the ball, P.x lies in [Cx-R, Cx+R] and P.z in
    [Cz-R, Cz+R] (Cz-R > 0), and x/z over that rectangle takes its extremes
    at the corners.  Two pixels of margin cover rounding.
    """
    zlo = center[2] - radius
    zhi = center[2] + radius
    if zlo <= 1e-6:
        return 0, W, 0, H
    def span(c, f, o, n):
        vals = [(c + s * radius) / z for s in (-1.0, 1.0) for z in (zlo, zhi)]
        lo = int(np.floor(f * min(vals) + o)) - 2
        hi = int(np.ceil(f * max(vals) + o)) + 3
        return max(lo, 0), min(hi, n)
    xa, xb = span(center[0], fx, cx, W)
    ya, yb = span(center[1], fy, cy, H)
    return xa, xb, ya, yb


def _point_at_pixel(rng, H, W, fx, fy, cx, cy, z, margin=0.15):
    px = rng.uniform(margin * W, (1 - margin) * W)
    py = rng.uniform(margin * H, (1 - margin) * H)
    return np.array([(px - cx) / fx * z, (py - cy) / fy * z, z], dtype=np.float64)


# ----------------------------------------------------------------------------
# primitives: each returns (t, normal, face) on its pixel rectangle; t = inf on
# a miss.  Rays are given by their u (columns) and v (rows) coordinates; the
# third ray component is 1.
# ----------------------------------------------------------------------------

def _lin(c, u, v):
    """c0*u + c1*v + c2 over the (rows, cols) grid, by broadcasting."""
    return (c[0] * u)[None, :] + (c[1] * v)[:, None] + c[2]


def _hit_plane(u, v, p):
    n, C, e1, e2, h1, h2 = p["n"], p["C"], p["e1"], p["e2"], p["h1"], p["h2"]
    den = _lin(n, u, v)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (n @ C) / den
    # (t*ray - C).e = t*(ray.e) - C.e
    a1 = t * _lin(e1, u, v) - (C @ e1)
    a2 = t * _lin(e2, u, v) - (C @ e2)
    ok = (t > 0) & (np.abs(a1) <= h1) & (np.abs(a2) <= h2) & np.isfinite(t)
    t = np.where(ok, t, np.inf)
    sgn = np.where(den > 0, -1.0, 1.0)    # camera-facing side
    nn = sgn[..., None] * n
    return t, nn, np.zeros(t.shape, dtype=np.int32)


def _hit_sphere(u, v, p):
    C, R = p["C"], p["R"]
    rr = (u * u)[None, :] + (v * v)[:, None] + 1.0
    rc = _lin(C, u, v)
    disc = rc * rc - rr * (C @ C - R * R)
    with np.errstate(invalid="ignore"):
        t = (rc - np.sqrt(disc)) / rr
    ok = (disc >= 0) & (t > 0)
    t = np.where(ok, t, np.inf)
    tt = np.where(ok, t, 0.0)
    nn = np.empty(t.shape + (3,), dtype=np.float64)
    nn[..., 0] = (tt * u[None, :] - C[0]) / R
    nn[..., 1] = (tt * v[:, None] - C[1]) / R
    nn[..., 2] = (tt - C[2]) / R
    return t, nn, np.zeros(t.shape, dtype=np.int32)


def _hit_box(u, v, p):
    C, Rm, h = p["C"], p["R"], p["h"]        # Rm: local->world rotation
    o = Rm.T @ (-C)                           # camera centre in the box frame
    tn = np.full((v.size, u.size), -np.inf)
    tf = np.full((v.size, u.size), np.inf)
    axis = np.zeros((v.size, u.size), dtype=np.int32)
    dsel = np.zeros((v.size, u.size))
    for k in range(3):
        d = _lin(Rm[:, k], u, v)              # k-th local component of the ray
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (-h[k] - o[k]) / d
            t2 = (h[k] - o[k]) / d
        lo = np.fmin(t1, t2)
        hi = np.fmax(t1, t2)
        lo = np.where(np.isnan(lo), -np.inf, lo)
        hi = np.where(np.isnan(hi), np.inf, hi)
        better = lo > tn
        tn = np.where(better, lo, tn)
        axis = np.where(better, k, axis)
        dsel = np.where(better, d, dsel)
        tf = np.minimum(tf, hi)
    ok = (tn <= tf) & (tn > 0)
    t = np.where(ok, tn, np.inf)
    sgn = -np.sign(dsel)                      # outward face normal faces the camera
    nn = np.zeros(t.shape + (3,), dtype=np.float64)
    for k in range(3):
        sel = (axis == k) * sgn
        nn += sel[..., None] * Rm[:, k]
    face = axis * 2 + (sgn > 0)
    return t, nn, face.astype(np.int32)


_HIT = {"plane": _hit_plane, "sphere": _hit_sphere, "box": _hit_box}
_NFACES = {"plane": 1, "sphere": 1, "box": 6}


# ----------------------------------------------------------------------------
# random primitives
# ----------------------------------------------------------------------------

def _rand_plane(rng, H, W, fx, fy, cx, cy):
    z = rng.uniform(1.0, 3.0)
    C = _point_at_pixel(rng, H, W, fx, fy, cx, cy, z)
    th = np.deg2rad(rng.uniform(15.0, 50.0))
    ph = rng.uniform(0.0, 2.0 * np.pi)
    n = -np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    a = np.cross(n, [0.0, 1.0, 0.0]); a /= np.linalg.norm(a)
    b = np.cross(n, a)
    psi = rng.uniform(0.0, np.pi)
    e1 = np.cos(psi) * a + np.sin(psi) * b
    e2 = np.cross(n, e1)
    h1 = 0.5 * rng.uniform(0.6, 1.5)
    h2 = 0.5 * rng.uniform(0.6, 1.5)
    return {"kind": "plane", "n": n, "C": C, "e1": e1, "e2": e2, "h1": h1, "h2": h2,
            "radius": float(np.hypot(h1, h2))}


def _rand_sphere(rng, H, W, fx, fy, cx, cy):
    R = rng.uniform(0.2, 0.5)
    z = rng.uniform(1.0, 3.5)
    C = _point_at_pixel(rng, H, W, fx, fy, cx, cy, z)
    return {"kind": "sphere", "C": C, "R": R, "radius": R}


def _rand_box(rng, H, W, fx, fy, cx, cy):
    h = 0.5 * rng.uniform(0.3, 0.8, size=3)
    yaw = np.deg2rad(rng.uniform(-45.0, 45.0))
    zf = rng.uniform(0.8, 2.5)
    c, s = np.cos(yaw), np.sin(yaw)
    Rm = np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
    # centre so that the nearest corner sits at depth zf
    zext = abs(Rm[2, 0]) * h[0] + abs(Rm[2, 2]) * h[2]
    C = _point_at_pixel(rng, H, W, fx, fy, cx, cy, zf + zext)
    return {"kind": "box", "C": C, "R": Rm, "h": h, "radius": float(np.linalg.norm(h))}


_RAND = {"plane": _rand_plane, "sphere": _rand_sphere, "box": _rand_box}


# ----------------------------------------------------------------------------
# frame assembly
# ----------------------------------------------------------------------------

def render(H: int, W: int, fx: float, fy: float, cx: float, cy: float,
           prims: Sequence[dict], wall_z: Optional[float] = WALL_Z):
    """Ray-cast `prims` (nearest hit wins) in front of a fronto wall.

    Returns (depth_clean float64, labels uint16, normals float64 [H,W,3]).
    With wall_z=None there is no wall and unhit pixels get depth +inf.
    """
    depth = np.full((H, W), np.inf if wall_z is None else float(wall_z))
    labels = np.zeros((H, W), dtype=np.uint16)
    normals = np.zeros((H, W, 3), dtype=np.float64)
    if wall_z is not None:
        normals[..., 2] = -1.0
    next_id = 1
    for p in prims:
        xa, xb, ya, yb = _bbox(p["C"], p["radius"], H, W, fx, fy, cx, cy)
        base = next_id
        next_id += _NFACES[p["kind"]]
        if xa >= xb or ya >= yb:
            continue
        u = (np.arange(xa, xb, dtype=np.float64) - cx) / fx
        v = (np.arange(ya, yb, dtype=np.float64) - cy) / fy
        t, nn, face = _HIT[p["kind"]](u, v, p)
        sub = depth[ya:yb, xa:xb]
        win = t < sub
        sub[win] = t[win]
        labels[ya:yb, xa:xb][win] = (base + face[win]).astype(np.uint16)
        normals[ya:yb, xa:xb][win] = nn[win]
    return depth, labels, normals


def make_scene(H: int, W: int, *, fx: float, fy: Optional[float] = None,
               cx: Optional[float] = None, cy: Optional[float] = None,
               n_planes: int = 2, n_spheres: int = 3, n_boxes: int = 1,
               seed: int = 1, noise: bool = True, hole_p: float = HOLE_P,
               prims: Optional[Sequence[dict]] = None, noise_k: float = NOISE_K) -> Scene:
    """One seeded frame: primitives in front of the wall, noise of standard
    deviation noise_k * z^2 and holes."""
    fy = fx if fy is None else fy
    cx = (W - 1) / 2.0 if cx is None else cx
    cy = (H - 1) / 2.0 if cy is None else cy
    rng = np.random.default_rng(seed)
    if prims is None:
        prims = []
        for kind, k in (("plane", n_planes), ("sphere", n_spheres), ("box", n_boxes)):
            for _ in range(k):
                prims.append(_RAND[kind](rng, H, W, fx, fy, cx, cy))
    clean, labels, normals = render(H, W, fx, fy, cx, cy, prims)
    if noise:
        z = rng.standard_normal((H, W))
        noisy = clean + z * (noise_k * clean * clean)
    else:
        noisy = clean.copy()
    depth = noisy.astype(np.float32)
    if hole_p > 0:
        holes = rng.random((H, W)) < hole_p
        depth[holes] = 0.0
    return Scene(depth=depth, depth_clean=clean, labels=labels, normals=normals,
                 fx=float(fx), fy=float(fy), cx=float(cx), cy=float(cy), seed=seed,
                 prims=list(prims))


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

def frame_640x480(seed: int = 1, **kw) -> Scene:
    """640x480, fx=fy=525, principal point (319.5, 239.5), 2 planes + 3 spheres + 1 box."""
    return make_scene(480, 640, fx=525.0, cx=319.5, cy=239.5,
                      n_planes=2, n_spheres=3, n_boxes=1, seed=seed, **kw)


def frame_1920x1080(seed: int = 2, **kw) -> Scene:
    """1920x1080, fx=fy=1050, centred principal point, 4 planes + 4 spheres + 4 boxes."""
    return make_scene(1080, 1920, fx=1050.0, cx=959.5, cy=539.5,
                      n_planes=4, n_spheres=4, n_boxes=4, seed=seed, **kw)


def scaled_intrinsics(H: int, W: int) -> Tuple[float, float, float, float]:
    """fx=fy scaled from 525 at 640 columns; principal point at the centre."""
    f = 525.0 * W / 640.0
    return (f, f, (W - 1) / 2.0, (H - 1) / 2.0)


def sized_frame(H: int, W: int, seed: int, **kw) -> Scene:
    fx, fy, cx, cy = scaled_intrinsics(H, W)
    if W <= 640:
        counts = dict(n_planes=2, n_spheres=3, n_boxes=1)
    else:
        counts = dict(n_planes=4, n_spheres=4, n_boxes=4)
    return make_scene(H, W, fx=fx, fy=fy, cx=cx, cy=cy, seed=seed, **counts, **kw)


# (count, H, W) of the 256-frame mixed batch, in frame order
BATCH_MIX: List[Tuple[int, int, int]] = [(64, 240, 320), (96, 480, 640),
                                         (64, 720, 1280), (32, 1080, 1920)]


def batch_shapes(mix: Sequence[Tuple[int, int, int]] = BATCH_MIX) -> List[Tuple[int, int]]:
    out = []
    for k, H, W in mix:
        out += [(H, W)] * k
    return out


def batch_frames(seed0: int = 1000, mix: Sequence[Tuple[int, int, int]] = BATCH_MIX,
                 indices: Optional[Sequence[int]] = None, workers: int = 0,
                 **kw) -> List[Scene]:
    """The mixed batch; frame i has seed seed0 + i.  `indices` picks a subset."""
    shapes = batch_shapes(mix)
    idx = list(range(len(shapes))) if indices is None else list(indices)
    jobs = [(shapes[i][0], shapes[i][1], seed0 + i, kw) for i in idx]
    if workers and workers > 1 and len(jobs) > 1:
        import concurrent.futures as cf
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(_sized_job, jobs))
    return [_sized_job(j) for j in jobs]


def _sized_job(job):
    H, W, seed, kw = job
    return sized_frame(H, W, seed, **kw)


# request sizes of the serving stream
SERVE_SIZES: List[Tuple[int, int]] = [(240, 320), (480, 640), (720, 1280),
                                      (1080, 1920), (3072, 4096)]


# ----------------------------------------------------------------------------
# analytic primitives for closed-form tests
# ----------------------------------------------------------------------------

def plane_depth(H: int, W: int, fx: float, fy: float, cx: float, cy: float,
                n: Sequence[float], c: float) -> np.ndarray:
    """Exact FP64 z-depth of the infinite plane {X : n.X = c} seen by every pixel."""
    rays = pixel_rays(H, W, fx, fy, cx, cy)
    n = np.asarray(n, dtype=np.float64)
    return c / (rays @ n)


def sphere_depth(H: int, W: int, fx: float, fy: float, cx: float, cy: float,
                 C: Sequence[float], R: float):
    """FP64 z-depth and outward normal of a sphere; +inf where the ray misses."""
    p = {"C": np.asarray(C, dtype=np.float64), "R": float(R)}
    u = (np.arange(W, dtype=np.float64) - cx) / fx
    v = (np.arange(H, dtype=np.float64) - cy) / fy
    t, nn, _ = _hit_sphere(u, v, p)
    return t, nn
