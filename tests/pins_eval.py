"""Pins of the evaluation oracle (oracle/evaluation.py): the angle images of
Eqs. 14-15 against spherical coordinates, the MSE against hand-counted
cases, and the plane fit against exact planes and its validity footprint."""
from __future__ import annotations

import numpy as np

from oracle import evaluation as oev
from pins import camera_facing_plane
from synth import scenes

VALID, INVALID = 0, 2


def pin_angles_closed_forms():
    """Axis directions and a diagonal have known spherical angles; I_phi is
    wrapped into [0, 2 pi)."""
    cases = {(0, 0, 1): (0.0, 0.0), (0, 0, -1): (np.pi, 0.0), (1, 0, 0): (np.pi / 2, 0.0),
             (0, 1, 0): (np.pi / 2, np.pi / 2), (-1, 0, 0): (np.pi / 2, np.pi),
             (0, -1, 0): (np.pi / 2, 1.5 * np.pi), (0, 0, 0): (0.0, 0.0),
             (1, 1, 0): (np.pi / 2, np.pi / 4), (1, -1, -np.sqrt(2)): (0.75 * np.pi, 1.75 * np.pi)}
    n = np.array([list(k) for k in cases], dtype=np.float64)
    n[:, :] /= np.maximum(np.linalg.norm(n, axis=1, keepdims=True), 1e-300)
    t, p = oev.angle_images(n[None])
    for i, (th, ph) in enumerate(cases.values()):
        assert abs(t[0, i] - th) < 1e-12 and abs(p[0, i] - ph) < 1e-12, (list(cases)[i], t[0, i], p[0, i])


def pin_angles_round_trip():
    """n = (sin t cos p, sin t sin p, cos t) gives back (t, p) for t in
    (0, pi), p in [0, 2 pi)."""
    rng = np.random.default_rng(41)
    t = rng.uniform(1e-3, np.pi - 1e-3, 5000)
    p = rng.uniform(0.0, 2 * np.pi, 5000)
    n = np.stack([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)], axis=-1)
    tt, pp = oev.angle_images(n[None])
    assert np.abs(tt[0] - t).max() < 1e-12
    assert np.abs(pp[0] - p).max() < 1e-11
    assert pp.min() >= 0.0 and pp.max() < 2 * np.pi


def pin_mse_hand_case():
    """Two 2x2 maps: one pixel masked in each, the other two differ by known
    angles."""
    a = np.zeros((2, 2, 3))
    b = np.zeros((2, 2, 3))
    a[0, 0] = (0, 0, -1)                      # theta pi, phi 0
    b[0, 0] = (np.sin(3.0), 0, np.cos(3.0))   # theta 3, phi 0
    a[0, 1] = (0, 1, 0)                       # theta pi/2, phi pi/2
    b[0, 1] = (-1, 0, 0)                      # theta pi/2, phi pi
    a[1, 0] = b[1, 0] = (1, 0, 0)
    ma = np.array([[VALID, VALID], [VALID, INVALID]], dtype=np.uint8)
    mb = np.array([[VALID, VALID], [INVALID, VALID]], dtype=np.uint8)
    mt, mp, k = oev.angle_mse(a, ma, b, mb)
    assert k == 2
    assert abs(mt - ((np.pi - 3.0) ** 2 + 0.0) / 2) < 1e-15
    assert abs(mp - (0.0 + (np.pi / 2) ** 2) / 2) < 1e-15
    assert oev.angle_mse(a, ma, a, ma) == (0.0, 0.0, 3)
    assert oev.angle_mse(a, ma, b, np.full((2, 2), INVALID, np.uint8)) == (0.0, 0.0, 0)


def pin_plane_fit_exact_planes():
    """Coplanar window points: the fit is the plane's normal (camera-facing),
    and the smallest eigenvalue is 0 to rounding."""
    H, W = 14, 17
    fx, fy, cx, cy = 410.0, 445.0, 7.5, 6.25
    for th, ph, c in ((0.0, 0.0, 2.0), (35.0, 120.0, 1.7), (50.0, 300.0, 2.6)):
        n = camera_facing_plane(th, ph)
        d = scenes.plane_depth(H, W, fx, fy, cx, cy, n, -c)
        for r in (1, 2, 3):
            out, codes, eigs = oev.plane_fit(d, fx, fy, cx, cy, r)
            v = codes == VALID
            inner = np.zeros((H, W), bool)
            inner[r:H - r, r:W - r] = True
            assert np.array_equal(v, inner)
            assert np.abs(out[v] - n).max() < 1e-9
            assert np.all(eigs[v][:, 0] <= 1e-12 * eigs[v][:, 2])
            assert np.all(out[~v] == 0)


def pin_plane_fit_footprint():
    """A bad depth invalidates exactly the pixels whose window holds it."""
    H, W, r = 15, 16, 2
    d = np.full((H, W), 1.3)
    d[7, 9] = 0.0
    _, codes, _ = oev.plane_fit(d, 500.0, 500.0, 7.5, 7.0, r)
    exp = np.ones((H, W), bool)
    exp[r:H - r, r:W - r] = False
    exp[7 - r:7 + r + 1, 9 - r:9 + r + 1] = True
    assert np.array_equal(codes == INVALID, exp)


def pin_plane_fit_sphere():
    """On a sphere the 25-point fit approaches the analytic normal at second
    order in the pixel pitch: within 1e-4 at f = 1050."""
    f = 1050.0
    H = W = 31
    d, nn = scenes.sphere_depth(H, W, f, f, 15.0, 15.0, (0.02, 0.01, 1.5), 0.4)
    pts = [(x, y) for y in range(3, H - 3, 4) for x in range(3, W - 3, 4)]
    out, codes, _ = oev.plane_fit(d, f, f, 15.0, 15.0, 2, pixels=pts)
    for x, y in pts:
        assert codes[y, x] == VALID
        assert np.abs(out[y, x] - nn[y, x]).max() < 1e-4


EVAL_PINS = [pin_angles_closed_forms, pin_angles_round_trip, pin_mse_hand_case,
             pin_plane_fit_exact_planes, pin_plane_fit_footprint, pin_plane_fit_sphere]
