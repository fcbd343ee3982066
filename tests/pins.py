"""Checks that pin the oracle to facts fixed by the paper and by geometry.

Each check takes an oracle instance (oracle.Oracle) and raises AssertionError
when the oracle disagrees with the fact.  tests/test_oracle_pins.py runs them
on the real oracle; tests/test_oracle_mutants.py runs them on copies of the
oracle with a planted mistake and requires that at least one check fails.

None of the expected values below comes from the oracle itself: they are
exact plane / sphere geometry, algebraic identities, symmetries of the
binary32 decision, brute-force plane-PCA, or closed-form thresholds.
"""
from __future__ import annotations

import numpy as np

from oracle import pca
from synth import scenes

VALID, BOUNDARY, INVALID = 0, 1, 2


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

def camera_facing_plane(theta_deg: float, phi_deg: float) -> np.ndarray:
    th, ph = np.deg2rad(theta_deg), np.deg2rad(phi_deg)
    return -np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])


def rays(H, W, fx, fy, cx, cy):
    return scenes.pixel_rays(H, W, fx, fy, cx, cy)


def interior(H, W, a):
    m = np.zeros((H, W), dtype=bool)
    m[a:H - a, a:W - a] = True
    return m


# Intrinsics with fx != fy and an off-centre principal point, so that a
# swapped axis, focal length or principal-point coordinate changes results.
H0, W0 = 40, 56
FX0, FY0, CX0, CY0 = 500.0, 560.0, 31.25, 17.5


# ----------------------------------------------------------------------------
# geometry pins
# ----------------------------------------------------------------------------

def pin_plane_exact_f64(o):
    """A plane's central-difference tangents lie in the plane, so the
    estimate equals the plane normal exactly (Eq. 7 / Eqs. 10-12 on exact
    depth); FP64 leaves only rounding, bounded here by 1e-12."""
    for alpha in (1, 2, 3):
        for th, ph, c in ((0.0, 0.0, 2.0), (35.0, 20.0, 1.7), (55.0, 200.0, 2.4),
                          (20.0, 290.0, 3.1)):
            n = camera_facing_plane(th, ph)
            d = scenes.plane_depth(H0, W0, FX0, FY0, CX0, CY0, n, -c)
            assert np.all(d > 0)
            out = o.normals_f64(d, FX0, FY0, CX0, CY0, alpha=alpha, mode="none")
            inn = interior(H0, W0, alpha)
            assert np.all(out["mask"][inn] == VALID), "interior plane pixels must be valid"
            err = np.abs(out["normals"][inn] - n).max()
            assert err <= 1e-12, f"plane normal error {err:.3g} (alpha={alpha}, th={th})"


def pin_plane_f32_bound(o):
    """Binary32-rounded plane depth perturbs each tap by at most 2^-24
    relative; over a tangent of length about alpha*d/f that tilts the normal
    by at most a few times 2^-24 * f / alpha.  Checked with the bound
    4 * 2^-24 * max(fx, fy) / alpha."""
    for alpha in (1, 2):
        n = camera_facing_plane(40.0, 65.0)
        d = scenes.plane_depth(H0, W0, FX0, FY0, CX0, CY0, n, -2.2).astype(np.float32)
        out = o.normals_f32(d, FX0, FY0, CX0, CY0, alpha=alpha, mode="none")
        inn = interior(H0, W0, alpha)
        assert np.all(out["mask"][inn] == VALID)
        err = np.abs(out["normals"][inn] - n).max()
        bound = 4 * 2.0 ** -24 * max(FX0, FY0) / alpha
        assert err <= bound, f"f32 plane error {err:.3g} > {bound:.3g}"


def pin_sphere_second_order(o):
    """On a sphere the central differences of Eq. 7 are second-order: the
    error against the analytic normal (X - C)/R falls about 4x each time the
    focal length (pixel density) doubles over the same region."""
    C, R = (0.04, -0.03, 2.0), 0.5
    errs = []
    for f in (525.0, 1050.0, 2100.0):
        half = int(round(0.1 * f))               # |u|, |v| <= 0.1
        Hs = Ws = 2 * half + 1
        cx = cy = float(half)
        d, nn = scenes.sphere_depth(Hs, Ws, f, f, cx, cy, C, R)
        assert np.all(np.isfinite(d))
        out = o.normals_f64(d, f, f, cx, cy, alpha=1, mode="none")
        inn = interior(Hs, Ws, 1)
        e = np.abs(out["normals"][inn] - nn[inn]).max()
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert errs[0] < 1e-3, f"sphere error at f=525 too large: {errs[0]:.3g}"
    assert 3.2 < r1 < 4.8 and 3.2 < r2 < 4.8, f"sphere error ratios {r1:.3f}, {r2:.3f}"


def pin_pca_planar(o):
    """Brute-force plane-PCA of the 5 stencil points and of the 25-point 5x5
    window equals the estimate on planar depth (all points coplanar)."""
    n = camera_facing_plane(30.0, 140.0)
    Hs, Ws = 12, 14
    fx, fy, cx, cy = 400.0, 430.0, 5.5, 7.25
    d = scenes.plane_depth(Hs, Ws, fx, fy, cx, cy, n, -1.9)
    for alpha in (1, 2):
        out = o.normals_f64(d, fx, fy, cx, cy, alpha=alpha, mode="none")
        p5 = pca.pca_normals(d, fx, fy, cx, cy, pca.stencil_offsets(alpha))
        p25 = pca.pca_normals(d, fx, fy, cx, cy, pca.window_offsets(2))
        inn = interior(Hs, Ws, max(alpha, 2))
        assert np.abs(out["normals"][inn] - p5[inn]).max() < 1e-9
        assert np.abs(out["normals"][inn] - p25[inn]).max() < 1e-9


def pin_pca_sphere(o):
    """On a sphere the estimate and the 5-point plane-PCA both approach the
    analytic normal at second order; at f=1050 both are within 1e-4 of it and
    of each other."""
    f = 1050.0
    Hs = Ws = 31
    cx = cy = 15.0
    d, nn = scenes.sphere_depth(Hs, Ws, f, f, cx, cy, (0.02, 0.01, 1.5), 0.4)
    out = o.normals_f64(d, f, f, cx, cy, alpha=1, mode="none")
    pts = [(x, y) for y in range(2, Hs - 2, 3) for x in range(2, Ws - 2, 3)]
    p5 = pca.pca_normals(d, f, f, cx, cy, pca.stencil_offsets(1), pixels=pts)
    for x, y in pts:
        assert np.abs(out["normals"][y, x] - nn[y, x]).max() < 1e-4
        assert np.abs(p5[y, x] - nn[y, x]).max() < 1e-4


def pin_eq7_identity(o):
    """Eq. 7: the average of the four perpendicular-pair cross products
    equals 0.25 s24 x s35 (Eqs. 10-12), for any depths, d1 included."""
    rng = np.random.default_rng(7)
    d = rng.uniform(0.5, 4.0, size=(24, 30)).astype(np.float32)
    out = o.normals_f32(d, FX0, FY0, CX0, CY0, alpha=1, mode="none", eq7=True)
    assert out["eq7_gap"] <= 1e-10, f"Eq. 7 gap {out['eq7_gap']:.3g}"
    dd = rng.uniform(0.5, 4.0, size=(24, 30))
    out = o.normals_f64(dd, FX0, FY0, CX0, CY0, alpha=2, mode="none", eq7=True)
    assert out["eq7_gap"] <= 1e-10, f"Eq. 7 gap {out['eq7_gap']:.3g}"


def pin_unit_and_facing(o):
    """Outputs are unit vectors, and camera-facing: n . (u, v, 1) < 0 holds
    for every valid pixel because the paper's n has
    n . (u, v, 1) = alpha^2 (d2+d4)(d3+d5) / (4 fx fy) > 0."""
    s = scenes.make_scene(48, 64, fx=70.0, fy=75.0, cx=30.5, cy=22.0, seed=11)
    out = o.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, alpha=2, mode="none")
    v = out["mask"] == VALID
    assert v.sum() > 500
    nrm = out["normals"][v]
    assert np.abs(np.linalg.norm(nrm, axis=1) - 1).max() < 1e-12
    r = rays(48, 64, s.fx, s.fy, s.cx, s.cy)[v]
    assert np.all(np.einsum("ij,ij->i", nrm, r) < 0)
    assert np.all(out["normals"][~v] == 0)


def pin_center_tap_unused(o):
    """Eqs. 10-12 do not contain d1: changing a pixel's own depth leaves its
    normal unchanged and changes the normals of the four pixels that use it
    as tap 2, 3, 4 or 5."""
    rng = np.random.default_rng(3)
    d = rng.uniform(1.0, 2.0, size=(20, 22)).astype(np.float32)
    a = 2
    base = o.normals_f32(d, FX0, FY0, CX0, CY0, alpha=a, mode="none")
    d2 = d.copy()
    x0, y0 = 10, 9
    d2[y0, x0] = 1.75
    new = o.normals_f32(d2, FX0, FY0, CX0, CY0, alpha=a, mode="none")
    assert np.array_equal(base["normals"][y0, x0], new["normals"][y0, x0])
    for (x, y) in ((x0 - a, y0), (x0 + a, y0), (x0, y0 - a), (x0, y0 + a)):
        assert not np.array_equal(base["normals"][y, x], new["normals"][y, x])
    changed = np.any(base["normals"] != new["normals"], axis=-1)
    assert changed.sum() == 4


def pin_invalid_taps(o):
    """A bad depth value (hole 0, negative, NaN, +-inf) invalidates exactly
    the pixel itself and the four pixels whose stencil reads it."""
    for bad in (0.0, -0.0, -1.0, np.nan, np.inf, -np.inf):
        for a in (1, 3):
            d = np.full((21, 23), 2.5, dtype=np.float32)
            x0, y0 = 11, 10
            d[y0, x0] = bad
            out = o.normals_f32(d, FX0, FY0, CX0, CY0, alpha=a, mode="rel", tau=4.0)
            exp = ~interior(21, 23, a)
            for (x, y) in ((x0, y0), (x0 - a, y0), (x0 + a, y0), (x0, y0 - a), (x0, y0 + a)):
                exp[y, x] = True
            got = out["mask"] == INVALID
            assert np.array_equal(got, exp), f"invalid pattern wrong for {bad} alpha={a}"


def pin_border(o):
    """A stencil that leaves the image makes the pixel INVALID: a border of
    width alpha; frames narrower than 2 alpha + 1 are all INVALID."""
    for a in (1, 2, 5):
        for (Hs, Ws) in ((17, 19), (2 * a + 1, 2 * a + 1), (2 * a, 30), (30, 2 * a)):
            d = np.full((Hs, Ws), 1.5, dtype=np.float32)
            out = o.normals_f32(d, FX0, FY0, 7.0, 6.0, alpha=a, mode="none")
            exp = np.where(interior(Hs, Ws, a), VALID, INVALID)
            assert np.array_equal(out["mask"], exp), f"border wrong a={a} {Hs}x{Ws}"
            cnt = np.bincount(out["mask"].ravel(), minlength=3)
            assert np.array_equal(out["counts"], cnt)


def pin_counts(o):
    s = scenes.frame_640x480(seed=5)
    out = o.normals_f32(s.depth, *s.intrinsics, alpha=2)
    cnt = np.bincount(out["mask"].ravel(), minlength=3)
    assert np.array_equal(out["counts"].astype(np.int64), cnt)
    assert int(out["counts"].sum()) == 480 * 640
    # the mask is applied to the normal map: masked pixels carry no normal
    assert cnt[BOUNDARY] > 0 and cnt[INVALID] > 0
    assert np.all(out["normals"][out["mask"] != VALID] == 0)
    assert np.all(np.abs(np.linalg.norm(out["normals"][out["mask"] == VALID], axis=-1) - 1) < 1e-12)


# ----------------------------------------------------------------------------
# binary32 decision pins
# ----------------------------------------------------------------------------

def _noisy(seed=21, H=60, W=80):
    # a scene with steps, noise and holes; cx, cy with few mantissa bits so
    # that mirrored principal points are exact
    return scenes.make_scene(H, W, fx=90.0, fy=96.0, cx=37.25, cy=28.5, seed=seed)


def pin_mask_scale_invariance(o):
    """Scaling every depth by 2^k scales |m|^2 and the REL threshold by
    2^(4k) exactly in binary32, so the REL mask is unchanged; ABS with tau
    scaled by 2^(2k) is unchanged too."""
    s = _noisy()
    for mode, tau in (("rel", 1.3), ("rel", 4.0), ("abs", 2e-4)):
        base = o.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, alpha=1, mode=mode, tau=tau)
        for k in (-3, 2, 5):
            dk = (s.depth * np.float32(2.0 ** k)).astype(np.float32)
            tk = tau * (4.0 ** k) if mode == "abs" else tau
            out = o.normals_f32(dk, s.fx, s.fy, s.cx, s.cy, alpha=1, mode=mode, tau=tk)
            assert np.array_equal(out["mask"], base["mask"]), f"{mode} mask not scale-invariant k={k}"
            assert np.array_equal(out["normals"], base["normals"])


def pin_mask_mirror(o):
    """Mirroring the columns with cx' = (W-1) - cx negates P and x - cx
    exactly, so the mask mirrors bit for bit and n_x changes sign."""
    s = _noisy()
    H, W = s.depth.shape
    for mode, tau in (("rel", 1.2), ("abs", 5e-4)):
        base = o.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, alpha=2, mode=mode, tau=tau)
        m = o.normals_f32(np.ascontiguousarray(s.depth[:, ::-1]), s.fx, s.fy,
                          (W - 1) - s.cx, s.cy, alpha=2, mode=mode, tau=tau)
        assert np.array_equal(m["mask"][:, ::-1], base["mask"])
        flip = m["normals"][:, ::-1].copy()
        flip[..., 0] *= -1
        assert np.array_equal(flip, base["normals"])
        v = o.normals_f32(np.ascontiguousarray(s.depth[::-1, :]), s.fx, s.fy,
                          s.cx, (H - 1) - s.cy, alpha=2, mode=mode, tau=tau)
        assert np.array_equal(v["mask"][::-1, :], base["mask"])
        flip = v["normals"][::-1, :].copy()
        flip[..., 1] *= -1
        assert np.array_equal(flip, base["normals"])


def pin_mask_transpose(o):
    """Transposing the image with fx <-> fy and cx <-> cy swaps P <-> Q and
    S <-> T; every binary32 step maps to a commuted copy of itself, so the
    mask transposes bit for bit and n_x <-> n_y."""
    s = _noisy()
    for mode, tau in (("rel", 1.5), ("abs", 3e-4)):
        base = o.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, alpha=1, mode=mode, tau=tau)
        t = o.normals_f32(np.ascontiguousarray(s.depth.T), s.fy, s.fx, s.cy, s.cx,
                          alpha=1, mode=mode, tau=tau)
        assert np.array_equal(t["mask"].T, base["mask"])
        tn = t["normals"].transpose(1, 0, 2)[..., [1, 0, 2]]
        assert np.abs(tn - base["normals"]).max() <= 1e-15


def pin_rel_fronto(o):
    """A fronto-parallel plane has d2 = d4 and d3 = d5, so P = Q = 0 and
    |m|^2 = (alpha S T)^2 exactly: REL fires iff tau^2 < 1 (rho = 1)."""
    for D in (0.5, 1.37, 3.99):
        d = np.full((12, 13), D, dtype=np.float32)
        inn = interior(12, 13, 2)
        for tau, fire in ((0.9999999, True), (0.5, True), (1.0, False), (1.0000001, False)):
            out = o.normals_f32(d, FX0, FY0, 6.0, 6.0, alpha=2, mode="rel", tau=tau)
            exp = BOUNDARY if fire else VALID
            assert np.all(out["mask"][inn] == exp), f"REL fronto D={D} tau={tau}"


def pin_abs_fronto(o):
    """ABS on a fronto plane at depth D: r = |n| = alpha^2 D^2 / (fx fy)
    (Eq. 12 with P = Q = 0).  With powers of two r is exact; tau at r does
    not fire (strict), just below fires, just above does not."""
    D, f, a = 2.0, 512.0, 2
    r = a * a * D * D / (f * f)
    d = np.full((10, 11), D, dtype=np.float32)
    inn = interior(10, 11, a)
    for tau, fire in ((r, False), (r * (1 - 2 ** -10), True), (r * (1 + 2 ** -10), False)):
        out = o.normals_f32(d, f, f, 5.0, 4.0, alpha=a, mode="abs", tau=tau)
        exp = BOUNDARY if fire else VALID
        assert np.all(out["mask"][inn] == exp), f"ABS fronto tau={tau}"
    out = o.normals_f64(d.astype(np.float64), f, f, 5.0, 4.0, alpha=a, mode="none", want_r=True)
    assert np.abs(out["r"][inn] - r).max() <= 1e-15 * r


def pin_rel_tilted_plane(o):
    """On a plane m is parallel to the plane normal and m . (u, v, 1) =
    -alpha S T, so rho = 1 / |n_p . (u, v, 1)| exactly.  The REL mask must
    fire exactly where that exceeds tau (pixels within 0.1% of the contour
    excluded)."""
    Hs, Ws = 48, 64
    fx, fy, cx, cy = 60.0, 64.0, 20.25, 30.5
    n = camera_facing_plane(62.0, 15.0)
    d = scenes.plane_depth(Hs, Ws, fx, fy, cx, cy, n, -1.5)
    dot = np.abs(rays(Hs, Ws, fx, fy, cx, cy) @ n)
    rho_true = 1.0 / dot
    out64 = o.normals_f64(d, fx, fy, cx, cy, alpha=1, mode="none", want_rho=True)
    inn = interior(Hs, Ws, 1) & np.all(np.isfinite(d) & (d > 0))
    assert np.abs(out64["rho"][inn] / rho_true[inn] - 1).max() < 1e-12
    tau = float(np.median(rho_true[inn]))
    out = o.normals_f32(d.astype(np.float32), fx, fy, cx, cy, alpha=1, mode="rel", tau=tau)
    keep = inn & (np.abs(rho_true / tau - 1) > 1e-3)
    fired = out["mask"] == BOUNDARY
    assert keep.sum() > 1000
    assert np.array_equal(fired[keep], (rho_true > tau)[keep])


def pin_step_edges(o):
    """Masks fire at every generated depth step and only at edges.

    rho >= fx |P| / (alpha S) (the x component of m alone), so a pixel whose
    taps 2 and 4 lie on different objects with |d2 - d4| >= 1.25 tau alpha
    (d2 + d4) / fx must be masked (likewise 3, 5 with fy).  Conversely a
    BOUNDARY pixel must have its five taps on more than one face, or touch a
    grazing surface: the true rho = 1/|n . (u, v, 1)| at one of its taps
    above tau / 1.25 (noise-free scenes, so nothing else can fire)."""
    for (a, tau, f, H, W, seed) in ((2, 4.0, 262.5, 240, 320, 31), (1, 4.0, 525.0, 480, 640, 33)):
        s = scenes.make_scene(H, W, fx=f, seed=seed, noise=False, hole_p=0.0)
        out = o.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, alpha=a, mode="rel", tau=tau)
        m = out["mask"]
        L = s.labels.astype(np.int32)
        D = s.depth.astype(np.float64)
        sl = np.s_[a:H - a, a:W - a]

        def sh(arr, dx, dy):
            return arr[a + dy:H - a + dy, a + dx:W - a + dx]
        taps = ((0, 0), (a, 0), (0, a), (-a, 0), (0, -a))
        d2, d3, d4, d5 = (sh(D, *t) for t in taps[1:])
        l1, l2, l3, l4, l5 = (sh(L, *t) for t in taps)
        stepx = (l2 != l4) & (np.abs(d2 - d4) >= 1.25 * tau * a * (d2 + d4) / s.fx)
        stepy = (l3 != l5) & (np.abs(d3 - d5) >= 1.25 * tau * a * (d3 + d5) / s.fy)
        e_step = stepx | stepy
        assert e_step.sum() > 100
        assert np.all(m[sl][e_step] != VALID), "a depth step was not masked"
        e_any = ~((l1 == l2) & (l1 == l3) & (l1 == l4) & (l1 == l5))
        R = rays(H, W, s.fx, s.fy, s.cx, s.cy)
        rho_true = 1.0 / np.abs(np.einsum("ijk,ijk->ij", s.normals, R))
        rho_taps = np.max([sh(rho_true, *t) for t in taps], axis=0)
        grazing = rho_taps > tau / 1.25
        fired = m[sl] == BOUNDARY
        assert fired.sum() > 100
        assert np.all((e_any | grazing)[fired]), "mask fired away from edges"


def pin_fp32_degenerate(o):
    """Binary32 |m|^2 overflow (depth 1e30; on a fronto plane |m|^2 is about
    16 alpha^2 d^4) or underflow below FLT_MIN (depth 1e-30) makes the pixel
    INVALID; depth 1e8 still fits."""
    for D in (1e30, 1e-30):
        d = np.full((9, 9), D, dtype=np.float32)
        out = o.normals_f32(d, FX0, FY0, 4.0, 4.0, alpha=1, mode="rel", tau=4.0)
        assert np.all(out["mask"] == INVALID)
    d = np.full((9, 9), 1e8, dtype=np.float32)
    out = o.normals_f32(d, FX0, FY0, 4.0, 4.0, alpha=1, mode="rel", tau=4.0)
    assert np.all(out["mask"][interior(9, 9, 1)] == VALID)


def pin_row_bands(o):
    """The row-band entries (rows [a, b) of a frame, in full-frame
    coordinates, written from the first element of the output) must place
    each row where the full-frame call puts it.  Two independent facts: on a
    binary32 plane the band's own rows are INVALID exactly where their
    full-frame row y is within alpha of the top or bottom edge, and VALID
    with the plane normal (within the binary32 bound) elsewhere; and on a
    noisy scene every method's band equals the matching rows of the
    full-frame output bit for bit.  Each band is written into buffers of the
    whole frame's size pre-filled with a sentinel, so a band written at the
    wrong offset shows as sentinel rows."""
    def band(method, scales, d, intr, a, rb, re, mode="rel"):
        H, W = d.shape
        nb = np.full((H, W, 3), -7.0)
        mb = np.full((H, W), 0xEE, dtype=np.uint8)
        if method == "four_pair_rows":
            r = o.normals_f32_rows(d, *intr, a, mode, 4.0, rb, re, out=(nb, mb))
        else:
            r = o.variant_f32(d, *intr, alpha=a, mode=mode, tau=4.0, method=method,
                              scales=scales, rows=(rb, re), out=(nb, mb))
        n = re - rb
        assert np.all(nb[n:] == -7.0) and np.all(mb[n:] == 0xEE), \
            f"{method}: band [{rb},{re}) wrote past its {n} rows"
        return nb[:n], mb[:n], r["counts"]

    # absolute row positions from a plane (independent of the full-frame call)
    n_pl = camera_facing_plane(30.0, 120.0)
    d = scenes.plane_depth(H0, W0, FX0, FY0, CX0, CY0, n_pl, -2.0).astype(np.float32)
    intr = (FX0, FY0, CX0, CY0)
    for a in (1, 2):
        for rb, re in ((0, 3), (1, 7), (5, 6), (H0 - 4, H0), (a + 3, H0 - 2)):
            nrm, msk, _ = band("four_pair_rows", 0, d, intr, a, rb, re, mode="none")
            ys = np.arange(rb, re)
            row_in = (ys >= a) & (ys <= H0 - 1 - a)
            col_in = (np.arange(W0) >= a) & (np.arange(W0) <= W0 - 1 - a)
            exp = np.where(row_in[:, None] & col_in[None, :], VALID, INVALID)
            assert np.array_equal(msk, exp), f"band [{rb},{re}) alpha={a}: rows misplaced"
            err = np.abs(nrm[exp == VALID] - n_pl).max() if np.any(exp == VALID) else 0.0
            assert err <= 4 * 2.0 ** -24 * max(FX0, FY0) / a, f"band plane error {err:.3g}"

    # every method's band equals the full frame's rows, bit for bit
    s = _noisy(seed=33, H=36, W=44)
    intr = s.intrinsics
    for method, scales, a in (("four_pair_rows", 0, 2), ("four_pair", 0, 1),
                              ("pair_removal", 0, 2), ("multiscale", 2, 1)):
        if method == "four_pair_rows":
            full = o.normals_f32(s.depth, *intr, alpha=a, mode="rel", tau=4.0)
        else:
            full = o.variant_f32(s.depth, *intr, alpha=a, mode="rel", tau=4.0, method=method,
                                 scales=scales)
        for rb, re in ((1, 4), (6, 7), (9, 36), (20, 36)):
            nrm, msk, cnt = band(method, scales, s.depth, intr, a, rb, re)
            assert np.array_equal(msk, full["mask"][rb:re]), f"{method} band [{rb},{re}) mask"
            assert np.array_equal(nrm, full["normals"][rb:re]), f"{method} band [{rb},{re})"
            assert np.array_equal(cnt.astype(np.int64), np.bincount(msk.ravel(), minlength=3))


ALL_PINS = [pin_plane_exact_f64, pin_plane_f32_bound, pin_sphere_second_order,
            pin_pca_planar, pin_pca_sphere, pin_eq7_identity, pin_unit_and_facing,
            pin_center_tap_unused, pin_invalid_taps, pin_border, pin_counts,
            pin_mask_scale_invariance, pin_mask_mirror, pin_mask_transpose,
            pin_rel_fronto, pin_abs_fronto, pin_rel_tilted_plane, pin_step_edges,
            pin_fp32_degenerate, pin_row_bands]
