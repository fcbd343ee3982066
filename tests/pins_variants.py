"""Pins of the oracle's two variants of the estimator.

PAIR_REMOVAL tests each of the four perpendicular-pair normals that Eq. 7
averages on its own and averages the pairs that pass; MULTISCALE is the
authors' earlier single-pair estimator (Eqs. 1-3) averaged over pixel
offsets (Eqs. 4-6).  As in pins.py, each check takes an oracle instance and
raises AssertionError when the oracle disagrees with a fact fixed by the
paper or by geometry: Eq. 7's identity, exact planes, the first-order
truncation of a one-sided pair, the triple-product identity
n_jk . ray = alpha^2 d_j d_k / (fx fy), piecewise-planar step scenes whose
expected surviving pairs follow from the test's own lower bound, closed-form
thresholds, and symmetries of the binary32 decisions.
"""
from __future__ import annotations

import numpy as np

from synth import scenes
from pins import (FX0, FY0, CX0, CY0, H0, W0, VALID, BOUNDARY, INVALID,
                  camera_facing_plane, interior, rays)

PR, MS = "pair_removal", "multiscale"

# taps 1..5 of the stencil of Section 3.1 (index 0 unused) and the pairs of
# Eq. 7 in its order: (2,3), (3,4), (4,5), (5,2)
TAP_D = {1: (0, 0), 2: (1, 0), 3: (0, 1), 4: (-1, 0), 5: (0, -1)}
PAIRS = ((2, 3), (3, 4), (4, 5), (5, 2))


def _step_scene(H, W, fx, fy, cx, cy):
    """Planes meeting at steps: A left of column xs, B right of it above row
    ys, C right of it below, and a one-pixel column S inside A (thinner than
    any stencil, so its own pixels keep no pair); B, C and S lie at least
    0.45 m behind A."""
    xs, ys = W // 2, H // 2
    nA = camera_facing_plane(25.0, 30.0)
    nB = camera_facing_plane(35.0, 160.0)
    nC = camera_facing_plane(20.0, 250.0)
    nS = camera_facing_plane(10.0, 90.0)
    dA = scenes.plane_depth(H, W, fx, fy, cx, cy, nA, -1.6)
    dB = scenes.plane_depth(H, W, fx, fy, cx, cy, nB, -2.6)
    dC = scenes.plane_depth(H, W, fx, fy, cx, cy, nC, -3.2)
    dS = scenes.plane_depth(H, W, fx, fy, cx, cy, nS, -2.4)
    lab = np.zeros((H, W), dtype=np.int32)
    lab[:ys, xs:] = 1
    lab[ys:, xs:] = 2
    lab[:, xs // 2] = 3
    d = np.choose(lab, [dA, dB, dC, dS])
    assert np.all(d > 0) and np.min(np.minimum(np.minimum(dB, dC), dS) - dA) > 0.45
    return d, lab, np.stack([nA, nB, nC, nS])


def _expected_keep(lab, a):
    """Bit p set where both taps of pair p lie on the plane of tap 1."""
    H, W = lab.shape
    keep = np.zeros((H, W), dtype=np.uint8)
    for y in range(a, H - a):
        for x in range(a, W - a):
            own = lab[y, x]
            for p, (j, k) in enumerate(PAIRS):
                tj = lab[y + a * TAP_D[j][1], x + a * TAP_D[j][0]]
                tk = lab[y + a * TAP_D[k][1], x + a * TAP_D[k][0]]
                if tj == own and tk == own:
                    keep[y, x] |= 1 << p
    return keep


# ----------------------------------------------------------------------------
# PAIR_REMOVAL
# ----------------------------------------------------------------------------

def pin_pairs_all_kept_is_eq7(o):
    """With every pair passing (no test), the average of the four pair
    normals is Eq. 7's n: same codes and FP64 normals as the four-pair
    method; and under REL a pixel whose four pairs all pass is VALID in the
    four-pair method with the same normal (rho of an average of vectors with
    positive ray components is at most the largest pair rho)."""
    s = scenes.make_scene(40, 52, fx=60.0, fy=66.0, cx=24.5, cy=18.0, seed=21)
    a = o.variant_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 2, "none", method=PR, want_keep=True,
                      gap=True)
    b = o.variant_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 2, "none", method="four_pair")
    assert np.array_equal(a["mask"], b["mask"])
    assert np.all(a["keep"][a["mask"] == VALID] == 15)
    assert np.abs(a["normals"] - b["normals"]).max() <= 1e-12
    assert a["gap"] <= 1e-10, f"sum of pair normals vs Eqs. 10-12: {a['gap']:.3g}"
    a = o.variant_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 2, "rel", 2.0, method=PR, want_keep=True)
    b = o.variant_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 2, "rel", 2.0, method="four_pair")
    full = a["keep"] == 15
    assert full.sum() > 200 and (a["keep"][a["mask"] == VALID] != 15).sum() > 20
    assert np.all(b["mask"][full] == VALID)
    assert np.abs(a["normals"][full] - b["normals"][full]).max() <= 1e-12
    assert np.all(a["keep"][b["mask"] == BOUNDARY] != 15)


def pin_pairs_plane_exact_f64(o):
    """On a plane every pair's tangents lie in the plane, so each pair normal
    and their average are the plane normal (FP64 rounding only)."""
    for alpha in (1, 3):
        for th, ph, c in ((0.0, 0.0, 2.0), (40.0, 75.0, 1.8), (30.0, 220.0, 2.9)):
            n = camera_facing_plane(th, ph)
            d = scenes.plane_depth(H0, W0, FX0, FY0, CX0, CY0, n, -c)
            out = o.variant_f64(d, FX0, FY0, CX0, CY0, alpha, "rel", 4.0, method=PR,
                                want_keep=True)
            inn = interior(H0, W0, alpha)
            assert np.all(out["mask"][inn] == VALID) and np.all(out["keep"][inn] == 15)
            assert np.abs(out["normals"][inn] - n).max() <= 1e-12


def pin_pairs_ray_component(o):
    """Triple-product identity: each pair has n_jk . ray = alpha^2 d_j d_k /
    (fx fy), so the average of the passing pairs has r / rho equal to the
    mean of alpha^2 d_h d_v / (fx fy) over them.  Checked on the step scene,
    where pixels keep one to four pairs."""
    H, W, a = 30, 34, 2
    fx, fy, cx, cy = 250.0, 270.0, 15.5, 13.0
    d, lab, _ = _step_scene(H, W, fx, fy, cx, cy)
    out = o.variant_f64(d, fx, fy, cx, cy, a, "rel", 4.0, method=PR, want_keep=True,
                        want_r=True, want_rho=True)
    seen = set()
    for y in range(a, H - a):
        for x in range(a, W - a):
            k = int(out["keep"][y, x])
            if out["mask"][y, x] != VALID:
                continue
            seen.add(bin(k).count("1"))
            vals = []
            for p, (j, kk) in enumerate(PAIRS):
                if k & (1 << p):
                    dj = d[y + a * TAP_D[j][1], x + a * TAP_D[j][0]]
                    dk = d[y + a * TAP_D[kk][1], x + a * TAP_D[kk][0]]
                    vals.append(a * a * dj * dk / (fx * fy))
            want = np.mean(vals)
            got = out["r"][y, x] / out["rho"][y, x]
            assert abs(got - want) <= 1e-12 * want, (x, y, k, got, want)
    assert {1, 2, 4} <= seen, f"keep sizes seen: {sorted(seen)}"


def pin_pairs_step_keeps_own_plane(o):
    """Piecewise-planar steps: a pair with a tap across a step has
    rho >= fx |d_h - d1| / (alpha d_h) (its first component alone), far above
    tau here, so it fails; a pair with all three taps on one plane has the
    plane's rho, below tau for these tilts.  So the passing pairs are exactly
    those on the plane of tap 1, the pixel is BOUNDARY only when there is
    none, and a VALID pixel's normal is the exact normal of its own plane.
    FP64 decisions on exact depth, then binary32 decisions on rounded depth."""
    H, W = 30, 34
    fx, fy, cx, cy = 250.0, 270.0, 15.5, 13.0
    d, lab, nrm = _step_scene(H, W, fx, fy, cx, cy)
    for a in (1, 2):
        want_keep = _expected_keep(lab, a)
        inn = interior(H, W, a)
        want_code = np.where(inn, np.where(want_keep > 0, VALID, BOUNDARY), INVALID)
        for dd, f32 in ((d, False), (d.astype(np.float32), True)):
            fn = o.variant_f32 if f32 else o.variant_f64
            out = fn(dd, fx, fy, cx, cy, a, "rel", 4.0, method=PR, want_keep=True)
            assert np.array_equal(out["keep"], want_keep), f"alpha={a} f32={f32}"
            assert np.array_equal(out["mask"], want_code)
            v = out["mask"] == VALID
            err = np.abs(out["normals"][v] - nrm[lab[v]]).max()
            bound = 4 * 2.0 ** -24 * max(fx, fy) / a if f32 else 1e-9
            assert err <= bound, f"own-plane normal error {err:.3g} (alpha={a}, f32={f32})"
        assert (want_keep[inn] == 15).sum() > 0 and (want_keep[inn] == 0).sum() > 0


def pin_pairs_rel_split_matches_fp64(o):
    """The binary32 pair decisions agree with the FP64 decisions of the
    definition wherever the FP64 decision is clear of the threshold.  On a
    sphere each pair's rho = |n_p| / (n_p . ray) varies over the frame and
    among the four pairs of a pixel; tau is put at the median four-pair rho,
    so that many pairs fail and many pass, and a pair is clear when its FP64
    decision is the same at tau (1 - 1e-4) and tau (1 + 1e-4) (binary32
    rounding moves a rho by a few 1e-7).  Both sides see the same binary32
    depths."""
    H, W, a = 40, 48, 2
    fx, fy, cx, cy = 70.0, 64.0, 22.5, 19.0
    depth, _ = scenes.sphere_depth(H, W, fx, fy, cx, cy, (0.05, -0.04, 1.2), 0.55)
    d32 = depth.astype(np.float32)
    d64 = d32.astype(np.float64)
    assert np.all(np.isfinite(d64))
    inn = interior(H, W, a)
    rho = o.variant_f64(d64, fx, fy, cx, cy, a, "rel", 1e6, method="four_pair",
                        want_rho=True)["rho"]
    tau = float(np.median(rho[inn]))

    def keep64(t):
        return o.variant_f64(d64, fx, fy, cx, cy, a, "rel", t, method=PR, want_keep=True)["keep"]

    k64, lo, hi = keep64(tau), keep64(tau * (1 - 1e-4)), keep64(tau * (1 + 1e-4))
    k32 = o.variant_f32(d32, fx, fy, cx, cy, a, "rel", tau, method=PR, want_keep=True)["keep"]
    kept = failed = unclear = 0
    for p in range(4):
        b64, b32 = (k64[inn] >> p) & 1, (k32[inn] >> p) & 1
        clear = ((lo[inn] >> p) & 1) == ((hi[inn] >> p) & 1)
        assert np.array_equal(b32[clear], b64[clear]), f"pair {p}"
        kept += int((b64[clear] == 1).sum())
        failed += int((b64[clear] == 0).sum())
        unclear += int((~clear).sum())
    assert kept > 300 and failed > 300 and unclear < 20, (kept, failed, unclear)


def _pair_normals_bruteforce(d, x, y, a, fx, fy, cx, cy):
    """FP64 pair normals n_jk = (X_j - X_1) x (X_k - X_1) of Eq. 7 at pixel
    (x, y), each X back-projected with its own pixel offset (Eqs. 8-9)."""
    X = {}
    for t, (dx, dy) in TAP_D.items():
        xx, yy = x + a * dx, y + a * dy
        z = float(d[yy, xx])
        X[t] = np.array([(xx - cx) / fx * z, (yy - cy) / fy * z, z])
    return [np.cross(X[j] - X[1], X[k] - X[1]) for j, k in PAIRS]


def pin_pairs_overflow_of_kept_vector(o):
    """Binary32 degeneracy (R10) on the vectors pair removal keeps: a pixel
    is INVALID when a pair's |m_p|^2 or the |.|^2 of the kept vector (the
    closed form when all four pass, else the sum of the passing pairs)
    exceeds FLT_MAX, with m_p = -(fx fy / alpha) n_p.  A sphere scaled so
    that these squared lengths straddle FLT_MAX, decided by brute force in
    FP64 from the definition on the same binary32 depths: all pairs passing
    (REL tau = 1e6), and about half failing (tau at the median pair rho, on
    a larger scale); pixels whose decision sits within 1e-3 of the overflow
    or 1e-4 of tau are skipped."""
    H, W, a = 18, 22, 1
    fx, fy, cx, cy = 40.0, 36.0, 10.5, 8.0
    depth, _ = scenes.sphere_depth(H, W, fx, fy, cx, cy, (0.03, -0.02, 1.2), 0.55)
    k = fx * fy / a
    fmax = float(np.finfo(np.float32).max)
    pix = [(x, y) for y in range(a, H - a) for x in range(a, W - a)]

    def pairs(d, x, y):
        ray = np.array([(x - cx) / fx, (y - cy) / fy, 1.0])
        ns = _pair_normals_bruteforce(d, x, y, a, fx, fy, cx, cy)
        return ns, [np.linalg.norm(n) / float(n @ ray) for n in ns]

    rho_med = float(np.median([r for x, y in pix for r in pairs(depth, x, y)[1]]))
    seen = {}
    for tau in (1e6, rho_med):
        # scale: the median |.|^2 of the kept vectors (of the sums of fewer than
        # four pairs in the second pass) at FLT_MAX; it grows as depth^4
        qk = []
        for x, y in pix:
            ns, rho = pairs(depth, x, y)
            kept = [n for n, r in zip(ns, rho) if r <= tau]
            if kept and (tau > 1e5 or len(kept) < 4):  # the second pass scales to the sums
                qk.append((k * np.linalg.norm(np.sum(kept, axis=0))) ** 2)
        d32 = (depth * (fmax / float(np.median(qk))) ** 0.25).astype(np.float32)
        d64 = d32.astype(np.float64)
        got = o.variant_f32(d32, fx, fy, cx, cy, a, "rel", tau, method=PR)["mask"]
        for x, y in pix:
            ns, rho = pairs(d64, x, y)
            if min(abs(r / tau - 1.0) for r in rho) < 1e-4:
                continue
            kept = [n for n, r in zip(ns, rho) if r <= tau]
            if not kept:
                continue
            vals = [(k * np.linalg.norm(n)) ** 2 for n in ns]
            vals.append((k * np.linalg.norm(np.sum(kept, axis=0))) ** 2)
            if min(abs(v / fmax - 1.0) for v in vals) < 1e-3:
                continue
            want = INVALID if max(vals) > fmax else VALID
            assert got[y, x] == want, (tau, x, y, len(kept), [v / fmax for v in vals])
            key = ("closed" if len(kept) == 4 else "sum", want)
            seen[key] = seen.get(key, 0) + 1
    for key, least in ((("closed", VALID), 40), (("closed", INVALID), 40), (("sum", VALID), 10),
                       (("sum", INVALID), 10)):
        assert seen.get(key, 0) >= least, seen


def pin_pairs_fronto_thresholds(o):
    """Fronto plane at depth D: every pair vector is (0, 0, -alpha C) with
    C = D^2, so |m|^2 = (alpha C)^2 exactly and REL passes iff tau >= 1.
    Each pair's r = |n_jk| = alpha^2 D^2 / (fx fy): with D = 2, fx = fy = 512
    and alpha = 2 that is 2^-14 exactly, and ABS flips there."""
    Hs, Ws = 11, 13
    for D in (0.5, 1.37, 3.99):
        d = np.full((Hs, Ws), D, dtype=np.float32)
        inn = interior(Hs, Ws, 2)
        ok = o.variant_f32(d, 500.0, 520.0, 6.0, 5.0, 2, "rel", 1.0, method=PR, want_keep=True)
        assert np.all(ok["mask"][inn] == VALID) and np.all(ok["keep"][inn] == 15)
        bad = o.variant_f32(d, 500.0, 520.0, 6.0, 5.0, 2, "rel", 0.9999999, method=PR)
        assert np.all(bad["mask"][inn] == BOUNDARY)
    d = np.full((Hs, Ws), 2.0, dtype=np.float32)
    inn = interior(Hs, Ws, 2)
    r = 2.0 ** -14
    at = o.variant_f32(d, 512.0, 512.0, 6.0, 5.0, 2, "abs", r, method=PR)
    assert np.all(at["mask"][inn] == VALID)
    below = o.variant_f32(d, 512.0, 512.0, 6.0, 5.0, 2, "abs",
                          float(np.nextafter(np.float32(r), np.float32(0))), method=PR)
    assert np.all(below["mask"][inn] == BOUNDARY)


def pin_pairs_symmetries(o):
    """Binary32 decisions: depth x 2^k leaves codes and passing pairs
    unchanged (every |m|^2 and threshold scales by 2^4k); a column mirror
    with cx -> W-1-cx swaps taps 2 and 4 (pairs 0<->1, 2<->3) and negates
    the x component; a row mirror swaps taps 3 and 5 (pairs 0<->3, 1<->2)."""
    s = scenes.make_scene(36, 44, fx=58.0, fy=63.0, cx=20.0, cy=17.5, seed=23)
    H, W = s.depth.shape
    base = o.variant_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 1, "rel", 2.0, method=PR,
                         want_keep=True)
    assert (base["mask"] == BOUNDARY).sum() > 5 and ((base["keep"] > 0) & (base["keep"] < 15)).sum() > 20
    for k in (-3, 2):
        sc = o.variant_f32(s.depth * np.float32(2.0 ** k), s.fx, s.fy, s.cx, s.cy, 1, "rel", 2.0,
                           method=PR, want_keep=True)
        assert np.array_equal(sc["mask"], base["mask"]) and np.array_equal(sc["keep"], base["keep"])

    def perm(keep, mp):
        out = np.zeros_like(keep)
        for p, q in enumerate(mp):
            out |= ((keep >> p) & 1) << q
        return out

    m = o.variant_f32(np.ascontiguousarray(s.depth[:, ::-1]), s.fx, s.fy, (W - 1) - s.cx, s.cy, 1,
                      "rel", 2.0, method=PR, want_keep=True)
    assert np.array_equal(m["mask"][:, ::-1], base["mask"])
    assert np.array_equal(perm(m["keep"][:, ::-1], (1, 0, 3, 2)), base["keep"])
    v = base["mask"] == VALID
    assert np.abs(m["normals"][:, ::-1][..., 0][v] + base["normals"][..., 0][v]).max() < 1e-12
    m = o.variant_f32(np.ascontiguousarray(s.depth[::-1, :]), s.fx, s.fy, s.cx, (H - 1) - s.cy, 1,
                      "rel", 2.0, method=PR, want_keep=True)
    assert np.array_equal(m["mask"][::-1, :], base["mask"])
    assert np.array_equal(perm(m["keep"][::-1, :], (3, 2, 1, 0)), base["keep"])


# ----------------------------------------------------------------------------
# MULTISCALE
# ----------------------------------------------------------------------------

def pin_ms_single_pair_definition(o):
    """Eqs. 1-3 are the closed form of s12 x s13: the oracle's gap between
    them is rounding only, and its K = 1 output equals -n/|n| of the cross
    product of the back-projected tangents computed here."""
    rng = np.random.default_rng(31)
    d = rng.uniform(0.6, 3.5, size=(18, 21))
    for a in (1, 2):
        out = o.variant_f64(d, FX0, FY0, CX0, CY0, a, "none", method=MS, scales=1, gap=True)
        assert out["gap"] <= 1e-10
        H, W = d.shape
        for y in range(0, H - a):
            for x in range(0, W - a):
                def X(xx, yy):
                    z = d[yy, xx]
                    return np.array([(xx - CX0) / FX0 * z, (yy - CY0) / FY0 * z, z])
                n = np.cross(X(x + a, y) - X(x, y), X(x, y + a) - X(x, y))
                want = -n / np.linalg.norm(n)
                assert out["mask"][y, x] == VALID
                assert np.abs(out["normals"][y, x] - want).max() <= 1e-12
    f = rng.uniform(0.6, 3.5, size=(18, 21)).astype(np.float32)
    out = o.variant_f32(f, FX0, FY0, CX0, CY0, 2, "none", method=MS, scales=3, gap=True)
    assert out["gap"] <= 1e-10


def pin_ms_average_of_scales(o):
    """Eqs. 4-6: the K-scale vector is the average of the single-scale
    vectors at offsets alpha, 2 alpha, .., K alpha (recovered as -out * r from
    K = 1 runs at those offsets)."""
    rng = np.random.default_rng(33)
    d = rng.uniform(0.8, 3.0, size=(20, 24))
    for alpha, K in ((1, 3), (2, 2)):
        ms = o.variant_f64(d, FX0, FY0, CX0, CY0, alpha, "none", method=MS, scales=K, want_r=True)
        acc = np.zeros(d.shape + (3,))
        for i in range(1, K + 1):
            one = o.variant_f64(d, FX0, FY0, CX0, CY0, alpha * i, "none", method=MS, scales=1,
                                want_r=True)
            acc += -one["normals"] * one["r"][..., None]
        acc /= K
        v = ms["mask"] == VALID
        assert v.sum() > 100
        got = -ms["normals"][v] * ms["r"][v][:, None]
        scale = np.linalg.norm(acc[v], axis=1).max()
        assert np.abs(got - acc[v]).max() <= 1e-12 * scale


def pin_ms_plane_exact_f64(o):
    """One-sided tangents of a plane lie in the plane: every scale, and the
    average, is the plane normal."""
    for alpha, K in ((1, 1), (1, 4), (2, 3)):
        for th, ph, c in ((0.0, 0.0, 2.0), (45.0, 10.0, 1.6), (25.0, 300.0, 3.3)):
            n = camera_facing_plane(th, ph)
            d = scenes.plane_depth(H0, W0, FX0, FY0, CX0, CY0, n, -c)
            out = o.variant_f64(d, FX0, FY0, CX0, CY0, alpha, "rel", 4.0, method=MS, scales=K)
            v = np.zeros((H0, W0), dtype=bool)
            v[:H0 - alpha * K, :W0 - alpha * K] = True
            assert np.all(out["mask"][v] == VALID)
            assert np.abs(out["normals"][v] - n).max() <= 1e-12


def pin_ms_sphere_first_order(o):
    """A one-sided pair is a first-order difference: on a sphere its error
    against the analytic normal halves when the focal length doubles, for
    one scale and for an average of scales (unlike the second-order
    four-pair form)."""
    C, R = (0.04, -0.03, 2.0), 0.5
    for alpha, K in ((1, 1), (1, 2)):
        errs = []
        for f in (525.0, 1050.0, 2100.0):
            half = int(round(0.1 * f))
            n = 2 * half + 1
            d, nn = scenes.sphere_depth(n, n, f, f, float(half), float(half), C, R)
            out = o.variant_f64(d, f, f, float(half), float(half), alpha, "none", method=MS,
                                scales=K)
            v = out["mask"] == VALID
            errs.append(np.abs(out["normals"][v] - nn[v]).max())
        r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
        assert 1.7 < r1 < 2.3 and 1.7 < r2 < 2.3, f"ratios {r1:.3f} {r2:.3f}"


def pin_ms_border_and_taps(o):
    """Only (x + i alpha, y) and (x, y + i alpha) are read: the INVALID
    border is K alpha wide on the right and bottom only, and a bad depth
    invalidates exactly itself and the pixels i alpha to its left and above."""
    Hs, Ws = 19, 23
    for alpha, K in ((1, 3), (2, 2)):
        reach = alpha * K
        d = np.full((Hs, Ws), 1.7, dtype=np.float32)
        out = o.variant_f32(d, FX0, FY0, CX0, CY0, alpha, "rel", 4.0, method=MS, scales=K)
        exp = np.zeros((Hs, Ws), dtype=bool)
        exp[:, Ws - reach:] = True
        exp[Hs - reach:, :] = True
        assert np.array_equal(out["mask"] == INVALID, exp)
        for bad in (0.0, np.nan, -2.0):
            dd = d.copy()
            x0, y0 = 11, 9
            dd[y0, x0] = bad
            out = o.variant_f32(dd, FX0, FY0, CX0, CY0, alpha, "rel", 4.0, method=MS, scales=K)
            e = exp.copy()
            e[y0, x0] = True
            for i in range(1, K + 1):
                e[y0, x0 - i * alpha] = True
                e[y0 - i * alpha, x0] = True
            assert np.array_equal(out["mask"] == INVALID, e)


def pin_ms_fronto_thresholds(o):
    """Fronto plane at depth D: each scale's vector is (0, 0, -a_i D^2), the
    weighted sum is (0, 0, -D^2 sum a_i^2), so REL passes iff tau >= 1; and
    r of the average is D^2 (sum a_i^2) / (K fx fy), where ABS flips."""
    Hs, Ws = 12, 14
    for D in (0.5, 2.25):
        d = np.full((Hs, Ws), D, dtype=np.float32)
        ok = o.variant_f32(d, 500.0, 520.0, 6.0, 5.0, 1, "rel", 1.0, method=MS, scales=3)
        bad = o.variant_f32(d, 500.0, 520.0, 6.0, 5.0, 1, "rel", 0.9999999, method=MS, scales=3)
        v = ok["mask"] != INVALID
        assert v.sum() > 50 and np.all(ok["mask"][v] == VALID) and np.all(bad["mask"][v] == BOUNDARY)
    d = np.full((Hs, Ws), 2.0, dtype=np.float32)
    for alpha, K in ((1, 3), (2, 2), (4, 1)):
        a2 = sum((i * alpha) ** 2 for i in range(1, K + 1))
        r = 4.0 * a2 / (K * 512.0 * 512.0)
        hi = o.variant_f32(d, 512.0, 512.0, 6.0, 5.0, alpha, "abs", r * (1 + 1e-6), method=MS,
                           scales=K)
        lo = o.variant_f32(d, 512.0, 512.0, 6.0, 5.0, alpha, "abs", r * (1 - 1e-6), method=MS,
                           scales=K)
        v = hi["mask"] != INVALID
        assert v.sum() > 30
        assert np.all(hi["mask"][v] == VALID) and np.all(lo["mask"][v] == BOUNDARY), (alpha, K)


def pin_ms_symmetries(o):
    """Binary32 decisions: depth x 2^k leaves the codes unchanged, and the
    pair (2, 3) maps to itself under a transpose with fx <-> fy, cx <-> cy,
    so the codes transpose exactly."""
    s = scenes.make_scene(34, 40, fx=55.0, fy=61.0, cx=19.5, cy=16.0, seed=37)
    base = o.variant_f32(s.depth, s.fx, s.fy, s.cx, s.cy, 1, "rel", 2.0, method=MS, scales=2)
    assert (base["mask"] == BOUNDARY).sum() > 5
    for k in (-2, 3):
        sc = o.variant_f32(s.depth * np.float32(2.0 ** k), s.fx, s.fy, s.cx, s.cy, 1, "rel", 2.0,
                           method=MS, scales=2)
        assert np.array_equal(sc["mask"], base["mask"])
    t = o.variant_f32(np.ascontiguousarray(s.depth.T), s.fy, s.fx, s.cy, s.cx, 1, "rel", 2.0,
                      method=MS, scales=2)
    assert np.array_equal(t["mask"].T, base["mask"])
    v = base["mask"] == VALID
    tn = np.transpose(t["normals"], (1, 0, 2))
    assert np.abs(tn[..., 0][v] - base["normals"][..., 1][v]).max() < 1e-12


VARIANT_PINS = [
    pin_pairs_rel_split_matches_fp64,
    pin_pairs_overflow_of_kept_vector,
    pin_pairs_all_kept_is_eq7,
    pin_pairs_plane_exact_f64,
    pin_pairs_ray_component,
    pin_pairs_step_keeps_own_plane,
    pin_pairs_fronto_thresholds,
    pin_pairs_symmetries,
    pin_ms_single_pair_definition,
    pin_ms_average_of_scales,
    pin_ms_plane_exact_f64,
    pin_ms_sphere_first_order,
    pin_ms_border_and_taps,
    pin_ms_fronto_thresholds,
    pin_ms_symmetries,
]
