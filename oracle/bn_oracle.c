/*
 * bn_oracle.c -- plain, slow, FP64 CPU oracle of the boundary-aware normal
 * estimator (Moradi, Memarmoghadam, Laurendeau, "Fast, Accurate and Object
 * Boundary-Aware Surface Normal Estimation from Depth Maps").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library: it includes nothing but
 * the C standard library.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (no FMA contraction and no reassociation, so every float expression below
 * rounds exactly once per written operation, in the written order).
 *
 * What it computes, per pixel p = (x, y) of an organized depth map d, x the
 * column and y the row:
 *
 *  1. Stencil (Section 3.1, Eq. 7 and Eqs. 8-12): the query point 1 and its
 *     four neighbours at pixel distance alpha in the four main directions,
 *       1 = (x, y)   2 = (x+a, y)   3 = (x, y+a)   4 = (x-a, y)   5 = (x, y-a).
 *     This assignment is the one that turns the four-pair average of Eq. 7
 *     into the closed forms of Eqs. 10-12 (u runs with the column and fx,
 *     v with the row and fy, as in the pinhole model under Eq. 3).
 *  2. Validity (the paper is silent; this build's reading): the pixel is
 *     INVALID when the stencil leaves the image or a tap d1..d5 is not a
 *     finite positive depth.
 *  3. Normal, in FP64 (Section 3.1):
 *       definition  n_def = 0.25 (s12 x s13 + s13 x s14 + s14 x s15 + s15 x s12)
 *                   with s1k = X_k - X_1 and X_k = (u_k d_k, v_k d_k, d_k)
 *                   (Eq. 7, first two lines; back-projection of Eqs. 8-9);
 *       closed form n = (nx, ny, nz) of Eqs. 10-12.
 *     The two agree in exact arithmetic (Eq. 7's chain of identities); the
 *     oracle evaluates both and reports their largest relative difference.
 *     The paper's n points away from the camera: n . (u1, v1, 1) equals
 *     alpha^2 (d2+d4)(d3+d5) / (4 fx fy) > 0.  The output is the unit normal
 *     facing the camera, -n / |n|.
 *  4. Boundary test (Section 3.2, Eq. 13): the length r = |n| grows with the
 *     tangent lengths, so thresholding r marks pixels whose tangents cross a
 *     depth discontinuity.  The paper gives no threshold value; three modes:
 *       ABS : r > tau                      (tau in m^2, paper-literal)
 *       REL : r / (n . ray) > tau          (r relative to the r of a
 *                                           camera-facing plane with the same
 *                                           neighbour depths; scale-free)
 *       NONE: never.
 *     The decision is taken in IEEE binary32, in the fixed order written in
 *     fp32_code() below, on the scaled vector m = -(4 fx fy / alpha) n, so that
 *     a GPU implementation taking the same order reproduces it bit for bit.
 *     A pixel whose binary32 |m|^2 is not a finite number >= FLT_MIN (the
 *     length cannot be formed in binary32) is INVALID.
 *  5. Masked pixels (BOUNDARY or INVALID) output the zero vector (Section
 *     3.2: the mask is applied to the normal map), and the codes are counted.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ORC_VALID 0
#define ORC_BOUNDARY 1
#define ORC_INVALID 2

#define ORC_REL 0
#define ORC_ABS 1
#define ORC_NONE 2

#define ORC_OK 0
#define ORC_EARG 1

/* ---------------------------------------------------------------------- */
/* small FP64 vector helpers                                               */
/* ---------------------------------------------------------------------- */

static void sub3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}

static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double norm3(const double a[3])
{
    return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
}

/* Back-projection of pixel (col, row) with depth d (Eqs. 8-9):
 * X = (u d, v d, d), u = (col - cx)/fx, v = (row - cy)/fy. */
static void backproject(double col, double row, double d, double fx, double fy,
                        double cx, double cy, double X[3])
{
    double u = (col - cx) / fx;
    double v = (row - cy) / fy;
    X[0] = u * d;
    X[1] = v * d;
    X[2] = d;
}

/* Eq. 7, first two lines: the average of the normals of the four
 * perpendicular tangent pairs (2,3), (3,4), (4,5), (5,2) around point 1. */
static void normal_definition(const double X1[3], const double X2[3], const double X3[3],
                              const double X4[3], const double X5[3], double n[3])
{
    double s12[3], s13[3], s14[3], s15[3], c[3];
    sub3(X2, X1, s12);
    sub3(X3, X1, s13);
    sub3(X4, X1, s14);
    sub3(X5, X1, s15);
    n[0] = n[1] = n[2] = 0.0;
    cross3(s12, s13, c); n[0] += c[0]; n[1] += c[1]; n[2] += c[2];   /* n23 */
    cross3(s13, s14, c); n[0] += c[0]; n[1] += c[1]; n[2] += c[2];   /* n34 */
    cross3(s14, s15, c); n[0] += c[0]; n[1] += c[1]; n[2] += c[2];   /* n45 */
    cross3(s15, s12, c); n[0] += c[0]; n[1] += c[1]; n[2] += c[2];   /* n52 */
    n[0] *= 0.25;
    n[1] *= 0.25;
    n[2] *= 0.25;
}

/* Eqs. 10-12: closed-form components of 0.25 s24 x s35. */
static void normal_closed_form(double d2, double d3, double d4, double d5,
                               double u1, double v1, double fx, double fy,
                               double alpha, double n[3])
{
    n[0] = -alpha / (4.0 * fy) * (d3 + d5) * (d2 - d4);                 /* Eq. 10 */
    n[1] = -alpha / (4.0 * fx) * (d2 + d4) * (d3 - d5);                 /* Eq. 11 */
    n[2] = -u1 * n[0] - v1 * n[1]
           + alpha * alpha / (4.0 * fx * fy) * (d2 + d4) * (d3 + d5);   /* Eq. 12 */
}

static int tap_ok_f64(double d)
{
    return isfinite(d) && d > 0.0;
}

static int tap_ok_f32(float d)
{
    return isfinite(d) && d > 0.0f;
}

/* ABS threshold on the binary32 |m|^2 scale: r > tau  <=>  |m| > 4 fx fy tau / alpha,
 * since r = |n| = alpha |m| / (4 fx fy).  Computed once in double, in this
 * order, and rounded to binary32. */
static float abs_threshold_f32(float fx, float fy, float tau, int alpha)
{
    double k = 4.0 * (double)fx;
    k = k * (double)fy;
    k = k * (double)tau;
    k = k / (double)alpha;
    k = k * k;
    return (float)k;
}

/* The binary32 decision of step 4, in its fixed operation order.
 * m = (fx T P, fy S Q, -(xc T P + yc S Q + alpha S T)) with P = d2-d4,
 * S = d2+d4, Q = d3-d5, T = d3+d5, xc = x-cx, yc = y-cy; `mz` below holds
 * the negated third component.  Returns the pixel code. */
static int fp32_code(float d2, float d3, float d4, float d5, int x, int y,
                     float fx, float fy, float cx, float cy, int alpha,
                     int mode, float tau, float kabs)
{
    float P = d2 - d4;
    float S = d2 + d4;
    float Q = d3 - d5;
    float T = d3 + d5;
    float a = T * P;
    float b = S * Q;
    float c = S * T;
    float mx = fx * a;
    float my = fy * b;
    float xc = (float)x - cx;
    float yc = (float)y - cy;
    float xa = xc * a;
    float yb = yc * b;
    float t3 = xa + yb;
    float w = (float)alpha * c;
    float mz = t3 + w;
    float mx2 = mx * mx;
    float my2 = my * my;
    float mz2 = mz * mz;
    float q = (mx2 + my2) + mz2;
    if (!isfinite(q) || q < FLT_MIN)
        return ORC_INVALID;
    if (mode == ORC_NONE)
        return ORC_VALID;
    float h;
    if (mode == ORC_REL) {
        float tt = tau * tau;
        float ww = w * w;
        h = tt * ww;
    } else {
        h = kabs;
    }
    return (q > h) ? ORC_BOUNDARY : ORC_VALID;
}

static int check_common(int H, int W, int64_t stride, double fx, double fy, int alpha,
                        int mode, double tau)
{
    if (H < 0 || W < 0 || stride < W)
        return ORC_EARG;
    if (!(fx > 0.0) || !(fy > 0.0) || !isfinite(fx) || !isfinite(fy))
        return ORC_EARG;
    if (alpha < 1)
        return ORC_EARG;
    if (mode != ORC_REL && mode != ORC_ABS && mode != ORC_NONE)
        return ORC_EARG;
    if (mode != ORC_NONE && (!(tau > 0.0) || !isfinite(tau)))
        return ORC_EARG;
    return ORC_OK;
}

/* FP64 normal at an interior pixel whose taps are valid.  Writes the
 * camera-facing unit normal, r = |n|, rho = |n| / (n . ray) and the relative
 * max-norm gap between the Eq. 7 definition and Eqs. 10-12. */
static void pixel_normal(double d1, double d2, double d3, double d4, double d5,
                         int x, int y, double fx, double fy, double cx, double cy,
                         int alpha, double out[3], double *r, double *rho, double *gap)
{
    double a = (double)alpha;
    double u1 = ((double)x - cx) / fx;
    double v1 = ((double)y - cy) / fy;
    double n[3];
    normal_closed_form(d2, d3, d4, d5, u1, v1, fx, fy, a, n);
    double len = norm3(n);
    out[0] = -n[0] / len;
    out[1] = -n[1] / len;
    out[2] = -n[2] / len;
    *r = len;
    *rho = len / (n[0] * u1 + n[1] * v1 + n[2]);
    if (gap) {
        double X1[3], X2[3], X3[3], X4[3], X5[3], nd[3];
        backproject((double)x, (double)y, d1, fx, fy, cx, cy, X1);
        backproject((double)(x + alpha), (double)y, d2, fx, fy, cx, cy, X2);
        backproject((double)x, (double)(y + alpha), d3, fx, fy, cx, cy, X3);
        backproject((double)(x - alpha), (double)y, d4, fx, fy, cx, cy, X4);
        backproject((double)x, (double)(y - alpha), d5, fx, fy, cx, cy, X5);
        normal_definition(X1, X2, X3, X4, X5, nd);
        double e = 0.0;
        for (int k = 0; k < 3; ++k) {
            double dk = fabs(nd[k] - n[k]);
            if (dk > e) e = dk;
        }
        e = (len > 0.0) ? e / len : (e > 0.0 ? INFINITY : 0.0);
        if (e > *gap) *gap = e;
    }
}

/*
 * Binary32 depth in, FP64 normals out.  The validity and boundary decisions
 * follow steps 2 and 4 above (the latter in binary32).
 *
 *   depth      [H rows][stride] binary32, row-major
 *   normals    [H][W][3] FP64 out (camera-facing unit normal, or 0 if masked)
 *   mask       [H][W] codes out (0 valid, 1 boundary, 2 invalid)
 *   counts     [3] out: number of pixels per code (nullable)
 *   r_out      [H][W] out: FP64 r = |n| of Eqs. 10-12, NaN if INVALID (nullable)
 *   rho_out    [H][W] out: FP64 r / (n . ray), NaN if INVALID (nullable)
 *   eq7_gap    out: largest relative gap definition vs closed form over the
 *              non-INVALID pixels (nullable; when null the definition is skipped)
 *   row_begin, row_end: only rows [row_begin, row_end) of the frame are
 *              evaluated (in full-frame coordinates); the outputs hold those
 *              rows only.
 * Returns 0, or 1 on an argument error (nothing written).
 */
int bno_normals_f32_rows(const float *depth, int H, int W, int64_t stride,
                         float fx, float fy, float cx, float cy,
                         int alpha, int mode, float tau, int row_begin, int row_end,
                         double *normals, uint8_t *mask, uint64_t *counts,
                         double *r_out, double *rho_out, double *eq7_gap)
{
    if (check_common(H, W, stride, fx, fy, alpha, mode, tau) != ORC_OK)
        return ORC_EARG;
    if (row_begin < 0 || row_end > H || row_begin > row_end)
        return ORC_EARG;
    if ((H > 0 && W > 0) && (!depth || !normals || !mask))
        return ORC_EARG;
    float kabs = (mode == ORC_ABS) ? abs_threshold_f32(fx, fy, tau, alpha) : 0.0f;
    uint64_t cnt[3] = {0, 0, 0};
    double gap = 0.0;
    for (int y = row_begin; y < row_end; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)(y - row_begin) * W + x;
            int code = ORC_INVALID;
            double nrm[3] = {0.0, 0.0, 0.0};
            double r = NAN, rho = NAN;
            int inside = (x - alpha >= 0) && (x + alpha <= W - 1) &&
                         (y - alpha >= 0) && (y + alpha <= H - 1);
            if (inside) {
                const float *row = depth + (int64_t)y * stride;
                float d1 = row[x];
                float d2 = row[x + alpha];
                float d3 = depth[(int64_t)(y + alpha) * stride + x];
                float d4 = row[x - alpha];
                float d5 = depth[(int64_t)(y - alpha) * stride + x];
                if (tap_ok_f32(d1) && tap_ok_f32(d2) && tap_ok_f32(d3) &&
                    tap_ok_f32(d4) && tap_ok_f32(d5)) {
                    code = fp32_code(d2, d3, d4, d5, x, y, fx, fy, cx, cy, alpha,
                                     mode, tau, kabs);
                    if (code != ORC_INVALID) {
                        double out[3];
                        pixel_normal(d1, d2, d3, d4, d5, x, y, fx, fy, cx, cy, alpha,
                                     out, &r, &rho, eq7_gap ? &gap : NULL);
                        if (code == ORC_VALID) {
                            nrm[0] = out[0];
                            nrm[1] = out[1];
                            nrm[2] = out[2];
                        }
                    }
                }
            }
            normals[3 * i + 0] = nrm[0];
            normals[3 * i + 1] = nrm[1];
            normals[3 * i + 2] = nrm[2];
            mask[i] = (uint8_t)code;
            if (r_out) r_out[i] = r;
            if (rho_out) rho_out[i] = rho;
            cnt[code] += 1;
        }
    }
    if (counts) {
        counts[0] = cnt[0];
        counts[1] = cnt[1];
        counts[2] = cnt[2];
    }
    if (eq7_gap) *eq7_gap = gap;
    return ORC_OK;
}

/* The whole frame: bno_normals_f32_rows over rows [0, H). */
int bno_normals_f32(const float *depth, int H, int W, int64_t stride,
                    float fx, float fy, float cx, float cy,
                    int alpha, int mode, float tau,
                    double *normals, uint8_t *mask, uint64_t *counts,
                    double *r_out, double *rho_out, double *eq7_gap)
{
    return bno_normals_f32_rows(depth, H, W, stride, fx, fy, cx, cy, alpha, mode, tau,
                                0, H, normals, mask, counts, r_out, rho_out, eq7_gap);
}

/*
 * FP64 depth in, FP64 everything: for closed-form tests on exact depth.
 * Same validity rule (taps finite and > 0, stencil inside); the boundary
 * decision is taken in FP64 on r (ABS) or rho (REL).  Intrinsics in FP64.
 */
int bno_normals_f64(const double *depth, int H, int W, int64_t stride,
                    double fx, double fy, double cx, double cy,
                    int alpha, int mode, double tau,
                    double *normals, uint8_t *mask, uint64_t *counts,
                    double *r_out, double *rho_out, double *eq7_gap)
{
    if (check_common(H, W, stride, fx, fy, alpha, mode, tau) != ORC_OK)
        return ORC_EARG;
    if ((H > 0 && W > 0) && (!depth || !normals || !mask))
        return ORC_EARG;
    uint64_t cnt[3] = {0, 0, 0};
    double gap = 0.0;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            int code = ORC_INVALID;
            double nrm[3] = {0.0, 0.0, 0.0};
            double r = NAN, rho = NAN;
            int inside = (x - alpha >= 0) && (x + alpha <= W - 1) &&
                         (y - alpha >= 0) && (y + alpha <= H - 1);
            if (inside) {
                const double *row = depth + (int64_t)y * stride;
                double d1 = row[x];
                double d2 = row[x + alpha];
                double d3 = depth[(int64_t)(y + alpha) * stride + x];
                double d4 = row[x - alpha];
                double d5 = depth[(int64_t)(y - alpha) * stride + x];
                if (tap_ok_f64(d1) && tap_ok_f64(d2) && tap_ok_f64(d3) &&
                    tap_ok_f64(d4) && tap_ok_f64(d5)) {
                    double out[3];
                    pixel_normal(d1, d2, d3, d4, d5, x, y, fx, fy, cx, cy, alpha,
                                 out, &r, &rho, eq7_gap ? &gap : NULL);
                    if (!isfinite(r) || !(r > 0.0)) {
                        code = ORC_INVALID;
                    } else {
                        int fire = 0;
                        if (mode == ORC_ABS) fire = r > tau;
                        else if (mode == ORC_REL) fire = rho > tau;
                        code = fire ? ORC_BOUNDARY : ORC_VALID;
                    }
                    if (code == ORC_VALID) {
                        nrm[0] = out[0];
                        nrm[1] = out[1];
                        nrm[2] = out[2];
                    }
                }
            }
            normals[3 * i + 0] = nrm[0];
            normals[3 * i + 1] = nrm[1];
            normals[3 * i + 2] = nrm[2];
            mask[i] = (uint8_t)code;
            if (r_out) r_out[i] = r;
            if (rho_out) rho_out[i] = rho;
            cnt[code] += 1;
        }
    }
    if (counts) {
        counts[0] = cnt[0];
        counts[1] = cnt[1];
        counts[2] = cnt[2];
    }
    if (eq7_gap) *eq7_gap = gap;
    return ORC_OK;
}

/*
 * Differentiation (test infrastructure for the adjoint kernel).
 *
 * With the codes frozen (the mask is piecewise constant in the depth), the
 * output of a VALID pixel is out = -n/|n| with n the closed form of
 * Eqs. 10-12, a smooth function of its taps d2..d5 (d1 does not enter);
 * masked pixels output a constant 0.
 */

/* FP64 normals of the pixels whose given code is VALID (others 0). */
int bno_normals_frozen_f64(const double *depth, int H, int W, int64_t stride,
                           double fx, double fy, double cx, double cy, int alpha,
                           const uint8_t *codes, double *normals)
{
    if (check_common(H, W, stride, fx, fy, alpha, ORC_NONE, 1.0) != ORC_OK)
        return ORC_EARG;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            double *o = normals + 3 * i;
            o[0] = o[1] = o[2] = 0.0;
            if (codes[i] != ORC_VALID)
                continue;
            if (x - alpha < 0 || x + alpha > W - 1 || y - alpha < 0 || y + alpha > H - 1)
                return ORC_EARG;
            const double *row = depth + (int64_t)y * stride;
            double r, rho;
            pixel_normal(row[x], row[x + alpha], depth[(int64_t)(y + alpha) * stride + x],
                         row[x - alpha], depth[(int64_t)(y - alpha) * stride + x],
                         x, y, fx, fy, cx, cy, alpha, o, &r, &rho, NULL);
        }
    }
    return ORC_OK;
}

/*
 * Vector-Jacobian product of the frozen normal map:
 *   grad_depth[j] = sum over VALID pixels p of (d out_p / d depth_j) . grad_normals[p]
 * Chain rule through Eqs. 10-12, scattered pixel by pixel onto the four taps:
 *   g_n = d/dn of out . g = -(g - (nh . g) nh) / |n|,  nh = n/|n|
 *   with P = d2-d4, S = d2+d4, Q = d3-d5, T = d3+d5, u1 = (x-cx)/fx, v1 = (y-cy)/fy:
 *   dL/dP = (g_nx - u1 g_nz) (-alpha T / (4 fy))
 *   dL/dT = (g_nx - u1 g_nz) (-alpha P / (4 fy)) + g_nz alpha^2 S / (4 fx fy)
 *   dL/dQ = (g_ny - v1 g_nz) (-alpha S / (4 fx))
 *   dL/dS = (g_ny - v1 g_nz) (-alpha Q / (4 fx)) + g_nz alpha^2 T / (4 fx fy)
 *   d2 += dP + dS,  d4 += -dP + dS,  d3 += dQ + dT,  d5 += -dQ + dT.
 * grad_depth is [H][W] (dense), overwritten.
 */
int bno_normals_vjp_f64(const double *depth, int H, int W, int64_t stride,
                        double fx, double fy, double cx, double cy, int alpha,
                        const uint8_t *codes, const double *grad_normals, double *grad_depth)
{
    if (check_common(H, W, stride, fx, fy, alpha, ORC_NONE, 1.0) != ORC_OK)
        return ORC_EARG;
    for (int64_t i = 0; i < (int64_t)H * W; ++i)
        grad_depth[i] = 0.0;
    const double a = (double)alpha;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            if (codes[i] != ORC_VALID)
                continue;
            if (x - alpha < 0 || x + alpha > W - 1 || y - alpha < 0 || y + alpha > H - 1)
                return ORC_EARG;
            const double *row = depth + (int64_t)y * stride;
            double d2 = row[x + alpha];
            double d4 = row[x - alpha];
            double d3 = depth[(int64_t)(y + alpha) * stride + x];
            double d5 = depth[(int64_t)(y - alpha) * stride + x];
            double u1 = ((double)x - cx) / fx;
            double v1 = ((double)y - cy) / fy;
            double n[3];
            normal_closed_form(d2, d3, d4, d5, u1, v1, fx, fy, a, n);
            double len = norm3(n);
            double nh[3] = {n[0] / len, n[1] / len, n[2] / len};
            const double *g = grad_normals + 3 * i;
            double ng = nh[0] * g[0] + nh[1] * g[1] + nh[2] * g[2];
            double gn[3];
            for (int k = 0; k < 3; ++k)
                gn[k] = -(g[k] - ng * nh[k]) / len;
            double P = d2 - d4, S = d2 + d4, Q = d3 - d5, T = d3 + d5;
            double ex = gn[0] - u1 * gn[2];
            double ey = gn[1] - v1 * gn[2];
            double k2 = a * a / (4.0 * fx * fy);
            double dP = ex * (-a * T / (4.0 * fy));
            double dT = ex * (-a * P / (4.0 * fy)) + gn[2] * k2 * S;
            double dQ = ey * (-a * S / (4.0 * fx));
            double dS = ey * (-a * Q / (4.0 * fx)) + gn[2] * k2 * T;
            grad_depth[i + alpha] += dP + dS;
            grad_depth[i - alpha] += -dP + dS;
            grad_depth[i + (int64_t)alpha * W] += dQ + dT;
            grad_depth[i - (int64_t)alpha * W] += -dQ + dT;
        }
    }
    return ORC_OK;
}

/* The binary32 threshold of ABS mode, exposed for the closed-form tests. */
float bno_abs_threshold_f32(float fx, float fy, float tau, int alpha)
{
    return abs_threshold_f32(fx, fy, tau, alpha);
}

int bno_version(void)
{
    return 1;
}
