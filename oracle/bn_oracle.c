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
 * rounds exactly once per written operation, in the written order; the
 * fused multiply-adds that methods 1 and 2 name are written as C99 fmaf).
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
 *  2. Validity (the paper is silent; the reading taken here): the pixel is
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

/* ====================================================================== */
/* Variants of the estimator                                               */
/* ====================================================================== */
/*
 * Method 0, FOUR_PAIR: everything above (Section 3: the four-pair average
 *   of Eq. 7 in its closed form, Eqs. 10-12, with the whole pixel removed by
 *   the test of Section 3.2).
 *
 * Method 1, PAIR_REMOVAL: the four perpendicular-pair normals that Eq. 7
 *   averages, n23 = s12 x s13, n34 = s13 x s14, n45 = s14 x s15 and
 *   n52 = s15 x s12, each go through the test of Section 3.2 on their own
 *   (r = |n_jk|, or rho = r / (n_jk . ray)); the pixel's normal is the
 *   average of the pairs that pass, and the pixel is BOUNDARY when none
 *   passes.  Only the pairs whose tangents cross a depth discontinuity are
 *   dropped, instead of the whole pixel.  When all four pass, the average is
 *   Eq. 7's n exactly.  Each pair has n_jk . ray = alpha^2 d_j d_k/(fx fy) > 0
 *   (X1 is parallel to the ray, so the triple product keeps only the
 *   alpha-offset parts), so each pair's rho is well defined.
 *
 * Method 2, MULTISCALE: the authors' earlier single-pair estimator
 *   (Section 2): the normal of the pair (2, 3), Eqs. 1-3, at pixel offsets
 *   alpha_i = i * alpha for i = 1..K, averaged over i as in Eqs. 4-6; the
 *   test of Section 3.2 applied to the average.  Only the taps
 *   (x + alpha_i, y) and (x, y + alpha_i) are read, so the invalid border is
 *   K*alpha wide on the right and bottom edges only.
 *
 * Binary32 decisions.  Each pair normal is decided on its scaled vector
 *   m_jk = -(fx fy / alpha) n_jk = (fx A, fy B, -(xc A + yc B + alpha C))
 *   with, for the horizontal tap h (2 or 4, direction sh = +1 or -1 along
 *   u) and the vertical tap v (3 or 5, sv = +1 or -1 along v):
 *     A = sh (d_h - d1) d_v,   B = sv d_h (d_v - d1),   C = d_h d_v,
 *   which for the pair (2, 3) is Eqs. 1-3 multiplied by -fx fy / alpha, and
 *   for the others follows from the same expansion of the cross product.
 *   m_jk . ray = -alpha C, so REL compares |m_jk|^2 with tau^2 (alpha C)^2,
 *   and ABS compares it with (fx fy tau / alpha)^2.  The four m_jk sum to
 *   the m of method 0.  Methods 1 and 2 take the third component, the
 *   weighted sums and each squared length with fused multiply-adds, every
 *   step rounded once (fp32_pair_fma below); method 0 keeps the separately
 *   rounded products and sums of its pinned sequence.
 *   MULTISCALE sums alpha_i m(alpha_i), which is -K fx fy times the average
 *   of Eqs. 4-6; REL compares with tau^2 (sum alpha_i^2 C_i)^2 and ABS with
 *   (K fx fy tau)^2.
 */

#define ORC_FOUR_PAIR 0
#define ORC_PAIR_REMOVAL 1
#define ORC_MULTISCALE 2

/* Pixel offsets of taps 1..5 (index 0 unused). */
static const int TAP_DX[6] = {0, 0, 1, 0, -1, 0};
static const int TAP_DY[6] = {0, 0, 0, 1, 0, -1};

/* The pairs (j, k) of Eq. 7, first line, in its order. */
static const int PAIR_J[4] = {2, 3, 4, 5};
static const int PAIR_K[4] = {3, 4, 5, 2};

/* FP64 definition: n_jk = s1j x s1k for the four pairs of Eq. 7. */
static void pair_normals_definition(const double d[6], int x, int y, int alpha,
                                    double fx, double fy, double cx, double cy,
                                    double n[4][3])
{
    double X[6][3];
    for (int t = 1; t <= 5; ++t)
        backproject((double)(x + alpha * TAP_DX[t]), (double)(y + alpha * TAP_DY[t]), d[t],
                    fx, fy, cx, cy, X[t]);
    for (int p = 0; p < 4; ++p) {
        double sj[3], sk[3];
        sub3(X[PAIR_J[p]], X[1], sj);
        sub3(X[PAIR_K[p]], X[1], sk);
        cross3(sj, sk, n[p]);
    }
}

/* Eqs. 1-3: the pair (2, 3) normal at pixel offset a, closed form. */
static void single_pair_closed_form(double d1, double d2, double d3, double u1, double v1,
                                    double fx, double fy, double a, double n[3])
{
    n[0] = -a / fy * d3 * (d2 - d1);                                   /* Eq. 1 */
    n[1] = -a / fx * d2 * (d3 - d1);                                   /* Eq. 2 */
    n[2] = a / fx * v1 * d2 * (d3 - d1) + a / fy * u1 * d3 * (d2 - d1)
           + a * a / (fx * fy) * d2 * d3;                               /* Eq. 3 */
}

/* Binary32 scaled vector of one pair (methods 1 and 2), given its
 * w = alpha dh dv (each method rounds that product in its own order): the
 * products
 *   A = sh (dh - d1) dv,  B = sv dh (dv - d1),  mx = fx A,  my = fy B,
 * then mz = fma(xc, A, fma(yc, B, w)) (the negated third component) and
 * q = fma(mx, mx, fma(my, my, mz * mz)), each fma rounded once (C99 fmaf). */
static void fp32_pair_fma(float dh, float dv, float d1, int sh, int sv, float fx, float fy,
                          float xc, float yc, float w, float *mx, float *my, float *mz,
                          float *q)
{
    float eh = dh - d1;
    float ev = dv - d1;
    float A = eh * dv;
    float B = dh * ev;
    if (sh < 0) A = -A;
    if (sv < 0) B = -B;
    float x = fx * A;
    float y = fy * B;
    float z = fmaf(xc, A, fmaf(yc, B, w));
    *mx = x;
    *my = y;
    *mz = z;
    *q = fmaf(x, x, fmaf(y, y, z * z));
}

static int q_degenerate(float q)
{
    return !isfinite(q) || q < FLT_MIN;
}

/* ABS thresholds of methods 1 and 2 on the binary32 |m|^2 scale, computed in
 * double in this order and rounded once. */
static float pair_abs_threshold_f32(float fx, float fy, float tau, int alpha)
{
    double k = (double)fx;
    k = k * (double)fy;
    k = k * (double)tau;
    k = k / (double)alpha;
    k = k * k;
    return (float)k;
}

static float multiscale_abs_threshold_f32(float fx, float fy, float tau, int scales)
{
    double k = (double)scales;
    k = k * (double)fx;
    k = k * (double)fy;
    k = k * (double)tau;
    k = k * k;
    return (float)k;
}

/* Method 1 binary32 decision.  Pairs in Eq. 7's order: (h, v) = (2, 3),
 * (4, 3), (4, 5), (2, 5).  A pair whose |m|^2 is not a finite number >=
 * FLT_MIN makes the pixel INVALID; *keep gets bit p for each pair p that
 * passes the test (REL: q > (tau^2 w) w, each product rounded); the passing
 * pairs' scaled vectors are summed in pair order, and a sum whose |.|^2
 * (fused as for one pair) is degenerate is INVALID too. */
static int fp32_pairs_code(const float d[6], int x, int y, float fx, float fy, float cx,
                           float cy, int alpha, int mode, float tau, float kpair, int *keep)
{
    const int th[4] = {2, 4, 4, 2};
    const int tv[4] = {3, 3, 5, 5};
    const int sh[4] = {1, -1, -1, 1};
    const int sv[4] = {1, 1, -1, -1};
    float xc = (float)x - cx;
    float yc = (float)y - cy;
    float af = (float)alpha;
    float mx[4], my[4], mz[4], w[4], q[4];
    *keep = 0;
    for (int p = 0; p < 4; ++p) {
        /* w = (alpha dh) dv: alpha times the horizontal tap first */
        w[p] = (af * d[th[p]]) * d[tv[p]];
        fp32_pair_fma(d[th[p]], d[tv[p]], d[1], sh[p], sv[p], fx, fy, xc, yc, w[p],
                      &mx[p], &my[p], &mz[p], &q[p]);
        if (q_degenerate(q[p]))
            return ORC_INVALID;
    }
    int k = 0;
    for (int p = 0; p < 4; ++p) {
        int fire = 0;
        if (mode == ORC_REL) {
            float tt = tau * tau;
            float tw = tt * w[p];
            float h = tw * w[p];
            fire = q[p] > h;
        } else if (mode == ORC_ABS) {
            fire = q[p] > kpair;
        }
        if (!fire) k |= 1 << p;
    }
    *keep = k;
    if (!k)
        return ORC_BOUNDARY;
    /* All four pass: their average is Eq. 7's n, taken in its closed form
     * (Eqs. 10-12), in which d1 cancels exactly instead of through rounded
     * sums; its third component and squared length fused as for one pair. */
    if (k == 15) {
        float P = d[2] - d[4];
        float S = d[2] + d[4];
        float Qv = d[3] - d[5];
        float T = d[3] + d[5];
        float a = T * P;
        float b = S * Qv;
        float c = S * T;
        float cx_ = fx * a;
        float cy_ = fy * b;
        float cw = af * c;
        float cz = fmaf(xc, a, fmaf(yc, b, cw));
        float Qc = fmaf(cx_, cx_, fmaf(cy_, cy_, cz * cz));
        return q_degenerate(Qc) ? ORC_INVALID : ORC_VALID;
    }
    int first = 1;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    for (int p = 0; p < 4; ++p) {
        if (!(k & (1 << p)))
            continue;
        if (first) {
            sx = mx[p];
            sy = my[p];
            sz = mz[p];
            first = 0;
        } else {
            sx = sx + mx[p];
            sy = sy + my[p];
            sz = sz + mz[p];
        }
    }
    float Q = fmaf(sx, sx, fmaf(sy, sy, sz * sz));
    return q_degenerate(Q) ? ORC_INVALID : ORC_VALID;
}

/* Method 2 binary32 decision: scales i = 1..K at offset a = i*alpha, the
 * pair (2, 3) vector of each (fp32_pair_fma) weighted by a and summed in
 * scale order with fused multiply-adds; |M|^2 fused as for one pair. */
static int fp32_multiscale_code(float d1, const float *d2s, const float *d3s, int scales, int x,
                                int y, float fx, float fy, float cx, float cy, int alpha, int mode,
                                float tau, float kms)
{
    float xc = (float)x - cx;
    float yc = (float)y - cy;
    float Mx = 0.0f, My = 0.0f, Mz = 0.0f, Wt = 0.0f;
    for (int i = 1; i <= scales; ++i) {
        float a = (float)(i * alpha);
        float mx, my, mz, q;
        float w = a * (d2s[i - 1] * d3s[i - 1]);
        fp32_pair_fma(d2s[i - 1], d3s[i - 1], d1, 1, 1, fx, fy, xc, yc, w, &mx, &my, &mz, &q);
        if (i == 1) {
            Mx = a * mx;
            My = a * my;
            Mz = a * mz;
            Wt = a * w;
        } else {
            Mx = fmaf(a, mx, Mx);
            My = fmaf(a, my, My);
            Mz = fmaf(a, mz, Mz);
            Wt = fmaf(a, w, Wt);
        }
    }
    float q = fmaf(Mx, Mx, fmaf(My, My, Mz * Mz));
    if (q_degenerate(q))
        return ORC_INVALID;
    if (mode == ORC_NONE)
        return ORC_VALID;
    float h;
    if (mode == ORC_REL) {
        float tt = tau * tau;
        float ww = Wt * Wt;
        h = tt * ww;
    } else {
        h = kms;
    }
    return (q > h) ? ORC_BOUNDARY : ORC_VALID;
}

/* FP64 output of method 1 from the passing pairs (bits of keep): the
 * average n of the pair normals, out = -n/|n|, r = |n|, rho = r/(n . ray).
 * gap: relative max-norm gap between the sum of all four pair normals and
 * 4 x Eqs. 10-12. */
static void pairs_normal_f64(const double d[6], int x, int y, double fx, double fy, double cx,
                             double cy, int alpha, int keep, double out[3], double *r,
                             double *rho, double *gap)
{
    double np[4][3];
    pair_normals_definition(d, x, y, alpha, fx, fy, cx, cy, np);
    double u1 = ((double)x - cx) / fx;
    double v1 = ((double)y - cy) / fy;
    double n[3] = {0.0, 0.0, 0.0};
    int cnt = 0;
    for (int p = 0; p < 4; ++p) {
        if (!(keep & (1 << p)))
            continue;
        n[0] += np[p][0];
        n[1] += np[p][1];
        n[2] += np[p][2];
        ++cnt;
    }
    if (cnt) {
        n[0] /= cnt;
        n[1] /= cnt;
        n[2] /= cnt;
    }
    double len = norm3(n);
    out[0] = -n[0] / len;
    out[1] = -n[1] / len;
    out[2] = -n[2] / len;
    *r = len;
    *rho = len / (n[0] * u1 + n[1] * v1 + n[2]);
    if (gap) {
        double all[3] = {0.0, 0.0, 0.0}, cf[3];
        for (int p = 0; p < 4; ++p)
            for (int c = 0; c < 3; ++c)
                all[c] += np[p][c];
        normal_closed_form(d[2], d[3], d[4], d[5], u1, v1, fx, fy, (double)alpha, cf);
        double l = 4.0 * norm3(cf), e = 0.0;
        for (int c = 0; c < 3; ++c) {
            double dc = fabs(all[c] - 4.0 * cf[c]);
            if (dc > e) e = dc;
        }
        e = (l > 0.0) ? e / l : (e > 0.0 ? INFINITY : 0.0);
        if (e > *gap) *gap = e;
    }
}

/* FP64 output of method 2: Eqs. 4-6 (the average over scales of Eqs. 1-3).
 * gap: relative gap between Eqs. 1-3 and the definition s12 x s13 at each
 * scale. */
static void multiscale_normal_f64(double d1, const double *d2s, const double *d3s, int scales,
                                  int x, int y, double fx, double fy, double cx, double cy,
                                  int alpha, double out[3], double *r, double *rho, double *gap)
{
    double u1 = ((double)x - cx) / fx;
    double v1 = ((double)y - cy) / fy;
    double n[3] = {0.0, 0.0, 0.0};
    for (int i = 1; i <= scales; ++i) {
        double a = (double)(i * alpha), ni[3];
        single_pair_closed_form(d1, d2s[i - 1], d3s[i - 1], u1, v1, fx, fy, a, ni);
        n[0] += ni[0];
        n[1] += ni[1];
        n[2] += ni[2];
        if (gap) {
            double X1[3], X2[3], X3[3], s2[3], s3[3], nd[3];
            backproject((double)x, (double)y, d1, fx, fy, cx, cy, X1);
            backproject((double)(x + i * alpha), (double)y, d2s[i - 1], fx, fy, cx, cy, X2);
            backproject((double)x, (double)(y + i * alpha), d3s[i - 1], fx, fy, cx, cy, X3);
            sub3(X2, X1, s2);
            sub3(X3, X1, s3);
            cross3(s2, s3, nd);
            double l = norm3(ni), e = 0.0;
            for (int c = 0; c < 3; ++c) {
                double dc = fabs(nd[c] - ni[c]);
                if (dc > e) e = dc;
            }
            e = (l > 0.0) ? e / l : (e > 0.0 ? INFINITY : 0.0);
            if (e > *gap) *gap = e;
        }
    }
    n[0] /= scales;
    n[1] /= scales;
    n[2] /= scales;
    double len = norm3(n);
    out[0] = -n[0] / len;
    out[1] = -n[1] / len;
    out[2] = -n[2] / len;
    *r = len;
    *rho = len / (n[0] * u1 + n[1] * v1 + n[2]);
}

static int check_method(int method, int scales)
{
    if (method == ORC_FOUR_PAIR || method == ORC_PAIR_REMOVAL)
        return (scales == 0 || scales == 1) ? ORC_OK : ORC_EARG;
    if (method == ORC_MULTISCALE)
        return scales >= 1 ? ORC_OK : ORC_EARG;
    return ORC_EARG;
}

/*
 * Any method, binary32 depth in, FP64 normals out, rows [row_begin, row_end)
 * of the frame.  Arguments as bno_normals_f32_rows, plus:
 *   method     0 FOUR_PAIR, 1 PAIR_REMOVAL, 2 MULTISCALE
 *   scales     K for MULTISCALE (>= 1); 0 or 1 otherwise
 *   keep_out   [rows][W] (nullable): PAIR_REMOVAL's passing pairs, bit p for
 *              the p-th pair of Eq. 7 (n23, n34, n45, n52); 0 elsewhere
 *   def_gap    (nullable) largest relative gap between each method's closed
 *              form and its definition over the pixels it evaluates
 * r_out and rho_out hold r and rho of the output vector of a VALID pixel
 * (method 0: also of a BOUNDARY one), NaN otherwise.
 */
int bno_variant_f32_rows(int method, int scales, const float *depth, int H, int W,
                         int64_t stride, float fx, float fy, float cx, float cy, int alpha,
                         int mode, float tau, int row_begin, int row_end, double *normals,
                         uint8_t *mask, uint64_t *counts, double *r_out, double *rho_out,
                         uint8_t *keep_out, double *def_gap)
{
    if (check_method(method, scales) != ORC_OK)
        return ORC_EARG;
    if (check_common(H, W, stride, fx, fy, alpha, mode, tau) != ORC_OK)
        return ORC_EARG;
    if (row_begin < 0 || row_end > H || row_begin > row_end)
        return ORC_EARG;
    if ((H > 0 && W > 0) && (!depth || !normals || !mask))
        return ORC_EARG;
    if (keep_out)
        memset(keep_out, 0, (size_t)(row_end - row_begin) * (size_t)W);
    if (method == ORC_FOUR_PAIR)
        return bno_normals_f32_rows(depth, H, W, stride, fx, fy, cx, cy, alpha, mode, tau,
                                    row_begin, row_end, normals, mask, counts, r_out, rho_out,
                                    def_gap);
    const int K = (method == ORC_MULTISCALE) ? scales : 1;
    const int reach = K * alpha;
    float kabs = 0.0f;
    if (mode == ORC_ABS)
        kabs = (method == ORC_PAIR_REMOVAL) ? pair_abs_threshold_f32(fx, fy, tau, alpha)
                                            : multiscale_abs_threshold_f32(fx, fy, tau, K);
    uint64_t cnt[3] = {0, 0, 0};
    double gap = 0.0;
    float f2[64], f3[64];
    double g2[64], g3[64];
    if (K > 64)
        return ORC_EARG;
    for (int y = row_begin; y < row_end; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)(y - row_begin) * W + x;
            int code = ORC_INVALID, keep = 0;
            double nrm[3] = {0.0, 0.0, 0.0};
            double r = NAN, rho = NAN;
            const float *row = depth + (int64_t)y * stride;
            if (method == ORC_PAIR_REMOVAL) {
                int inside = (x - alpha >= 0) && (x + alpha <= W - 1) &&
                             (y - alpha >= 0) && (y + alpha <= H - 1);
                if (inside) {
                    float d[6];
                    int ok = 1;
                    for (int t = 1; t <= 5; ++t) {
                        d[t] = depth[(int64_t)(y + alpha * TAP_DY[t]) * stride +
                                     (x + alpha * TAP_DX[t])];
                        ok = ok && tap_ok_f32(d[t]);
                    }
                    if (ok) {
                        code = fp32_pairs_code(d, x, y, fx, fy, cx, cy, alpha, mode, tau,
                                               kabs, &keep);
                        if (code == ORC_VALID) {
                            double dd[6];
                            for (int t = 1; t <= 5; ++t) dd[t] = (double)d[t];
                            pairs_normal_f64(dd, x, y, fx, fy, cx, cy, alpha, keep, nrm, &r,
                                             &rho, def_gap ? &gap : NULL);
                        }
                    }
                }
            } else {
                int inside = (x + reach <= W - 1) && (y + reach <= H - 1);
                if (inside) {
                    float d1 = row[x];
                    int ok = tap_ok_f32(d1);
                    for (int s = 1; s <= K; ++s) {
                        f2[s - 1] = row[x + s * alpha];
                        f3[s - 1] = depth[(int64_t)(y + s * alpha) * stride + x];
                        ok = ok && tap_ok_f32(f2[s - 1]) && tap_ok_f32(f3[s - 1]);
                    }
                    if (ok) {
                        code = fp32_multiscale_code(d1, f2, f3, K, x, y, fx, fy, cx, cy, alpha,
                                                    mode, tau, kabs);
                        if (code == ORC_VALID) {
                            for (int s = 0; s < K; ++s) {
                                g2[s] = (double)f2[s];
                                g3[s] = (double)f3[s];
                            }
                            multiscale_normal_f64((double)d1, g2, g3, K, x, y, fx, fy, cx, cy,
                                                  alpha, nrm, &r, &rho, def_gap ? &gap : NULL);
                        }
                    }
                }
            }
            normals[3 * i + 0] = nrm[0];
            normals[3 * i + 1] = nrm[1];
            normals[3 * i + 2] = nrm[2];
            mask[i] = (uint8_t)code;
            if (keep_out) keep_out[i] = (uint8_t)keep;
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
    if (def_gap) *def_gap = gap;
    return ORC_OK;
}

/*
 * Any method, FP64 depth in, everything in FP64 (closed-form tests on exact
 * depth).  The tests of Section 3.2 are taken in FP64: a pair (method 1) or
 * the average (methods 0 and 2) fires when rho > tau (REL) or r > tau (ABS).
 * A pixel whose output vector has a length that is not finite and > 0 is
 * INVALID.
 */
int bno_variant_f64(int method, int scales, const double *depth, int H, int W, int64_t stride,
                    double fx, double fy, double cx, double cy, int alpha, int mode, double tau,
                    double *normals, uint8_t *mask, uint64_t *counts, double *r_out,
                    double *rho_out, uint8_t *keep_out, double *def_gap)
{
    if (check_method(method, scales) != ORC_OK)
        return ORC_EARG;
    if (check_common(H, W, stride, fx, fy, alpha, mode, tau) != ORC_OK)
        return ORC_EARG;
    if ((H > 0 && W > 0) && (!depth || !normals || !mask))
        return ORC_EARG;
    if (keep_out)
        memset(keep_out, 0, (size_t)H * (size_t)W);
    if (method == ORC_FOUR_PAIR)
        return bno_normals_f64(depth, H, W, stride, fx, fy, cx, cy, alpha, mode, tau, normals,
                               mask, counts, r_out, rho_out, def_gap);
    const int K = (method == ORC_MULTISCALE) ? scales : 1;
    if (K > 64)
        return ORC_EARG;
    const int reach = K * alpha;
    uint64_t cnt[3] = {0, 0, 0};
    double gap = 0.0;
    double g2[64], g3[64];
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int64_t i = (int64_t)y * W + x;
            int code = ORC_INVALID, keep = 0;
            double nrm[3] = {0.0, 0.0, 0.0};
            double r = NAN, rho = NAN;
            const double *row = depth + (int64_t)y * stride;
            double u1 = ((double)x - cx) / fx;
            double v1 = ((double)y - cy) / fy;
            if (method == ORC_PAIR_REMOVAL) {
                int inside = (x - alpha >= 0) && (x + alpha <= W - 1) &&
                             (y - alpha >= 0) && (y + alpha <= H - 1);
                double d[6];
                int ok = inside;
                for (int t = 1; ok && t <= 5; ++t) {
                    d[t] = depth[(int64_t)(y + alpha * TAP_DY[t]) * stride +
                                 (x + alpha * TAP_DX[t])];
                    ok = tap_ok_f64(d[t]);
                }
                if (ok) {
                    double np[4][3];
                    pair_normals_definition(d, x, y, alpha, fx, fy, cx, cy, np);
                    for (int p = 0; p < 4; ++p) {
                        double rp = norm3(np[p]);
                        double rhop = rp / (np[p][0] * u1 + np[p][1] * v1 + np[p][2]);
                        int fire = 0;
                        if (mode == ORC_ABS) fire = rp > tau;
                        else if (mode == ORC_REL) fire = rhop > tau;
                        if (!fire) keep |= 1 << p;
                    }
                    if (!keep) {
                        code = ORC_BOUNDARY;
                    } else {
                        pairs_normal_f64(d, x, y, fx, fy, cx, cy, alpha, keep, nrm, &r, &rho,
                                         def_gap ? &gap : NULL);
                        code = (isfinite(r) && r > 0.0) ? ORC_VALID : ORC_INVALID;
                    }
                }
            } else {
                int inside = (x + reach <= W - 1) && (y + reach <= H - 1);
                int ok = inside;
                double d1 = ok ? row[x] : 0.0;
                ok = ok && tap_ok_f64(d1);
                for (int s = 1; ok && s <= K; ++s) {
                    g2[s - 1] = row[x + s * alpha];
                    g3[s - 1] = depth[(int64_t)(y + s * alpha) * stride + x];
                    ok = tap_ok_f64(g2[s - 1]) && tap_ok_f64(g3[s - 1]);
                }
                if (ok) {
                    multiscale_normal_f64(d1, g2, g3, K, x, y, fx, fy, cx, cy, alpha, nrm, &r,
                                          &rho, def_gap ? &gap : NULL);
                    if (!isfinite(r) || !(r > 0.0)) {
                        code = ORC_INVALID;
                    } else {
                        int fire = 0;
                        if (mode == ORC_ABS) fire = r > tau;
                        else if (mode == ORC_REL) fire = rho > tau;
                        code = fire ? ORC_BOUNDARY : ORC_VALID;
                    }
                }
            }
            if (code != ORC_VALID) {
                nrm[0] = nrm[1] = nrm[2] = 0.0;
                if (code == ORC_INVALID) r = rho = NAN;
            }
            normals[3 * i + 0] = nrm[0];
            normals[3 * i + 1] = nrm[1];
            normals[3 * i + 2] = nrm[2];
            mask[i] = (uint8_t)code;
            if (keep_out) keep_out[i] = (uint8_t)keep;
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
    if (def_gap) *def_gap = gap;
    return ORC_OK;
}

/* Binary32 ABS thresholds of methods 1 and 2, for the closed-form tests. */
float bno_variant_abs_threshold_f32(int method, int scales, float fx, float fy, float tau,
                                    int alpha)
{
    if (method == ORC_PAIR_REMOVAL)
        return pair_abs_threshold_f32(fx, fy, tau, alpha);
    if (method == ORC_MULTISCALE)
        return multiscale_abs_threshold_f32(fx, fy, tau, scales);
    return abs_threshold_f32(fx, fy, tau, alpha);
}

/* The binary32 threshold of ABS mode, exposed for the closed-form tests. */
float bno_abs_threshold_f32(float fx, float fy, float tau, int alpha)
{
    return abs_threshold_f32(fx, fy, tau, alpha);
}

int bno_version(void)
{
    return 2;
}
