// Evaluation tools of Section 4 on the GPU: the spherical angle images of a
// normal map (Eqs. 14-15), their mean squared error between two maps over
// the pixels valid in both, and the local plane-fit normals that the paper
// uses as ground truth on real depth maps (25 neighbours: a 5x5 window).
//
// These are off the estimator's hot path and run in FP64 (on this GPU's
// vector units as fast as unpacked binary32), storing binary32 results.
#include <cmath>

#include "bn_internal.h"
#include "bnormals.h"

namespace bn {

namespace {

constexpr int kMseBlocks = BN_MSE_WORKSPACE_DOUBLES / 3;  // partial sums per launch
constexpr double kTwoPi = 6.283185307179586476925286766559;

struct Angles {
    double theta, phi;
};

// I_phi = atan2(ny, nx) taken into [0, 2 pi); I_theta = atan2(|(nx, ny)|, nz).
__device__ __forceinline__ Angles angles_of(float x, float y, float z) {
    const double nx = x, ny = y, nz = z;
    double phi = atan2(ny, nx);
    if (phi < 0.0) phi += kTwoPi;
    Angles a;
    a.phi = phi;
    a.theta = atan2(sqrt(nx * nx + ny * ny), nz);
    return a;
}

__global__ __launch_bounds__(256) void k_angles(const float *__restrict__ normals, uint32_t npix,
                                                float *__restrict__ theta,
                                                float *__restrict__ phi) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= npix) return;
    const float *n = normals + 3 * (int64_t)i;
    const Angles a = angles_of(n[0], n[1], n[2]);
    theta[i] = (float)a.theta;
    phi[i] = (float)a.phi;
}

// Block sum of three doubles, deterministic for a fixed block size: lane
// shuffles, then the 4 wavefront totals in order.  Result in thread 0.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c) {
    __shared__ double s[4][3];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) {
        s[w][0] = a;
        s[w][1] = b;
        s[w][2] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = s[0][0] + s[1][0] + s[2][0] + s[3][0];
        b = s[0][1] + s[1][1] + s[2][1] + s[3][1];
        c = s[0][2] + s[1][2] + s[2][2] + s[3][2];
    }
}

// Partial sums of (dtheta^2, dphi^2, count) over a grid-stride share of the
// pixels, one triple per workgroup.  A null mask counts as all VALID.
__global__ __launch_bounds__(256) void k_mse_partial(const float *__restrict__ na,
                                                     const uint8_t *__restrict__ ma,
                                                     const float *__restrict__ nb,
                                                     const uint8_t *__restrict__ mb,
                                                     uint32_t npix, double *__restrict__ part) {
    double st = 0.0, sp = 0.0, k = 0.0;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < npix; i += gridDim.x * 256u) {
        const bool va = !ma || ma[i] == BN_VALID;
        const bool vb = !mb || mb[i] == BN_VALID;
        if (!(va && vb)) continue;
        const float *a = na + 3 * (int64_t)i;
        const float *b = nb + 3 * (int64_t)i;
        const Angles x = angles_of(a[0], a[1], a[2]);
        const Angles y = angles_of(b[0], b[1], b[2]);
        const double dt = x.theta - y.theta;
        const double dp = x.phi - y.phi;
        st += dt * dt;
        sp += dp * dp;
        k += 1.0;
    }
    block_sum3(st, sp, k);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = st;
        part[3 * blockIdx.x + 1] = sp;
        part[3 * blockIdx.x + 2] = k;
    }
}

// One workgroup: the partials in a fixed order, then the means.
__global__ __launch_bounds__(256) void k_mse_final(const double *__restrict__ part,
                                                   uint32_t nparts, double *__restrict__ out) {
    double st = 0.0, sp = 0.0, k = 0.0;
    for (uint32_t j = threadIdx.x; j < nparts; j += 256u) {
        st += part[3 * j + 0];
        sp += part[3 * j + 1];
        k += part[3 * j + 2];
    }
    block_sum3(st, sp, k);
    if (threadIdx.x == 0) {
        out[0] = k > 0.0 ? st / k : 0.0;
        out[1] = k > 0.0 ? sp / k : 0.0;
        out[2] = k;
    }
}

// Smallest-eigenvalue eigenvector of the symmetric 3x3 matrix
// [a0 a1 a2; a1 a3 a4; a2 a4 a5]: eigenvalue from the trigonometric
// solution of the characteristic cubic, eigenvector as the longest cross
// product of two rows of (A - lambda I).  False when it is not defined.
__device__ __forceinline__ bool smallest_eigvec(const double a[6], double n[3]) {
    const double q = (a[0] + a[3] + a[5]) / 3.0;
    const double b0 = a[0] - q, b3 = a[3] - q, b5 = a[5] - q;
    const double p2 = (b0 * b0 + b3 * b3 + b5 * b5 + 2.0 * (a[1] * a[1] + a[2] * a[2] + a[4] * a[4])) / 6.0;
    if (!(p2 > 0.0)) return false;
    const double p = sqrt(p2);
    const double det = b0 * (b3 * b5 - a[4] * a[4]) - a[1] * (a[1] * b5 - a[4] * a[2]) +
                       a[2] * (a[1] * a[4] - b3 * a[2]);
    double r = det / (2.0 * p2 * p);
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double lam = q + 2.0 * p * cos(acos(r) / 3.0 + kTwoPi / 3.0);
    const double r0[3] = {a[0] - lam, a[1], a[2]};
    const double r1[3] = {a[1], a[3] - lam, a[4]};
    const double r2[3] = {a[2], a[4], a[5] - lam};
    double c[3][3];
    c[0][0] = r0[1] * r1[2] - r0[2] * r1[1];
    c[0][1] = r0[2] * r1[0] - r0[0] * r1[2];
    c[0][2] = r0[0] * r1[1] - r0[1] * r1[0];
    c[1][0] = r0[1] * r2[2] - r0[2] * r2[1];
    c[1][1] = r0[2] * r2[0] - r0[0] * r2[2];
    c[1][2] = r0[0] * r2[1] - r0[1] * r2[0];
    c[2][0] = r1[1] * r2[2] - r1[2] * r2[1];
    c[2][1] = r1[2] * r2[0] - r1[0] * r2[2];
    c[2][2] = r1[0] * r2[1] - r1[1] * r2[0];
    int best = 0;
    double bn = -1.0;
    for (int k = 0; k < 3; ++k) {
        const double l = c[k][0] * c[k][0] + c[k][1] * c[k][1] + c[k][2] * c[k][2];
        if (l > bn) {
            bn = l;
            best = k;
        }
    }
    if (!(bn > 0.0) || !isfinite(bn)) return false;
    const double inv = 1.0 / sqrt(bn);
    n[0] = c[best][0] * inv;
    n[1] = c[best][1] * inv;
    n[2] = c[best][2] * inv;
    return true;
}

// Plane fit over the (2R+1)^2 window of each pixel: points back-projected
// relative to the window's centre pixel (Eqs. 8-9), scatter matrix about
// their mean, smallest-eigenvalue eigenvector turned towards the camera.
template <int R>
__global__ __launch_bounds__(256) void k_plane_fit(const float *__restrict__ depth, int32_t H,
                                                   int32_t W, int64_t stride, float fx, float fy,
                                                   float cx, float cy,
                                                   float *__restrict__ normals,
                                                   uint8_t *__restrict__ mask) {
    const uint32_t gx = ((uint32_t)W + 63u) / 64u;  // workgroups per band of 4 rows
    const int32_t x = (int32_t)((blockIdx.x % gx) * 64u + (threadIdx.x & 63u));
    const int32_t y = (int32_t)((blockIdx.x / gx) * 4u + (threadIdx.x >> 6));
    if (x >= W || y >= H) return;
    const int64_t i = (int64_t)y * W + x;
    float *out = normals + 3 * i;
    bool ok = x >= R && y >= R && x + R < W && y + R < H;
    double n[3] = {0.0, 0.0, 0.0};
    if (ok) {
        const double ifx = 1.0 / (double)fx, ify = 1.0 / (double)fy;
        const double u0 = ((double)x - (double)cx) * ifx;
        const double v0 = ((double)y - (double)cy) * ify;
        const double d0 = depth[(int64_t)y * stride + x];
        const double X0[3] = {u0 * d0, v0 * d0, d0};
        double s[3] = {0.0, 0.0, 0.0}, m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int dy = -R; dy <= R; ++dy) {
            const float *row = depth + (int64_t)(y + dy) * stride;
            const double v = ((double)(y + dy) - (double)cy) * ify;
            for (int dx = -R; dx <= R; ++dx) {
                const float df = row[x + dx];
                ok = ok && (tap_ok(df) != 0u);
                const double d = df;
                const double u = ((double)(x + dx) - (double)cx) * ifx;
                const double p0 = u * d - X0[0], p1 = v * d - X0[1], p2 = d - X0[2];
                s[0] += p0;
                s[1] += p1;
                s[2] += p2;
                m[0] += p0 * p0;
                m[1] += p0 * p1;
                m[2] += p0 * p2;
                m[3] += p1 * p1;
                m[4] += p1 * p2;
                m[5] += p2 * p2;
            }
        }
        const double N = (double)((2 * R + 1) * (2 * R + 1));
        const double c[3] = {s[0] / N, s[1] / N, s[2] / N};
        const double a[6] = {m[0] - N * c[0] * c[0], m[1] - N * c[0] * c[1],
                             m[2] - N * c[0] * c[2], m[3] - N * c[1] * c[1],
                             m[4] - N * c[1] * c[2], m[5] - N * c[2] * c[2]};
        ok = ok && smallest_eigvec(a, n);
        if (ok && n[0] * u0 + n[1] * v0 + n[2] > 0.0) {
            n[0] = -n[0];
            n[1] = -n[1];
            n[2] = -n[2];
        }
    }
    out[0] = ok ? (float)n[0] : 0.0f;
    out[1] = ok ? (float)n[1] : 0.0f;
    out[2] = ok ? (float)n[2] : 0.0f;
    mask[i] = ok ? (uint8_t)BN_VALID : (uint8_t)BN_INVALID;
}

typedef void (*FitFn)(const float *, int32_t, int32_t, int64_t, float, float, float, float,
                      float *, uint8_t *);

FitFn fit_kernel(int r) {
    switch (r) {
        case 1: return k_plane_fit<1>;
        case 2: return k_plane_fit<2>;
        case 3: return k_plane_fit<3>;
    }
    return nullptr;
}

}  // namespace

}  // namespace bn

using namespace bn;

extern "C" {

int bn_normal_angles(const float *normals, int32_t height, int32_t width, float *theta,
                     float *phi, void *stream) {
    if (height < 0 || width < 0) return BN_ERR_INVALID_ARG;
    if ((int64_t)height * width > BN_MAX_PIXELS) return BN_ERR_UNSUPPORTED;
    if (height == 0 || width == 0) return BN_OK;
    if (!normals || !theta || !phi) return BN_ERR_INVALID_ARG;
    const uint32_t npix = (uint32_t)height * (uint32_t)width;
    hipLaunchKernelGGL(k_angles, dim3((npix + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       normals, npix, theta, phi);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

int bn_angle_mse(const float *normals_a, const uint8_t *mask_a, const float *normals_b,
                 const uint8_t *mask_b, int32_t height, int32_t width, double *workspace,
                 double *result, void *stream) {
    if (height < 0 || width < 0) return BN_ERR_INVALID_ARG;
    if ((int64_t)height * width > BN_MAX_PIXELS) return BN_ERR_UNSUPPORTED;
    if (!workspace || !result) return BN_ERR_INVALID_ARG;
    const uint32_t npix = (uint32_t)height * (uint32_t)width;
    if (npix > 0 && (!normals_a || !normals_b)) return BN_ERR_INVALID_ARG;
    uint32_t blocks = (npix + 255) / 256;
    if (blocks > (uint32_t)kMseBlocks) blocks = kMseBlocks;
    if (blocks == 0) blocks = 1;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mse_partial, dim3(blocks), dim3(256), 0, s, normals_a, mask_a,
                       normals_b, mask_b, npix, workspace);
    if (hipGetLastError() != hipSuccess) return BN_ERR_DEVICE;
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, s, (const double *)workspace, blocks,
                       result);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

int bn_plane_fit_normals(const float *depth, int32_t height, int32_t width, int64_t depth_stride,
                         float fx, float fy, float cx, float cy, int32_t radius, float *normals,
                         uint8_t *mask, void *stream) {
    if (radius < 1) return BN_ERR_INVALID_ARG;
    if (radius > BN_MAX_FIT_RADIUS) return BN_ERR_UNSUPPORTED;
    int rc = check_frame_args(depth, height, width, depth_stride, fx, fy, cx, cy, normals, mask);
    if (rc != BN_OK) return rc;
    if (height == 0 || width == 0) return BN_OK;
    FitFn fn = fit_kernel(radius);
    const uint64_t blocks =
        (uint64_t)(((uint32_t)width + 63u) / 64u) * (uint64_t)(((uint32_t)height + 3u) / 4u);
    hipLaunchKernelGGL(fn, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, depth,
                       height, width,
                       depth_stride, fx, fy, cx, cy, normals, mask);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

}  // extern "C"
