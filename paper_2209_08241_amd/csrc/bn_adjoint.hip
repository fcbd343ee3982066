// Adjoint of the normal map with respect to the depth (vector-Jacobian
// product), codes held fixed: the mask is piecewise constant in the depth,
// so its derivative vanishes almost everywhere.
//
// For a VALID pixel the output is o/|o| with o = (mx, my, -mz) the scaled
// vector of Eqs. 10-12 (see bn_device.h), a smooth function of the taps
// d2..d5 through P = d2-d4, S = d2+d4, Q = d3-d5, T = d3+d5.  With
// g_o = (g - (n.g) n)/|o| the gradient with respect to o,
//   dP = g_ox fx T - g_oz xc T          dQ = g_oy fy S - g_oz yc S
//   dS = g_oy fy Q - g_oz (yc Q + a T)  dT = g_ox fx P - g_oz (xc P + a S)
// and the taps receive  d2: dP + dS,  d4: -dP + dS,  d3: dQ + dT,
// d5: -dQ + dT.
//
// Gather form: a workgroup owns a TX x TY tile of output depths (64 x 16, or
// 32 x 8 on frames under 2^20 pixels, which would otherwise leave most
// compute units idle).  It stages the depth of the tile plus a 2-alpha ring
// in LDS, evaluates every pixel of
// the tile plus an alpha ring once (its code and its four tap gradients, in
// LDS), and each output depth then sums the four contributions that land on
// it, in a fixed order.  No atomics: the result is deterministic.
#include "bn_device.h"
#include "bn_internal.h"

#pragma clang fp contract(off)

namespace bn {

// One TX x TY tile of the gradient of one frame.
template <int A, int TX, int TY>
__device__ __forceinline__ void vjp_tile(const FrameArgs &f, const float *__restrict__ gn,
                                         float *__restrict__ gd, uint32_t tile,
                                         uint32_t tiles_x) {
    constexpr int kAdjTX = TX, kAdjTY = TY;
    constexpr int DX = kAdjTX + 4 * A, DY = kAdjTY + 4 * A;  // depth tile
    constexpr int GX = kAdjTX + 2 * A, GY = kAdjTY + 2 * A;  // evaluated pixels
    __shared__ float s_d[DY * DX];
    __shared__ float s_g[4][GY * GX];  // tap gradients: to d2, d3, d4, d5
    constexpr int NE = (GY * GX + kBlock - 1) / kBlock;  // evaluated pixels per thread
    const int x0 = (int)(tile % tiles_x) * kAdjTX;
    const int y0 = (int)(tile / tiles_x) * kAdjTY;
    // The cotangents of this thread's pixels are loaded first, all at once:
    // a load behind each pixel's code would expose one memory latency per
    // pixel.  (Masked pixels' cotangents are read and then ignored.)
    float cg[NE][3];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        const int k = (int)threadIdx.x + i * kBlock;
        const int X = x0 - A + k % GX;
        const int Y = y0 - A + k / GX;
        cg[i][0] = cg[i][1] = cg[i][2] = 0.f;
        if (k < GY * GX && X >= 0 && X < f.W && Y >= 0 && Y < f.H) {
            const float *g = gn + 3 * ((int64_t)Y * f.W + X);
            cg[i][0] = g[0];
            cg[i][1] = g[1];
            cg[i][2] = g[2];
        }
    }
    for (int k = threadIdx.x; k < DY * DX; k += kBlock) {
        const int X = x0 - 2 * A + k % DX;
        const int Y = y0 - 2 * A + k / DX;
        float v = 0.f;
        if (X >= 0 && X < f.W && Y >= 0 && Y < f.H) v = f.depth[(int64_t)Y * f.stride + X];
        s_d[k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        const int k = (int)threadIdx.x + i * kBlock;
        if (k >= GY * GX) break;
        const int c = k % GX, r = k / GX;
        const int X = x0 - A + c;
        const int Y = y0 - A + r;
        float g2 = 0.f, g3 = 0.f, g4 = 0.f, g5 = 0.f;
        if (X >= 0 && X < f.W && Y >= 0 && Y < f.H) {
            const int dc = c + A, dr = r + A;  // position in the depth tile
            const float d1 = s_d[dr * DX + dc];
            const float d2 = s_d[dr * DX + dc + A];
            const float d4 = s_d[dr * DX + dc - A];
            const float d3 = s_d[(dr + A) * DX + dc];
            const float d5 = s_d[(dr - A) * DX + dc];
            const bool inside = (X >= A) & (X + A < f.W) & (Y >= A) & (Y + A < f.H);
            const float xc = (float)X - f.cx;
            const float yc = (float)Y - f.cy;
            const PixelTerms t = eval_terms(inside, d1, d2, d3, d4, d5, xc, yc, f);
            if (t.code == BN_VALID) {
                const float inv = __builtin_amdgcn_rsqf(t.q);
                const float nx = t.mx * inv, ny = t.my * inv, nz = -(t.mz * inv);
                const float gx = cg[i][0], gy = cg[i][1], gz = cg[i][2];
                const float dot = (nx * gx + ny * gy) + nz * gz;
                const float ox = (gx - dot * nx) * inv;
                const float oy = (gy - dot * ny) * inv;
                const float oz = (gz - dot * nz) * inv;
                const float dP = ox * f.fx * t.T - oz * xc * t.T;
                const float dQ = oy * f.fy * t.S - oz * yc * t.S;
                const float dS = oy * f.fy * t.Q - oz * (yc * t.Q + f.af * t.T);
                const float dT = ox * f.fx * t.P - oz * (xc * t.P + f.af * t.S);
                g2 = dP + dS;
                g4 = dS - dP;
                g3 = dQ + dT;
                g5 = dT - dQ;
            }
        }
        s_g[0][k] = g2;
        s_g[1][k] = g3;
        s_g[2][k] = g4;
        s_g[3][k] = g5;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kAdjTX * kAdjTY; k += kBlock) {
        const int c = k % kAdjTX, r = k / kAdjTX;
        const int X = x0 + c, Y = y0 + r;
        if (X >= f.W || Y >= f.H) continue;
        const int gc = c + A, gr = r + A;  // this depth's own position among evaluated pixels
        // it is tap 2 of (X-A, Y), tap 4 of (X+A, Y), tap 3 of (X, Y-A), tap 5 of (X, Y+A)
        const float v = ((s_g[0][gr * GX + gc - A] + s_g[2][gr * GX + gc + A]) +
                         s_g[1][(gr - A) * GX + gc]) +
                        s_g[3][(gr + A) * GX + gc];
        gd[(int64_t)Y * f.W + X] = v;
    }
}

template <int A, int TX, int TY>
__global__ __launch_bounds__(kBlock) void k_vjp(FrameArgs f, const float *__restrict__ gn,
                                                float *__restrict__ gd, uint32_t tiles_x) {
    vjp_tile<A, TX, TY>(f, gn, gd, xcd_tile(blockIdx.x, gridDim.x), tiles_x);
}

// A stack: workgroup b takes tile b % T of frame b / T.
template <int A, int TX, int TY>
__global__ __launch_bounds__(kBlock) void k_vjp_stack(const StackArgs s) {
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t k = b / s.tiles_per_frame;
    const uint32_t tile = b - k * s.tiles_per_frame;
    const int64_t npix = (int64_t)s.f.npix;
    vjp_tile<A, TX, TY>(stack_frame(s, k), s.gn + (int64_t)k * npix * 3, s.gd + (int64_t)k * npix,
                        tile, s.tiles_x);
}

typedef void (*VjpFn)(FrameArgs, const float *, float *, uint32_t);
typedef void (*VjpStackFn)(const StackArgs);

template <int TX, int TY>
static VjpFn vjp_kernel_t(int a) {
    switch (a) {
        case 1: return k_vjp<1, TX, TY>;
        case 2: return k_vjp<2, TX, TY>;
        case 3: return k_vjp<3, TX, TY>;
        case 4: return k_vjp<4, TX, TY>;
        case 5: return k_vjp<5, TX, TY>;
        case 6: return k_vjp<6, TX, TY>;
        case 7: return k_vjp<7, TX, TY>;
        case 8: return k_vjp<8, TX, TY>;
    }
    return nullptr;
}

template <int TX, int TY>
static VjpStackFn vjp_stack_kernel_t(int a) {
    switch (a) {
        case 1: return k_vjp_stack<1, TX, TY>;
        case 2: return k_vjp_stack<2, TX, TY>;
        case 3: return k_vjp_stack<3, TX, TY>;
        case 4: return k_vjp_stack<4, TX, TY>;
        case 5: return k_vjp_stack<5, TX, TY>;
        case 6: return k_vjp_stack<6, TX, TY>;
        case 7: return k_vjp_stack<7, TX, TY>;
        case 8: return k_vjp_stack<8, TX, TY>;
    }
    return nullptr;
}

}  // namespace bn

using namespace bn;

extern "C" int bn_normals_vjp(const float *depth, int32_t height, int32_t width,
                              int64_t depth_stride, float fx, float fy, float cx, float cy,
                              const bn_params *params, const float *grad_normals,
                              float *grad_depth, void *stream) {
    int rc = check_params_args(params);
    if (rc != BN_OK) return rc;
    if (params->variant != VAR_AUTO || params->method != BN_METHOD_FOUR_PAIR)
        return BN_ERR_UNSUPPORTED;
    // the frame checks of the forward entry point; the gradients stand in
    // for its outputs
    rc = check_frame_args(depth, height, width, depth_stride, fx, fy, cx, cy,
                          grad_normals ? grad_normals : nullptr,
                          reinterpret_cast<const uint8_t *>(grad_depth));
    if (rc != BN_OK) return rc;
    if (height == 0 || width == 0) return BN_OK;
    const bool small = (int64_t)height * width < (1 << 20);
    const uint32_t TX = small ? 32u : 64u, TY = small ? 8u : 16u;
    VjpFn fn = small ? vjp_kernel_t<32, 8>(params->alpha) : vjp_kernel_t<64, 16>(params->alpha);
    if (!fn) return BN_ERR_UNSUPPORTED;
    FrameArgs f;
    fill_frame_args(f, depth, height, width, depth_stride, fx, fy, cx, cy, params, nullptr,
                    nullptr, nullptr, 1);
    const uint32_t tx = ((uint32_t)width + TX - 1) / TX;
    const uint32_t ty = ((uint32_t)height + TY - 1) / TY;
    hipLaunchKernelGGL(fn, dim3(tx * ty), dim3(kBlock), 0, (hipStream_t)stream, f, grad_normals,
                       grad_depth, tx);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

extern "C" int bn_normals_vjp_stack(const float *depth, int32_t n, int32_t height, int32_t width,
                                    int64_t depth_stride, int64_t depth_frame_stride,
                                    const bn_intrinsics *intrinsics, const bn_params *params,
                                    const float *grad_normals, float *grad_depth, void *stream) {
    int rc = check_params_args(params);
    if (rc != BN_OK) return rc;
    if (params->variant != VAR_AUTO || params->method != BN_METHOD_FOUR_PAIR)
        return BN_ERR_UNSUPPORTED;
    StackArgs s;
    // the gradients stand in for the forward's outputs in the checks
    rc = stack_args(s, depth, n, height, width, depth_stride, depth_frame_stride, intrinsics,
                    params, const_cast<float *>(grad_normals),
                    reinterpret_cast<uint8_t *>(grad_depth), nullptr, 1);
    if (rc == BN_OK && s.n > 0 && (uintptr_t)grad_depth % 4) rc = BN_ERR_INVALID_ARG;
    if (rc != BN_OK || s.n == 0) return rc;
    s.f.normals = nullptr;  // the gradients travel in gn / gd
    s.f.mask = nullptr;
    // each frame is small when the stack as a whole would not fill the chip
    // with the larger tiles
    const bool small = (int64_t)height * width * n < (1 << 20);
    const uint32_t TX = small ? 32u : 64u, TY = small ? 8u : 16u;
    VjpStackFn fn = small ? vjp_stack_kernel_t<32, 8>(params->alpha)
                          : vjp_stack_kernel_t<64, 16>(params->alpha);
    if (!fn) return BN_ERR_UNSUPPORTED;
    s.gn = grad_normals;
    s.gd = grad_depth;
    s.tiles_x = ((uint32_t)width + TX - 1) / TX;
    s.tiles_per_frame = s.tiles_x * (((uint32_t)height + TY - 1) / TY);
    const uint64_t grid = (uint64_t)s.tiles_per_frame * s.n;
    hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kBlock), 0, (hipStream_t)stream, s);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}
