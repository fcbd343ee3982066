// Adjoint of the normal map with respect to the depth (vector-Jacobian
// product), codes held fixed: the mask is piecewise constant in the depth,
// so its derivative vanishes almost everywhere.
//
// For a VALID pixel the output is o/|o| with o = (mx, my, -mz) the scaled
// vector of Eqs. 10-12 (see bn_device.h), a smooth function of the taps
// d2..d5 through P = d2-d4, S = d2+d4, Q = d3-d5, T = d3+d5.  With
// g_o = (g - (n.g) n)/|o| the gradient with respect to o and
//   u = fx g_ox - xc g_oz,   v = fy g_oy - yc g_oz,   z = a g_oz,
// the partial derivatives are
//   dP = T u,   dQ = S v,   dS = Q v - T z,   dT = P u - S z
// and the taps receive  d2: dP + dS,  d4: -dP + dS,  d3: dQ + dT,
// d5: -dQ + dT.
//
// Gather form, no atomics (deterministic): the depth at (x, y) is tap 2 of
// (x-a, y), tap 4 of (x+a, y), tap 3 of (x, y-a) and tap 5 of (x, y+a), and
// its gradient is ((g2 + g4) + g3) + g5 of those four pixels, in that order
// in every kernel here, so all of them give the same bits.
//
// Vector kernels (rows of whole float4 groups, a <= 4): a workgroup owns a
// strip of 56 float4 groups (224 columns: the strip's gradient rows start on
// 128-byte lines, and so do its cotangent rows) and a band of NW RB rows,
// RB rows per wavefront, NW = 4 or 8 wavefronts.  Lane l evaluates group
// 56 s - 4 + l of each row (its
// codes and tap gradients, from float4 loads), so lanes 4..59 own the
// strip's outputs and lanes 3 and 60 are the halo; the horizontal taps and
// the tap-2 / tap-4 gradients move between neighbouring lanes by DPP.  Each
// wavefront rolls down its rows keeping the last 2a rows' gradients in
// registers; the a rows next to a neighbouring wavefront's rows are finished
// after one workgroup barrier, from the neighbour's gradients left in LDS,
// and the 2a rows above and below the band are evaluated once, shared out
// over the wavefronts.  Per output: 1 + 2a / (NW RB) row evaluations.
//
// Scalar kernels (any layout, any a): a workgroup owns a TX x TY tile of
// output depths (64 x 16, or 32 x 8 on frames under 2^20 pixels, which
// would otherwise leave most compute units idle).  It stages the depth of
// the tile plus a 2-alpha ring in LDS, evaluates every pixel of the tile
// plus an alpha ring once (its code and its four tap gradients, in LDS),
// and each output depth then sums the four contributions that land on it.
#include "bn_device.h"
#include "bn_internal.h"

#pragma clang fp contract(off)

namespace bn {

// Tap gradients of one pixel (meaningful when its code is VALID).  The
// gradient is not part of the pinned mask sequence (the code comes from
// eval_terms, unfused), so its products and sums are fused where a product
// feeds a sum; every kernel here calls this one function, so all of them
// still give the same bits.
struct TapGrads {
    float g2, g3, g4, g5;
};

__device__ __forceinline__ TapGrads tap_grads(const PixelTerms &t, float gx, float gy, float gz,
                                              float xc, float yc, const FrameArgs &f) {
    const float inv = __builtin_amdgcn_rsqf(t.q);
    const float nx = t.mx * inv, ny = t.my * inv, nz = -(t.mz * inv);
    const float dot = __builtin_fmaf(nz, gz, __builtin_fmaf(ny, gy, nx * gx));
    const float ox = __builtin_fmaf(-dot, nx, gx) * inv;
    const float oy = __builtin_fmaf(-dot, ny, gy) * inv;
    const float oz = __builtin_fmaf(-dot, nz, gz) * inv;
    const float u = __builtin_fmaf(f.fx, ox, -(xc * oz));
    const float v = __builtin_fmaf(f.fy, oy, -(yc * oz));
    const float z = f.af * oz;
    const float dP = t.T * u;
    const float dQ = t.S * v;
    const float dS = __builtin_fmaf(t.Q, v, -(t.T * z));
    const float dT = __builtin_fmaf(t.P, u, -(t.S * z));
    return TapGrads{dP + dS, dQ + dT, dS - dP, dT - dQ};
}

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
                const TapGrads d = tap_grads(t, cg[i][0], cg[i][1], cg[i][2], xc, yc, f);
                g2 = d.g2;
                g3 = d.g3;
                g4 = d.g4;
                g5 = d.g5;
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

// ---------------------------------------------------------------------------
// Vector kernels.
// ---------------------------------------------------------------------------
// Output float4 groups per strip: a multiple of 8, so that strips do not
// share 128-byte lines of the gradient (measured 1-2% faster than 62
// groups, although a 1920-wide row then takes 9 strips instead of 8).
constexpr int kVjpGroups = 56;
constexpr int kVjpLead = (64 - kVjpGroups) / 2;   // lanes left of the outputs

// One row of evaluated pixels: per lane, for its 4 pixels, the sum of the
// tap-2 gradient of the pixel a to the left and the tap-4 gradient of the
// pixel a to the right (h), and its own tap-3 and tap-5 gradients.
struct RowGrads {
    f4 h, g3, g5;
};

// The loads of one row: the depth of the lane's group in rows y, y-a and
// y+a, the halo lanes' outer group of row y, and the cotangents.
struct RowLoad {
    f4 c, up, dn, side, k0, k1, k2;
};

__device__ __forceinline__ bool vjp4_row_live(const FrameArgs &f, int y, int a) {
    return y >= a && y + a < f.H;
}

// Rows whose codes are all INVALID (the border rows and rows out of the
// frame) are skipped by the whole wavefront.  xl: the lane's column clamped
// into the frame.  Every load in a row is unconditional (a clamped lane
// loads some group of the row); the values a clamped load brings in only
// reach pixels that are not inside, whose codes are INVALID and whose
// gradients are therefore zero.
template <int A>
__device__ __forceinline__ void vjp4_load(const FrameArgs &f, const float *__restrict__ gn, int y,
                                          int x0, int xl, uint32_t lane, RowLoad &L) {
    if (!vjp4_row_live(f, y, A)) return;
    const float *rp = f.depth + (int64_t)y * f.stride;
    L.c = *reinterpret_cast<const f4 *>(rp + xl);
    L.up = *reinterpret_cast<const f4 *>(rp - (int64_t)A * f.stride + xl);
    L.dn = *reinterpret_cast<const f4 *>(rp + (int64_t)A * f.stride + xl);
    const f4 *gp = reinterpret_cast<const f4 *>(gn + 3 * (int64_t)y * f.W) + 3 * (xl >> 2);
    L.k0 = gp[0];
    L.k1 = gp[1];
    L.k2 = gp[2];
    if (lane == 0) L.side = *reinterpret_cast<const f4 *>(rp + max(x0 - 4, 0));
    if (lane == 63) L.side = *reinterpret_cast<const f4 *>(rp + min(x0 + 4, f.W - 4));
}

template <int A>
__device__ __forceinline__ RowGrads vjp4_eval(const FrameArgs &f, int y, int x0, uint32_t lane,
                                              const RowLoad &L) {
    RowGrads r;
    r.h = r.g3 = r.g5 = f4{0.f, 0.f, 0.f, 0.f};
    if (!vjp4_row_live(f, y, A)) return r;
    const bool gin = (x0 >= 0) & (x0 < f.W);
    const f4 c = L.c, up = L.up, dn = L.dn, k0 = L.k0, k1 = L.k1, k2 = L.k2;
    // Row window x0-4 .. x0+7 (the halo lanes loaded their outer float4).
    f4 lk = from_left(c), rk = from_right(c);
    if (lane == 0) lk = L.side;
    if (lane == 63) rk = L.side;
    const float row[12] = {lk.x, lk.y, lk.z, lk.w, c.x, c.y, c.z, c.w, rk.x, rk.y, rk.z, rk.w};
    const float upv[4] = {up.x, up.y, up.z, up.w};
    const float dnv[4] = {dn.x, dn.y, dn.z, dn.w};
    const float cg[12] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w, k2.x, k2.y, k2.z, k2.w};
    const float yc = (float)y - f.cy;
    float g2[4], g3[4], g4[4], g5[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int x = x0 + j;
        const bool inside = gin & (x >= A) & (x + A < f.W);
        const float xc = (float)x - f.cx;
        const PixelTerms t = eval_terms(inside, row[4 + j], row[4 + j + A], dnv[j],
                                        row[4 + j - A], upv[j], xc, yc, f);
        const bool valid = t.code == BN_VALID;
        const TapGrads d = tap_grads(t, cg[3 * j], cg[3 * j + 1], cg[3 * j + 2], xc, yc, f);
        g2[j] = valid ? d.g2 : 0.f;
        g3[j] = valid ? d.g3 : 0.f;
        g4[j] = valid ? d.g4 : 0.f;
        g5[j] = valid ? d.g5 : 0.f;
    }
    float h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float a = j - A >= 0 ? g2[j - A] : from_left(g2[j - A + 4]);
        const float b = j + A < 4 ? g4[j + A] : from_right(g4[j + A - 4]);
        h[j] = a + b;
    }
    r.h = f4{h[0], h[1], h[2], h[3]};
    r.g3 = f4{g3[0], g3[1], g3[2], g3[3]};
    r.g5 = f4{g5[0], g5[1], g5[2], g5[3]};
    return r;
}

template <int A>
__device__ __forceinline__ RowGrads vjp4_row(const FrameArgs &f, const float *__restrict__ gn,
                                             int y, int x0, int xl, uint32_t lane) {
    RowLoad L;
    vjp4_load<A>(f, gn, y, x0, xl, lane, L);
    return vjp4_eval<A>(f, y, x0, lane, L);
}

// Strip `strip`, band `band` of one frame (see the top of the file).
template <int A, int RB, int NW>
__device__ __forceinline__ void vjp4_band(const FrameArgs &f, const float *__restrict__ gn,
                                          float *__restrict__ gd, uint32_t strip,
                                          uint32_t band) {
    static_assert(A >= 1 && A <= 4 && RB >= 2 * A && (NW == 4 || NW == 8), "band shape");
    // x3[w]: tap-3 gradients of the a rows above wavefront w's rows;
    // x5[w]: tap-5 gradients of the a rows below wavefront w-1's rows.
    __shared__ f4 x3[NW + 1][A][64];
    __shared__ f4 x5[NW + 1][A][64];
    const uint32_t lane = threadIdx.x & 63u;
    // the wavefront index, uniform: row addresses and bounds are scalar
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int x0 = 4 * ((int)(strip * kVjpGroups + lane) - kVjpLead);
    const int xl = min(max(x0, 0), f.W - 4);
    const int y0 = (int)(band * (uint32_t)(NW * RB));
    const int yw = y0 + (int)w * RB;
    const bool out_lane = (lane >= (uint32_t)kVjpLead) &
                          (lane < (uint32_t)(kVjpLead + kVjpGroups)) & (x0 < f.W);
    auto put = [&](int y, f4 v) {
        if (out_lane && y < f.H)
            out_store(v, out_buf(gd + (int64_t)y * f.W, 4u * (uint32_t)f.W), 4u * (uint32_t)x0);
    };
    // The band's 2a outer rows, dealt round the wavefronts.
    for (int k = (int)w; k < 2 * A; k += NW) {
        if (k < A) {
            x3[0][k][lane] = vjp4_row<A>(f, gn, y0 - A + k, x0, xl, lane).g3;
        } else {
            x5[NW][k - A][lane] = vjp4_row<A>(f, gn, y0 + NW * RB + (k - A), x0, xl, lane).g5;
        }
    }
    f4 h[RB], g3[RB], top5[A], bot[A];
    // each row's loads are issued before the previous row is evaluated
    RowLoad cur, nxt;
    vjp4_load<A>(f, gn, yw, x0, xl, lane, cur);
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        if (i + 1 < RB) vjp4_load<A>(f, gn, yw + i + 1, x0, xl, lane, nxt);
        const RowGrads e = vjp4_eval<A>(f, yw + i, x0, lane, cur);
        cur = nxt;
        h[i] = e.h;
        g3[i] = e.g3;
        if (i < A) x5[w][i][lane] = e.g5;             // for the wavefront above
        if (i >= RB - A) x3[w + 1][i - (RB - A)][lane] = e.g3;  // for the one below
        const int j = i - A;                           // the row that e.g5 completes
        if (j >= 0 && j < A) top5[j] = e.g5;
        if (j >= A && j < RB - A) put(yw + j, (h[j] + g3[j - A]) + e.g5);
        if (i >= RB - A) bot[i - (RB - A)] = h[i] + g3[i - A];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < A; ++j) put(yw + j, (h[j] + x3[w][j][lane]) + top5[j]);
#pragma unroll
    for (int j = 0; j < A; ++j) put(yw + RB - A + j, bot[j] + x5[w + 1][j][lane]);
}

template <int A, int RB, int NW>
__global__ __launch_bounds__(64 * NW) void k_vjp4(FrameArgs f, const float *__restrict__ gn,
                                                  float *__restrict__ gd, uint32_t strips) {
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    vjp4_band<A, RB, NW>(f, gn, gd, b % strips, b / strips);
}

// A stack: workgroup b takes band-strip b % T of frame b / T.
template <int A, int RB, int NW>
__global__ __launch_bounds__(64 * NW) void k_vjp4_stack(const StackArgs s) {
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t k = b / s.tiles_per_frame;
    const uint32_t t = b - k * s.tiles_per_frame;
    const int64_t npix = (int64_t)s.f.npix;
    vjp4_band<A, RB, NW>(stack_frame(s, k), s.gn + (int64_t)k * npix * 3,
                         s.gd + (int64_t)k * npix, t % s.tiles_x, t / s.tiles_x);
}

// Rows per wavefront: the fewest that the band edges allow (RB >= 2a), so
// that the grid holds the most workgroups: 4 for a <= 2, 8 for a = 3, 4.
// (Measured with six buffer sets: 8-row bands for a = 2 took 14.9 against
// 11.6 us on a 1920x1080 frame, 35.9 against 31.2 us on 64 frames of
// 320x240, and the same on 16 frames of 640x480 or 4 of 1920x1080.)
// Wavefronts per workgroup: 8 (a band of 8 RB rows shares its 2a outer rows
// among more rows) when that still gives kVjpWide workgroups, else 4
// (measured: 16 x 640x480 25.4 against 26.1 us, 4 x 1920x1080 39.5
// against 41.2; one 1920x1080 frame, 306 workgroups of 8, 13.4 against
// 12.4 us).
constexpr uint64_t kVjpWide = 512;

struct Vjp4Shape {
    int rb, nw;
    uint32_t strips, bands;
};

static Vjp4Shape vjp4_shape(int32_t H, int32_t W, int32_t n, int alpha) {
    Vjp4Shape s;
    s.strips = (uint32_t)((W / 4 + kVjpGroups - 1) / kVjpGroups);
    s.rb = alpha <= 2 ? 4 : 8;
    const uint64_t wide = (uint64_t)s.strips * (uint64_t)((H + 8 * s.rb - 1) / (8 * s.rb)) * n;
    s.nw = wide >= kVjpWide ? 8 : 4;
    s.bands = (uint32_t)((H + s.nw * s.rb - 1) / (s.nw * s.rb));
    return s;
}

typedef void (*Vjp4Fn)(FrameArgs, const float *, float *, uint32_t);
typedef void (*Vjp4StackFn)(const StackArgs);

template <int NW>
static Vjp4Fn vjp4_kernel_w(int a) {
    switch (a) {
        case 1: return k_vjp4<1, 4, NW>;
        case 2: return k_vjp4<2, 4, NW>;
        case 3: return k_vjp4<3, 8, NW>;
        case 4: return k_vjp4<4, 8, NW>;
    }
    return nullptr;
}

template <int NW>
static Vjp4StackFn vjp4_stack_kernel_w(int a) {
    switch (a) {
        case 1: return k_vjp4_stack<1, 4, NW>;
        case 2: return k_vjp4_stack<2, 4, NW>;
        case 3: return k_vjp4_stack<3, 8, NW>;
        case 4: return k_vjp4_stack<4, 8, NW>;
    }
    return nullptr;
}

static Vjp4Fn vjp4_kernel(const Vjp4Shape &sh, int a) {
    return sh.nw == 8 ? vjp4_kernel_w<8>(a) : vjp4_kernel_w<4>(a);
}

static Vjp4StackFn vjp4_stack_kernel(const Vjp4Shape &sh, int a) {
    return sh.nw == 8 ? vjp4_stack_kernel_w<8>(a) : vjp4_stack_kernel_w<4>(a);
}

static bool aligned16(const void *p) { return ((uintptr_t)p % 16) == 0; }

// The vector kernels' layout: rows of whole, 16-byte aligned float4 groups.
static bool vjp4_layout(const float *depth, int32_t W, int64_t stride, int64_t fstride,
                        const float *gn, const float *gd, int alpha) {
    return alpha <= 4 && W % 4 == 0 && stride % 4 == 0 && fstride % 4 == 0 && aligned16(depth) &&
           aligned16(gn) && aligned16(gd);
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
    if ((uintptr_t)grad_depth % 4) return BN_ERR_INVALID_ARG;
    if (vjp4_layout(depth, width, depth_stride, 0, grad_normals, grad_depth, params->alpha)) {
        const Vjp4Shape sh = vjp4_shape(height, width, 1, params->alpha);
        Vjp4Fn fn = vjp4_kernel(sh, params->alpha);
        if (!fn) return BN_ERR_UNSUPPORTED;
        FrameArgs f;
        fill_frame_args(f, depth, height, width, depth_stride, fx, fy, cx, cy, params, nullptr,
                        nullptr, nullptr, 1);
        hipLaunchKernelGGL(fn, dim3(sh.strips * sh.bands), dim3(64 * sh.nw), 0, (hipStream_t)stream,
                           f, grad_normals, grad_depth, sh.strips);
        return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
    }
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
    s.gn = grad_normals;
    s.gd = grad_depth;
    if (vjp4_layout(depth, width, depth_stride, depth_frame_stride, grad_normals, grad_depth,
                    params->alpha)) {
        const Vjp4Shape sh = vjp4_shape(height, width, s.n, params->alpha);
        Vjp4StackFn fn = vjp4_stack_kernel(sh, params->alpha);
        if (!fn) return BN_ERR_UNSUPPORTED;
        s.tiles_x = sh.strips;
        s.tiles_per_frame = sh.strips * sh.bands;
        const uint64_t grid = (uint64_t)s.tiles_per_frame * s.n;
        hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(64 * sh.nw), 0, (hipStream_t)stream, s);
        return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
    }
    // each frame is small when the stack as a whole would not fill the chip
    // with the larger tiles
    const bool small = (int64_t)height * width * n < (1 << 20);
    const uint32_t TX = small ? 32u : 64u, TY = small ? 8u : 16u;
    VjpStackFn fn = small ? vjp_stack_kernel_t<32, 8>(params->alpha)
                          : vjp_stack_kernel_t<64, 16>(params->alpha);
    if (!fn) return BN_ERR_UNSUPPORTED;
    s.tiles_x = ((uint32_t)width + TX - 1) / TX;
    s.tiles_per_frame = s.tiles_x * (((uint32_t)height + TY - 1) / TY);
    const uint64_t grid = (uint64_t)s.tiles_per_frame * s.n;
    hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kBlock), 0, (hipStream_t)stream, s);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}
