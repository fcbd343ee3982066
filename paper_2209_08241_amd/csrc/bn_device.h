// Device-side pieces shared by every kernel of the library: the per-pixel
// evaluation (stencil validity, the reformulated normal of Eqs. 10-12 in the
// scaled form m = -(4 fx fy / alpha) n, the binary32 boundary decision of
// Section 3.2, and the two variants: per-pair removal and the multi-scale
// single pair of Eqs. 1-6), wavefront lane shifts, and the in-launch
// reduction of the per-frame counts.
#pragma once

#include <cstddef>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnormals.h"

// Every expression below must round once per written operation, in the
// written order: the boundary mask is specified bit for bit.
#pragma clang fp contract(off)

namespace bn {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;  // 4 wave64 per workgroup

// The in-launch reduction's device words for one frame (library-owned; zero
// between launches): line 0 holds the root word, lines 1..kSlots the slot
// words, one 128-byte line each so that the slots' atomics proceed in
// parallel.
constexpr uint32_t kSlots = 32;
struct WorkArea {
    unsigned long long w[16 * (kSlots + 1)];
};
static_assert(sizeof(WorkArea) == 128 * (kSlots + 1), "kSlots + 1 lines of 128 bytes");

// Everything a kernel needs to process one frame.
struct FrameArgs {
    const float *depth;
    float *normals;
    uint8_t *mask;
    bn_frame_stats *stats;  // the counts' destination (nullable)
    WorkArea *work;         // the in-launch reduction's words (library-owned)
    int64_t stride;   // depth row stride, elements
    int32_t H, W;
    float fx, fy, cx, cy;
    float af;         // (float)alpha
    float tt;         // tau*tau (REL)
    float hconst;     // K (ABS) or +inf (NONE), on the method's |m|^2 scale
    int32_t rel;      // 1 for REL
    uint32_t gpr;     // work items per row (W/4 for vector kernels, W for scalar)
    uint32_t nitems;  // gpr * H
    uint32_t npix;    // H * W
    int32_t alpha;    // integer alpha (multi-scale offsets)
    int32_t scales;   // K of the multi-scale method
    uint32_t overwrite;  // 1: counts replace the stats counters, 0: added (accumulate)
    double inv_gpr;   // 1.0 / gpr
};

// A stack of frames of one size in one launch: the first frame's arguments,
// the distance between frames' depth, and what differs per frame (the
// intrinsics and the ABS threshold that depends on them).  Outputs of frame
// k are frame k of dense [n][H][W][3] / [n][H][W] / [n] arrays.  Passed by
// value: the whole structure sits in the kernel-argument segment.
struct StackFrame {
    float fx, fy, cx, cy, hconst;
};

struct StackArgs {
    FrameArgs f;
    int64_t depth_fstride;     // elements from one frame's depth to the next
    uint32_t n;                // frames
    uint32_t tiles_per_frame;  // workgroups per frame
    uint32_t vec;              // 1: vector tiles
    uint32_t tiles_x;          // adjoint: tiles per row
    const float *gn;           // adjoint: cotangent [n][H][W][3]
    float *gd;                 // adjoint: gradient [n][H][W]
    StackFrame fr[BN_MAX_STACK];
};

// Frame pointers loaded from device memory (a batch's frame descriptors) are
// generic to the compiler, which then emits FLAT accesses through them; FLAT
// operations also count on the LDS counter, so every LDS wait of a tile
// would wait for the tile's memory traffic too.  Reading the pointer fields
// as global-address-space pointers lets the compiler use global
// instructions.  (The layout is FrameArgs' first five fields.)
#define BN_GLOBAL __attribute__((address_space(1)))
struct FramePointersGlobal {
    BN_GLOBAL const float *depth;
    BN_GLOBAL float *normals;
    BN_GLOBAL uint8_t *mask;
    BN_GLOBAL bn_frame_stats *stats;
    BN_GLOBAL WorkArea *work;
};

static_assert(sizeof(FramePointersGlobal) == 40 && offsetof(FrameArgs, work) == 32,
              "FramePointersGlobal mirrors the first fields of FrameArgs");

__device__ __forceinline__ void frame_pointers_global(FrameArgs &f, const FrameArgs *src) {
    const FramePointersGlobal g = *reinterpret_cast<const FramePointersGlobal *>(src);
    f.depth = (const float *)g.depth;
    f.normals = (float *)g.normals;
    f.mask = (uint8_t *)g.mask;
    f.stats = (bn_frame_stats *)g.stats;
    f.work = (WorkArea *)g.work;
}

// Arguments of frame k of a stack.
__device__ __forceinline__ FrameArgs stack_frame(const StackArgs &s, uint32_t k) {
    FrameArgs f = s.f;
    const StackFrame &p = s.fr[k];
    f.fx = p.fx;
    f.fy = p.fy;
    f.cx = p.cx;
    f.cy = p.cy;
    f.hconst = p.hconst;
    const int64_t npix = (int64_t)f.npix;
    f.depth += (int64_t)k * s.depth_fstride;
    if (f.normals) f.normals += (int64_t)k * npix * 3;
    if (f.mask) f.mask += (int64_t)k * npix;
    if (f.stats) f.stats += k;
    if (f.work) f.work += k;
    return f;
}

// Methods (bn_params.method).
constexpr int kFourPair = BN_METHOD_FOUR_PAIR;
constexpr int kPairRemoval = BN_METHOD_PAIR_REMOVAL;
constexpr int kMultiScale = BN_METHOD_MULTISCALE;
// Largest alpha * scales the multi-scale vector tiles serve: the row window
// then spans at most 4 float4s right of the lane's own, and the vertical taps
// at most min(8, 16 / alpha) float4s of the rows below.  Reaches up to
// kMsShortReach take a separate instantiation with half the registers
// (kernel method kMultiScaleLong marks the longer one; it is no public
// method value).
constexpr int kMsVecReach = 16;
constexpr int kMsShortReach = 8;
constexpr int kMultiScaleLong = 0x12;

__host__ __device__ constexpr bool is_multiscale(int m) {
    return m == kMultiScale || m == kMultiScaleLong;
}

// The kernel method of a request: the public method, with multi-scale
// reaches beyond kMsShortReach on the longer instantiation.
__host__ __device__ constexpr int kernel_method(int method, int alpha, int scales) {
    return method == kMultiScale && alpha * scales > kMsShortReach ? kMultiScaleLong : method;
}

// A constant placed in a scalar register.  The class tests below take their
// class mask as a second operand that cannot be a literal in this encoding;
// left to itself the compiler rebuilds the mask in a vector register before
// each pixel's tests (one VALU move each), where a scalar register serves
// them all.
__device__ __forceinline__ uint32_t sconst(uint32_t v) {
    uint32_t r;
    asm("s_mov_b32 %0, %1" : "=s"(r) : "i"(v));
    return r;
}

// A finite depth > 0: bit patterns 0x00000001 .. 0x7f7fffff, that is the
// classes positive subnormal and positive normal (one class test: it reads
// the bit pattern, whatever the denormal mode).
__device__ __forceinline__ uint32_t tap_ok(float d) {
    return __builtin_amdgcn_classf(d, sconst(0x180)) ? 1u : 0u;  // +subnormal | +normal
}

// q is a finite number >= FLT_MIN: bit patterns 0x00800000 .. 0x7f7fffff,
// the class positive normal.
__device__ __forceinline__ uint32_t q_ok(float q) {
    return __builtin_amdgcn_classf(q, sconst(0x100)) ? 1u : 0u;  // +normal
}

// Row of a flat work item: floor(i / gpr) exactly, for i < 2^28 and
// gpr <= 2^16.  (i + 0.5)/gpr sits at least 0.5/gpr away from an integer;
// the double rounding error is below (i+1) * 2^-52.
__device__ __forceinline__ uint32_t row_of(uint32_t i, double inv_gpr) {
    return (uint32_t)(((double)i + 0.5) * inv_gpr);
}

// One pixel, keeping the scaled vector and its pieces.  inside: the stencil
// lies in the image.  Taps d1..d5 as in the stencil of Section 3.1.
// Branch-free: lanes with bad input compute garbage that the code discards.
struct PixelTerms {
    float P, S, Q, T;
    float mx, my, mz;  // mz = t3 + w, the negated third component of m
    float q;
    uint32_t code;
};

__device__ __forceinline__ PixelTerms eval_terms(bool inside, float d1, float d2, float d3,
                                                 float d4, float d5, float xc, float yc,
                                                 const FrameArgs &f) {
    PixelTerms r;
    r.P = d2 - d4;
    r.S = d2 + d4;
    r.Q = d3 - d5;
    r.T = d3 + d5;
    const float a = r.T * r.P;
    const float b = r.S * r.Q;
    const float c = r.S * r.T;
    r.mx = f.fx * a;
    r.my = f.fy * b;
    const float xa = xc * a;
    const float yb = yc * b;
    const float t3 = xa + yb;
    const float w = f.af * c;
    r.mz = t3 + w;
    const float mx2 = r.mx * r.mx;
    const float my2 = r.my * r.my;
    const float mz2 = r.mz * r.mz;
    r.q = (mx2 + my2) + mz2;
    const float ww = w * w;
    const float hrel = f.tt * ww;
    const float h = f.rel ? hrel : f.hconst;
    const bool ok = ((inside ? 1u : 0u) & tap_ok(d1) & tap_ok(d2) & tap_ok(d3) & tap_ok(d4) &
                     tap_ok(d5) & q_ok(r.q)) != 0u;
    const bool fire = r.q > h;
    r.code = ok ? (fire ? (uint32_t)BN_BOUNDARY : (uint32_t)BN_VALID) : (uint32_t)BN_INVALID;
    return r;
}

struct PixelOut {
    float nx, ny, nz;
    uint32_t code;
};

// One pixel: its code and, when VALID, the camera-facing unit normal
// (mx, my, -mz) / sqrt(q); the zero vector otherwise.
__device__ __forceinline__ PixelOut eval_pixel(bool inside, float d1, float d2, float d3,
                                               float d4, float d5, float xc, float yc,
                                               const FrameArgs &f) {
    const PixelTerms t = eval_terms(inside, d1, d2, d3, d4, d5, xc, yc, f);
    PixelOut o;
    o.code = t.code;
    const bool valid = t.code == BN_VALID;
    const float inv = __builtin_amdgcn_rsqf(t.q);
    o.nx = valid ? t.mx * inv : 0.0f;
    o.ny = valid ? t.my * inv : 0.0f;
    o.nz = valid ? -(t.mz * inv) : 0.0f;
    return o;
}

// ---------------------------------------------------------------------------
// Pair removal.  The four perpendicular pairs of Eq. 7, n23, n34, n45, n52,
// each as m_p = -(fx fy / alpha) n_p = (fx A, fy B, -(xc A + yc B + alpha C))
// with, for horizontal tap h, vertical tap v and their directions sh, sv:
//   A = sh (d_h - d1) d_v,  B = sv d_h (d_v - d1),  C = d_h d_v
// (Eqs. 1-3 scaled for the pair (2, 3)).  Each pair is tested like the
// four-pair vector, with w_p = (alpha d_h) d_v (alpha C), its third component
// and squared length taken with fused multiply-adds; the passing pairs are
// summed in pair order, each sum starting from +0 (adding +0 for a failing
// pair changes no bit of the squared length).  When all four pass, the sum is the
// four-pair m, taken in its closed form (d1 cancels exactly there, while the
// rounded sum of the pairs can lose it to cancellation).
// ---------------------------------------------------------------------------
// The binary32 vector of one pair and its test, given w = (alpha d_h) d_v:
//   mx = fx A, my = fy B,
//   mz = fma(xc, A, fma(yc, B, w)),  q = fma(mx, mx, fma(my, my, mz mz)),
// each fused multiply-add rounded once; the pair fails iff
// q > fma(rel_k w, w, abs_k) with (rel_k, abs_k) = (tau^2, 0) for REL, that
// is q > (tau^2 w) w with both products rounded, and (0, K) otherwise (0 w is
// a signed zero for every finite w, so the threshold is K; a w that is not
// finite comes from a tap product that overflowed, whose q is not finite
// either, and the pixel is INVALID whatever the test says).
// keep: the pair passes; ok: its q is a finite number >= FLT_MIN.
struct PairT {
    float mx, my, mz;
    bool keep, ok;
};

__device__ __forceinline__ PairT pair_t(float A, float B, float w, float xc, float yc,
                                        float rel_k, float abs_k, const FrameArgs &f) {
    PairT r;
    r.mx = f.fx * A;
    r.my = f.fy * B;
    r.mz = __builtin_fmaf(xc, A, __builtin_fmaf(yc, B, w));
    const float q = __builtin_fmaf(r.mx, r.mx, __builtin_fmaf(r.my, r.my, r.mz * r.mz));
    const float h = __builtin_fmaf(rel_k * w, w, abs_k);
    r.keep = !(q > h);
    r.ok = __builtin_amdgcn_classf(q, sconst(0x100));
    return r;
}

// The four-pair closed form m (Eqs. 10-12) as pair removal takes it when all
// four pairs pass: the products of eval_terms, the third component fused as
// for one pair.
struct ClosedM {
    float mx, my, mz;
};

__device__ __forceinline__ ClosedM closed_m(float d2, float d3, float d4, float d5, float xc,
                                            float yc, const FrameArgs &f) {
    const float P = d2 - d4;
    const float S = d2 + d4;
    const float Q = d3 - d5;
    const float T = d3 + d5;
    const float a = T * P;
    const float b = S * Q;
    const float c = S * T;
    ClosedM r;
    r.mx = f.fx * a;
    r.my = f.fy * b;
    const float w = f.af * c;
    r.mz = __builtin_fmaf(xc, a, __builtin_fmaf(yc, b, w));
    return r;
}

// Pair removal.  The four pairs' vectors and tests, then the closed form;
// where some pair fails (a wavefront-uniform branch) the passing pairs'
// vectors are summed in pair order from +0.  Each step of that sum is
// fma(k, m_p, t) with k = 1 for a passing pair and 0 for a failing one: for a
// passing pair that is t + m_p rounded once, as the plain sum; for a failing
// one it adds a zero, which leaves every t of the sum unchanged (t is never
// -0: it starts as k m_0 + (+0)).  A failing pair whose vector is not finite
// has a q that is not finite either, and then the pixel is INVALID whatever
// the sum holds.  The squared length of the closed form or of the sum,
// whichever the pixel takes, is fused as a pair's.
__device__ __forceinline__ PixelOut eval_pixel_pairs(bool inside, float d1, float d2, float d3,
                                                     float d4, float d5, float xc, float yc,
                                                     const FrameArgs &f) {
    const float e2 = d2 - d1;
    const float e3 = d3 - d1;
    const float e4 = d4 - d1;
    const float e5 = d5 - d1;
    const float rel_k = f.rel ? f.tt : 0.0f;
    const float abs_k = f.rel ? 0.0f : f.hconst;
    const float a2 = f.af * d2;
    const float a4 = f.af * d4;
    // (h, v) = (2, 3), (4, 3), (4, 5), (2, 5); sh, sv = ++, -+, --, +-
    const PairT p0 = pair_t(e2 * d3, d2 * e3, a2 * d3, xc, yc, rel_k, abs_k, f);
    const PairT p1 = pair_t(-(e4 * d3), d4 * e3, a4 * d3, xc, yc, rel_k, abs_k, f);
    const PairT p2 = pair_t(-(e4 * d5), -(d4 * e5), a4 * d5, xc, yc, rel_k, abs_k, f);
    const PairT p3 = pair_t(e2 * d5, -(d2 * e5), a2 * d5, xc, yc, rel_k, abs_k, f);
    const bool all = p0.keep && p1.keep && p2.keep && p3.keep;
    const bool any = p0.keep || p1.keep || p2.keep || p3.keep;
    // all four pass: the four-pair closed form, in which d1 cancels exactly
    const ClosedM c = closed_m(d2, d3, d4, d5, xc, yc, f);
    float sx = c.mx, sy = c.my, sz = c.mz;
    if (__builtin_amdgcn_ballot_w64(!all) != 0) {
        const float k0 = p0.keep ? 1.0f : 0.0f;
        const float k1 = p1.keep ? 1.0f : 0.0f;
        const float k2 = p2.keep ? 1.0f : 0.0f;
        const float k3 = p3.keep ? 1.0f : 0.0f;
        float tx = __builtin_fmaf(k0, p0.mx, 0.0f);
        float ty = __builtin_fmaf(k0, p0.my, 0.0f);
        float tz = __builtin_fmaf(k0, p0.mz, 0.0f);
        tx = __builtin_fmaf(k1, p1.mx, tx);
        ty = __builtin_fmaf(k1, p1.my, ty);
        tz = __builtin_fmaf(k1, p1.mz, tz);
        tx = __builtin_fmaf(k2, p2.mx, tx);
        ty = __builtin_fmaf(k2, p2.my, ty);
        tz = __builtin_fmaf(k2, p2.mz, tz);
        tx = __builtin_fmaf(k3, p3.mx, tx);
        ty = __builtin_fmaf(k3, p3.my, ty);
        tz = __builtin_fmaf(k3, p3.mz, tz);
        sx = all ? sx : tx;
        sy = all ? sy : ty;
        sz = all ? sz : tz;
    }
    const float Q = __builtin_fmaf(sx, sx, __builtin_fmaf(sy, sy, sz * sz));
    const bool ok = inside && (tap_ok(d1) & tap_ok(d2) & tap_ok(d3) & tap_ok(d4) & tap_ok(d5)) &&
                    p0.ok && p1.ok && p2.ok && p3.ok;
    PixelOut o;
    o.code = !ok ? (uint32_t)BN_INVALID
                 : (!any ? (uint32_t)BN_BOUNDARY
                         : (q_ok(Q) ? (uint32_t)BN_VALID : (uint32_t)BN_INVALID));
    const bool valid = o.code == BN_VALID;
    const float inv = __builtin_amdgcn_rsqf(Q);
    o.nx = valid ? sx * inv : 0.0f;
    o.ny = valid ? sy * inv : 0.0f;
    o.nz = valid ? -(sz * inv) : 0.0f;
    return o;
}

// The five-tap methods: four-pair average or pair removal.
template <int M>
__device__ __forceinline__ PixelOut eval_method(bool inside, float d1, float d2, float d3,
                                                float d4, float d5, float xc, float yc,
                                                const FrameArgs &f) {
    if (M == kPairRemoval) return eval_pixel_pairs(inside, d1, d2, d3, d4, d5, xc, yc, f);
    return eval_pixel(inside, d1, d2, d3, d4, d5, xc, yc, f);
}

// ---------------------------------------------------------------------------
// Multi-scale single pair (Eqs. 1-6): at pixel (x, y), whose row starts at
// p = depth + y * stride + x, the pair (2, 3) vector at offsets
// a_i = i * alpha, i = 1..K, weighted by a_i and summed in scale order
// (-K fx fy times the average of Eqs. 4-6); REL compares with
// tau^2 (sum a_i w_i)^2.  Only the taps right of and below the pixel are
// read: inside means x + K alpha < W and y + K alpha < H.
// ---------------------------------------------------------------------------
// One scale: the pair (2, 3) vector at offset a (taps d2 = (x+a, y),
// d3 = (x, y+a)), its third component fused as in pair removal, weighted by
// a and added to the running sums with fused multiply-adds.
__device__ __forceinline__ void ms_accumulate(float d1, float d2, float d3, float a, float xc,
                                              float yc, const FrameArgs &f, float &Mx, float &My,
                                              float &Mz, float &Wt) {
    const float e2 = d2 - d1;
    const float e3 = d3 - d1;
    const float A = e2 * d3;
    const float B = d2 * e3;
    const float C = d2 * d3;
    const float mx = f.fx * A;
    const float my = f.fy * B;
    const float w = a * C;
    const float mz = __builtin_fmaf(xc, A, __builtin_fmaf(yc, B, w));
    Mx = __builtin_fmaf(a, mx, Mx);
    My = __builtin_fmaf(a, my, My);
    Mz = __builtin_fmaf(a, mz, Mz);
    Wt = __builtin_fmaf(a, w, Wt);
}

__device__ __forceinline__ PixelOut ms_finish(uint32_t ok, float Mx, float My, float Mz, float Wt,
                                              const FrameArgs &f) {
    const float q = __builtin_fmaf(Mx, Mx, __builtin_fmaf(My, My, Mz * Mz));
    const float ww = Wt * Wt;
    const float hrel = f.tt * ww;
    const float h = f.rel ? hrel : f.hconst;
    PixelOut o;
    o.code = (ok & q_ok(q)) ? (q > h ? (uint32_t)BN_BOUNDARY : (uint32_t)BN_VALID)
                            : (uint32_t)BN_INVALID;
    const bool valid = o.code == BN_VALID;
    const float inv = __builtin_amdgcn_rsqf(q);
    o.nx = valid ? Mx * inv : 0.0f;
    o.ny = valid ? My * inv : 0.0f;
    o.nz = valid ? -(Mz * inv) : 0.0f;
    return o;
}

__device__ __forceinline__ PixelOut eval_pixel_multiscale(bool inside, const float *p, float xc,
                                                          float yc, const FrameArgs &f) {
    const float d1 = *p;
    uint32_t ok = (inside ? 1u : 0u) & tap_ok(d1);
    float Mx = 0.0f, My = 0.0f, Mz = 0.0f, Wt = 0.0f;
    if (inside) {
        for (int i = 1; i <= f.scales; ++i) {
            const int off = i * f.alpha;
            const float d2 = p[off];
            const float d3 = p[(int64_t)off * f.stride];
            ok &= tap_ok(d2) & tap_ok(d3);
            ms_accumulate(d1, d2, d3, (float)off, xc, yc, f, Mx, My, Mz, Wt);
        }
    }
    return ms_finish(ok, Mx, My, Mz, Wt, f);
}

// ---------------------------------------------------------------------------
// Output stores.  Normals and codes are written once and read by no later
// work item of the launch, so they are stored streaming (nt) at device scope
// (sc1): written through the XCD's L2 rather than left dirty in it (the
// cache-policy bits 2 and 16 of the gfx9 buffer-store builtins).  Each
// wavefront stores through a buffer resource that covers exactly its own
// share of the output, whose size the hardware checks every lane's offset
// against (raw buffer, stride 0): a lane whose store would start at or past
// the end stores nothing.  The base is wavefront-uniform, so the resource
// lives in scalar registers.
// ---------------------------------------------------------------------------
constexpr int kOutPolicy = 2 | 16;          // nt | sc1
constexpr int kRsrcFormat = 0x00020000;     // word 3: 32-bit data format, no swizzle

struct OutBuf {
    __amdgpu_buffer_rsrc_t r;
};

// The wavefront's index in its workgroup, as a scalar.
__device__ __forceinline__ uint32_t wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// base: wavefront-uniform; bytes: the size of the share, < 2^31.
__device__ __forceinline__ OutBuf out_buf(void *base, uint32_t bytes) {
    return OutBuf{__builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, kRsrcFormat)};
}
__device__ __forceinline__ void out_store(f4 v, const OutBuf &b, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b128(v, b.r, off, 0, kOutPolicy);
}
__device__ __forceinline__ void out_store(uint32_t v, const OutBuf &b, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(v, b.r, off, 0, kOutPolicy);
}
__device__ __forceinline__ void out_store(float v, const OutBuf &b, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), b.r, off, 0, kOutPolicy);
}
__device__ __forceinline__ void out_store_byte(uint8_t v, const OutBuf &b, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b8(v, b.r, off, 0, kOutPolicy);
}

// ---------------------------------------------------------------------------
// Wavefront lane shifts (DPP wave_shr:1 / wave_shl:1).  Lane i receives the
// value of lane i-1 (from_left) or i+1 (from_right); the lane without a
// source receives 0.  Every lane of the wave must execute these.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ f4 from_left(f4 v) {
    return f4{from_left(v.x), from_left(v.y), from_left(v.z), from_left(v.w)};
}
__device__ __forceinline__ f4 from_right(f4 v) {
    return f4{from_right(v.x), from_right(v.y), from_right(v.z), from_right(v.w)};
}

// The builtin ballot takes the lane mask of a compare as it is (HIP's
// __ballot takes an int and forms a 0/1 value per lane first).
__device__ __forceinline__ uint32_t wave_count(bool pred) {
    return (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(pred));
}

// ---------------------------------------------------------------------------
// Per-frame counts, reduced inside the launch.
//
// A frame's pixels are split into `nparts` parts (workgroups or tiles),
// numbered in about the order the hardware dispatches them.  The last
// kDirect parts contribute their VALID and BOUNDARY counts with ONE relaxed
// 64-bit atomic add on the root word of the frame's WorkArea; every other
// part adds to the word of slot (part % kSlots), each slot on its own
// 128-byte line so that the adds of different slots proceed in parallel.
// A word packs the counts and an arrival ticket, so the value the atomic
// returns holds every earlier contribution: the last arrival of a slot
// (ticket = parts in the slot - 1) knows the slot total without any fence
// or reload, clears the slot and forwards the total to the root the same
// way; the last arrival at the root (a slot's forward or a direct part)
// stores (or adds) the frame totals in the destination's counters (INVALID
// = pixels - VALID - BOUNDARY) and clears the root.  The work area is
// therefore zero again after every launch.  The parts dispatched last
// usually finish last, and a direct part that finishes last waits for one
// return before it stores the totals where a slot's part waits for two
// (1080p four-pair launch: 7.23-7.31 against 7.31-7.40 us).
//
// Slot word: VALID [0,24) | BOUNDARY [24,48) | ticket [48,64)
//   (a slot holds fewer than 2^24 pixels and 2^16 parts for frames of at
//    most 2^28 pixels and parts of at most 2^12 pixels).
// Root word: VALID [0,29) | BOUNDARY [29,58) | ticket [58,64)
//   (at most 2^28 pixels, at most kSlots + kDirect = 63 arrivals).
// ---------------------------------------------------------------------------
constexpr uint32_t kDirect = 31;
static_assert(kSlots + kDirect <= 63, "root arrivals fit the 6-bit ticket");

__device__ __forceinline__ unsigned long long *stats_word(WorkArea *wa, uint32_t slot) {
    // slot 0..kSlots-1: the slots (lines 1..kSlots); kSlots: the root (line 0)
    return &wa->w[slot < kSlots ? 16 * (slot + 1) : 0];
}

// First half: the part's atomic (on its slot or the root).  Its result is
// used only in the second half, so the caller can place other work (the
// output stores) in between and hide the atomic's round trip behind it.
struct CountTicket {
    WorkArea *work;
    bn_frame_stats *out;
    unsigned long long *w1;
    unsigned long long mine1;
    unsigned long long old1;
    uint32_t ns, npix, overwrite, nroot;
    bool direct;
};

__device__ __forceinline__ CountTicket count_issue(WorkArea *work, bn_frame_stats *out,
                                                   uint32_t part, uint32_t nparts,
                                                   uint32_t nvalid, uint32_t nboundary,
                                                   uint32_t npix, uint32_t overwrite) {
    CountTicket k;
    k.overwrite = overwrite;
    k.work = work;
    k.out = out;
    k.npix = npix;
    const uint32_t nslotted = nparts > kDirect ? nparts - kDirect : 0u;
    k.direct = part >= nslotted;
    k.nroot = (nslotted < kSlots ? nslotted : kSlots) + (nparts - nslotted);
    if (k.direct) {
        k.ns = 0;
        k.w1 = stats_word(work, kSlots);
        k.mine1 = (unsigned long long)nvalid | ((unsigned long long)nboundary << 29) | (1ull << 58);
    } else {
        const uint32_t s = part % kSlots;
        k.ns = nslotted / kSlots + (s < nslotted % kSlots ? 1u : 0u);
        k.w1 = stats_word(work, s);
        k.mine1 = (unsigned long long)nvalid | ((unsigned long long)nboundary << 24) | (1ull << 48);
    }
    k.old1 = atomicAdd(k.w1, k.mine1);
    return k;
}

// Frame totals into the counters: stored (with reserved = 0), or added.
__device__ __forceinline__ void put_counts(bn_frame_stats *st, uint32_t vt, uint32_t bt,
                                           uint32_t npix, uint32_t overwrite) {
    if (overwrite) {
        st->n_valid = vt;
        st->n_boundary = bt;
        st->n_invalid = npix - vt - bt;
        st->reserved = 0u;
    } else {
        atomicAdd(&st->n_valid, vt);
        atomicAdd(&st->n_boundary, bt);
        atomicAdd(&st->n_invalid, npix - vt - bt);
    }
}

// An arrival at the root: the last one stores the frame totals.
__device__ __forceinline__ void root_arrival(const CountTicket &k, unsigned long long old2,
                                             unsigned long long mine2) {
    if ((uint32_t)(old2 >> 58) != k.nroot - 1u) return;
    const unsigned long long tot2 = old2 + mine2;
    atomicExch(stats_word(k.work, kSlots), 0ull);
    const uint32_t vt = (uint32_t)(tot2 & ((1ull << 29) - 1));
    const uint32_t bt = (uint32_t)((tot2 >> 29) & ((1ull << 29) - 1));
    put_counts(k.out, vt, bt, k.npix, k.overwrite);
}

__device__ __forceinline__ void count_finish(const CountTicket &k) {
    if (k.direct) {
        root_arrival(k, k.old1, k.mine1);
        return;
    }
    if ((uint32_t)(k.old1 >> 48) != k.ns - 1u) return;
    const unsigned long long tot1 = k.old1 + k.mine1;
    atomicExch(k.w1, 0ull);
    const uint32_t vs = (uint32_t)(tot1 & 0xffffffull);
    const uint32_t bs = (uint32_t)((tot1 >> 24) & 0xffffffull);
    const unsigned long long mine2 =
        (unsigned long long)vs | ((unsigned long long)bs << 29) | (1ull << 58);
    root_arrival(k, atomicAdd(stats_word(k.work, kSlots), mine2), mine2);
}

__device__ __forceinline__ void reduce_counts(WorkArea *work, bn_frame_stats *out,
                                              uint32_t part, uint32_t nparts, uint32_t nvalid,
                                              uint32_t nboundary, uint32_t npix,
                                              uint32_t overwrite) {
    count_finish(count_issue(work, out, part, nparts, nvalid, nboundary, npix, overwrite));
}

// Block-wide sum of wave-uniform counts over a workgroup of TB threads (one
// workgroup barrier): the totals, valid in thread 0 only.
template <int TB = kBlock>
__device__ __forceinline__ void block_sum(uint32_t cv, uint32_t cb, uint32_t &v, uint32_t &b) {
    __shared__ uint32_t s_cnt[TB / 64][2];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_cnt[wave][0] = cv;
        s_cnt[wave][1] = cb;
    }
    __syncthreads();
    v = 0;
    b = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < TB / 64; ++w) {
            v += s_cnt[w][0];
            b += s_cnt[w][1];
        }
    }
}

// Block-wide sum of wave-uniform counts; thread 0 then calls reduce_counts.
__device__ __forceinline__ void block_counts(const FrameArgs &f, uint32_t part, uint32_t nparts,
                                             uint32_t cv, uint32_t cb) {
    uint32_t v, b;
    block_sum(cv, cb, v, b);
    if (threadIdx.x == 0) reduce_counts(f.work, f.stats, part, nparts, v, b, f.npix, f.overwrite);
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b%8).
// Within each window of 8 * kXcdRun consecutive workgroups, give each XCD a
// contiguous run of kXcdRun tiles, so that the rows a tile shares with its
// neighbours (the stencil halo) are fetched into that XCD's L2 once, while
// the 8 XCDs still stream through nearby addresses.  (One contiguous run per
// XCD over the whole frame keeps the L2 benefit but sends the XCDs to 8
// distant regions of HBM at once; measured 10-20% slower on frames of
// 12-168 Mpixel.)  The last, partial window is split the same way into 8
// runs of its size / 8, and its remainder keeps its own numbers.
constexpr uint32_t kXcdRun = 64;

__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nblocks) {
    constexpr uint32_t kWin = 8 * kXcdRun;
    const uint32_t base = b / kWin * kWin;
    const uint32_t lb = b - base;
    if (base + kWin <= nblocks) return base + (lb & 7u) * kXcdRun + (lb >> 3);
    const uint32_t per = (nblocks - base) >> 3;
    if (lb >= (per << 3)) return b;
    return base + (lb & 7u) * per + (lb >> 3);
}

}  // namespace bn
