// Device-side pieces shared by every kernel of the library: the per-pixel
// evaluation (stencil validity, the reformulated normal of Eqs. 10-12 in the
// scaled form m = -(4 fx fy / alpha) n, the binary32 boundary decision of
// Section 3.2) and the frame arguments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnormals.h"

// Every expression below must round once per written operation, in the
// written order: the boundary mask is specified bit for bit.
#pragma clang fp contract(off)

namespace bn {

typedef float f4 __attribute__((ext_vector_type(4)));

// Everything a kernel needs to process one frame.
struct FrameArgs {
    const float *depth;
    float *normals;
    uint8_t *mask;
    bn_frame_stats *stats;
    int64_t stride;      // depth row stride, elements
    int32_t H, W;
    float fx, fy, cx, cy;
    float af;            // (float)alpha
    float tt;            // tau*tau (REL)
    float hconst;        // K (ABS) or +inf (NONE)
    int32_t rel;         // 1 for REL
    uint32_t gpr;        // work items per row (W/4 for vector kernels, W for scalar)
    uint32_t nitems;     // gpr * H
    double inv_gpr;      // 1.0 / gpr
};

// A finite depth > 0: bit patterns 0x00000001 .. 0x7f7fffff.  Integer test,
// so it does not depend on the denormal mode.
__device__ __forceinline__ uint32_t tap_ok(float d) {
    return (__float_as_uint(d) - 1u) < 0x7f7fffffu ? 1u : 0u;
}

// q is a finite number >= FLT_MIN: bit patterns 0x00800000 .. 0x7f7fffff.
__device__ __forceinline__ uint32_t q_ok(float q) {
    return (__float_as_uint(q) - 0x00800000u) < 0x7f000000u ? 1u : 0u;
}

// Row of a flat work item: floor(i / gpr) exactly, for i < 2^28 and
// gpr <= 2^16.  (i + 0.5)/gpr sits at least 0.5/gpr away from an integer;
// the double rounding error is below (i+1) * 2^-52.
__device__ __forceinline__ uint32_t row_of(uint32_t i, double inv_gpr) {
    return (uint32_t)(((double)i + 0.5) * inv_gpr);
}

struct PixelOut {
    float nx, ny, nz;
    uint32_t code;
};

// One pixel.  inside: the stencil lies in the image.  Taps d1..d5 as in
// the stencil of Section 3.1.  Branch-free: lanes with bad input compute
// garbage that the selects discard.
__device__ __forceinline__ PixelOut eval_pixel(bool inside, float d1, float d2, float d3,
                                               float d4, float d5, float xc, float yc,
                                               const FrameArgs &f) {
    const float P = d2 - d4;
    const float S = d2 + d4;
    const float Q = d3 - d5;
    const float T = d3 + d5;
    const float a = T * P;
    const float b = S * Q;
    const float c = S * T;
    const float mx = f.fx * a;
    const float my = f.fy * b;
    const float xa = xc * a;
    const float yb = yc * b;
    const float t3 = xa + yb;
    const float w = f.af * c;
    const float mz = t3 + w;
    const float mx2 = mx * mx;
    const float my2 = my * my;
    const float mz2 = mz * mz;
    const float q = (mx2 + my2) + mz2;
    const float ww = w * w;
    const float hrel = f.tt * ww;
    const float h = f.rel ? hrel : f.hconst;
    const bool ok = ((inside ? 1u : 0u) & tap_ok(d1) & tap_ok(d2) & tap_ok(d3) & tap_ok(d4) &
                     tap_ok(d5) & q_ok(q)) != 0u;
    const bool fire = q > h;
    PixelOut o;
    o.code = ok ? (fire ? (uint32_t)BN_BOUNDARY : (uint32_t)BN_VALID) : (uint32_t)BN_INVALID;
    const bool valid = ok && !fire;
    const float inv = __builtin_amdgcn_rsqf(q);
    o.nx = valid ? mx * inv : 0.0f;
    o.ny = valid ? my * inv : 0.0f;
    o.nz = valid ? -(mz * inv) : 0.0f;
    return o;
}

}  // namespace bn
