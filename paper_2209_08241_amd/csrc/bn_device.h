// Device-side pieces shared by every kernel of the library: the per-pixel
// evaluation (stencil validity, the reformulated normal of Eqs. 10-12 in the
// scaled form m = -(4 fx fy / alpha) n, the binary32 boundary decision of
// Section 3.2), wavefront lane shifts, and the in-launch reduction of the
// per-frame counts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnormals.h"

// Every expression below must round once per written operation, in the
// written order: the boundary mask is specified bit for bit.
#pragma clang fp contract(off)

namespace bn {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;  // 4 wave64 per workgroup

// Everything a kernel needs to process one frame.
struct FrameArgs {
    const float *depth;
    float *normals;
    uint8_t *mask;
    bn_frame_stats *stats;
    int64_t stride;   // depth row stride, elements
    int32_t H, W;
    float fx, fy, cx, cy;
    float af;         // (float)alpha
    float tt;         // tau*tau (REL)
    float hconst;     // K (ABS) or +inf (NONE)
    int32_t rel;      // 1 for REL
    uint32_t gpr;     // work items per row (W/4 for vector kernels, W for scalar)
    uint32_t nitems;  // gpr * H
    uint32_t npix;    // H * W
    double inv_gpr;   // 1.0 / gpr
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
// Wavefront lane shifts (DPP wave_shr:1 / wave_shl:1).  Lane i receives the
// value of lane i-1 (from_left) or i+1 (from_right); the lane without a
// source receives 0.  Every lane of the wave must execute these.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ f4 from_left(f4 v) {
    return f4{from_left(v.x), from_left(v.y), from_left(v.z), from_left(v.w)};
}
__device__ __forceinline__ f4 from_right(f4 v) {
    return f4{from_right(v.x), from_right(v.y), from_right(v.z), from_right(v.w)};
}

__device__ __forceinline__ uint32_t wave_count(bool pred) {
    return (uint32_t)__popcll(__ballot(pred));
}

// ---------------------------------------------------------------------------
// Per-frame counts, reduced inside the launch.
//
// A frame's pixels are split into `nparts` parts (workgroups or tiles).  Each
// part contributes its VALID and BOUNDARY counts with ONE relaxed 64-bit
// atomic add on the word of slot (part % BN_STATS_SLOTS), each slot on its
// own 128-byte line of the caller's bn_frame_stats so that the adds of
// different slots proceed in parallel.  The word packs the counts and an
// arrival ticket, so the value the atomic returns holds every earlier
// contribution: the last arrival of a slot (ticket = parts in the slot - 1)
// knows the slot total without any fence or reload.  It clears the slot and
// forwards the total the same way to the level-2 word; the last of those
// adds the frame totals to the counters (INVALID = pixels - VALID - BOUNDARY)
// and clears the level-2 word.  The workspace is therefore zero again after
// every launch.
//
// Level 1 word: VALID [0,24) | BOUNDARY [24,48) | ticket [48,64)
//   (a slot holds fewer than 2^24 pixels and 2^16 parts for frames of at
//    most 2^28 pixels and parts of at most 2^12 pixels).
// Level 2 word: VALID [0,29) | BOUNDARY [29,58) | ticket [58,64)
//   (at most 2^28 pixels, at most BN_STATS_SLOTS = 32 arrivals).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long *stats_word(bn_frame_stats *st, uint32_t slot) {
    // slot 0..31: level 1 (lines 1..32); BN_STATS_SLOTS: level 2 (header line)
    return reinterpret_cast<unsigned long long *>(
        slot < BN_STATS_SLOTS ? &st->work[14 + 16 * slot] : &st->work[0]);
}

// First half: the level-1 atomic.  Its result is used only in the second
// half, so the caller can place other work (the output stores) in between
// and hide the atomic's round trip behind it.
struct CountTicket {
    bn_frame_stats *st;
    unsigned long long *w1;
    unsigned long long mine1;
    unsigned long long old1;
    uint32_t ns, nparts, npix;
};

__device__ __forceinline__ CountTicket count_issue(bn_frame_stats *st, uint32_t part,
                                                   uint32_t nparts, uint32_t nvalid,
                                                   uint32_t nboundary, uint32_t npix) {
    CountTicket k;
    const uint32_t s = part % BN_STATS_SLOTS;
    k.st = st;
    k.ns = nparts / BN_STATS_SLOTS + (s < nparts % BN_STATS_SLOTS ? 1u : 0u);
    k.nparts = nparts;
    k.npix = npix;
    k.w1 = stats_word(st, s);
    k.mine1 = (unsigned long long)nvalid | ((unsigned long long)nboundary << 24) | (1ull << 48);
    k.old1 = atomicAdd(k.w1, k.mine1);
    return k;
}

__device__ __forceinline__ void count_finish(const CountTicket &k) {
    if ((uint32_t)(k.old1 >> 48) != k.ns - 1u) return;
    const unsigned long long tot1 = k.old1 + k.mine1;
    atomicExch(k.w1, 0ull);
    const uint32_t vs = (uint32_t)(tot1 & 0xffffffull);
    const uint32_t bs = (uint32_t)((tot1 >> 24) & 0xffffffull);
    const uint32_t nactive =
        k.nparts < (uint32_t)BN_STATS_SLOTS ? k.nparts : (uint32_t)BN_STATS_SLOTS;
    unsigned long long *w2 = stats_word(k.st, BN_STATS_SLOTS);
    const unsigned long long mine2 =
        (unsigned long long)vs | ((unsigned long long)bs << 29) | (1ull << 58);
    const unsigned long long old2 = atomicAdd(w2, mine2);
    if ((uint32_t)(old2 >> 58) != nactive - 1u) return;
    const unsigned long long tot2 = old2 + mine2;
    atomicExch(w2, 0ull);
    const uint32_t vt = (uint32_t)(tot2 & ((1ull << 29) - 1));
    const uint32_t bt = (uint32_t)((tot2 >> 29) & ((1ull << 29) - 1));
    atomicAdd(&k.st->n_valid, vt);
    atomicAdd(&k.st->n_boundary, bt);
    atomicAdd(&k.st->n_invalid, k.npix - vt - bt);
}

__device__ __forceinline__ void reduce_counts(bn_frame_stats *st, uint32_t part, uint32_t nparts,
                                              uint32_t nvalid, uint32_t nboundary,
                                              uint32_t npix) {
    count_finish(count_issue(st, part, nparts, nvalid, nboundary, npix));
}

// Block-wide sum of wave-uniform counts (one workgroup barrier): the totals,
// valid in thread 0 only.
__device__ __forceinline__ void block_sum(uint32_t cv, uint32_t cb, uint32_t &v, uint32_t &b) {
    __shared__ uint32_t s_cnt[kBlock / 64][2];
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
        for (int w = 0; w < kBlock / 64; ++w) {
            v += s_cnt[w][0];
            b += s_cnt[w][1];
        }
    }
}

// Block-wide sum of wave-uniform counts; thread 0 then calls reduce_counts.
__device__ __forceinline__ void block_counts(bn_frame_stats *st, uint32_t part, uint32_t nparts,
                                             uint32_t cv, uint32_t cb, uint32_t npix) {
    uint32_t v, b;
    block_sum(cv, cb, v, b);
    if (threadIdx.x == 0) reduce_counts(st, part, nparts, v, b, npix);
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b%8).
// Give each XCD a contiguous run of tiles so that the rows a tile shares with
// its neighbours (the stencil halo) are fetched into that XCD's L2 once.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nblocks) {
    const uint32_t per = nblocks >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7u) * per + (b >> 3);
}

}  // namespace bn
