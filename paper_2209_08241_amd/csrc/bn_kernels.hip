// Plain (one frame per launch) kernels for gfx950.
//
// The estimator is a memory-bound 5-point stencil: 4 bytes of depth in,
// 12 bytes of normal and 1 byte of code out per pixel, about 40 binary32
// operations in between.  The kernels therefore aim at full-width coalesced
// HBM traffic: 16-byte vector loads and stores, horizontal taps served from
// the same cache lines, vertical taps from the L2 of the XCD that reads the
// neighbouring rows, and per-frame counts reduced in registers (wavefront
// ballots) before one atomic per counter per workgroup.
#include "bn_device.h"
#include "bn_internal.h"

#pragma clang fp contract(off)

namespace bn {

constexpr int kBlock = 256;   // 4 wave64 per workgroup

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b%8).
// Give each XCD a contiguous run of tiles so that the rows a tile shares with
// its neighbours (the stencil halo) are fetched into that XCD's L2 once.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nblocks) {
    const uint32_t per = nblocks >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7u) * per + (b >> 3);
}

// Block-wide sum of the three code counts, then one atomic per non-zero
// counter.  cv/cb/ci are wave-uniform per-wave counts.
__device__ __forceinline__ void flush_counts(bn_frame_stats *stats, uint32_t cv, uint32_t cb,
                                             uint32_t ci) {
    __shared__ uint32_t s_cnt[kBlock / 64][3];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_cnt[wave][0] = cv;
        s_cnt[wave][1] = cb;
        s_cnt[wave][2] = ci;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += s_cnt[w][threadIdx.x];
        if (s) atomicAdd(&stats->n_valid + threadIdx.x, s);
    }
}

__device__ __forceinline__ uint32_t wave_count(bool pred) {
    return (uint32_t)__popcll(__ballot(pred));
}

// ---------------------------------------------------------------------------
// Scalar kernel: one pixel per thread, any row stride and alignment.
// ---------------------------------------------------------------------------
template <int A>
__global__ __launch_bounds__(kBlock) void k_scalar(FrameArgs f) {
    const uint32_t i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const bool live = i < f.nitems;
    uint32_t code = BN_INVALID;
    if (live) {
        const uint32_t y = row_of(i, f.inv_gpr);
        const uint32_t x = i - y * f.gpr;
        const bool inside = (x >= (uint32_t)A) & (x + A < (uint32_t)f.W) &
                            (y >= (uint32_t)A) & (y + A < (uint32_t)f.H);
        const float *p = f.depth + (int64_t)y * f.stride + x;
        float d1 = *p, d2 = 0.f, d3 = 0.f, d4 = 0.f, d5 = 0.f;
        if (inside) {
            d2 = p[A];
            d4 = p[-A];
            d3 = p[(int64_t)A * f.stride];
            d5 = p[-(int64_t)A * f.stride];
        }
        const float xc = (float)x - f.cx;
        const float yc = (float)y - f.cy;
        const PixelOut o = eval_pixel(inside, d1, d2, d3, d4, d5, xc, yc, f);
        float *n = f.normals + 3 * (int64_t)i;
        n[0] = o.nx;
        n[1] = o.ny;
        n[2] = o.nz;
        f.mask[i] = (uint8_t)o.code;
        code = o.code;
    }
    if (f.stats) {
        const uint32_t cv = wave_count(live & (code == BN_VALID));
        const uint32_t cb = wave_count(live & (code == BN_BOUNDARY));
        const uint32_t ci = wave_count(live & (code == BN_INVALID));
        flush_counts(f.stats, cv, cb, ci);
    }
}

// ---------------------------------------------------------------------------
// Vector kernel: four consecutive pixels of a row per thread.
// Requires width % 4 == 0, stride % 4 == 0, 16-byte aligned depth and
// normals and 4-byte aligned mask.  A wave covers 256 pixels of a row
// segment (or of consecutive rows): its three 16-byte normal stores and one
// 4-byte code store write 3 KiB + 256 B of contiguous memory.
// ---------------------------------------------------------------------------
template <int A>
struct Group4 {
    static constexpr int R = (A + 3) / 4;   // float4s needed on each side
    static constexpr int N = 4 * (2 * R + 1);
};

template <int A>
__device__ __forceinline__ void process_group4(const FrameArgs &f, uint32_t y, uint32_t x0,
                                               uint32_t &codes_out) {
    constexpr int R = Group4<A>::R;
    const float *rp = f.depth + (int64_t)y * f.stride;
    float row[Group4<A>::N];
#pragma unroll
    for (int k = -R; k <= R; ++k) {
        const int xs = (int)x0 + 4 * k;
        f4 v = {0.f, 0.f, 0.f, 0.f};
        if (k == 0 || (xs >= 0 && xs < f.W)) v = *reinterpret_cast<const f4 *>(rp + xs);
        row[4 * (k + R) + 0] = v.x;
        row[4 * (k + R) + 1] = v.y;
        row[4 * (k + R) + 2] = v.z;
        row[4 * (k + R) + 3] = v.w;
    }
    const bool rows_in = (y >= (uint32_t)A) & (y + A < (uint32_t)f.H);
    f4 up = {0.f, 0.f, 0.f, 0.f}, dn = {0.f, 0.f, 0.f, 0.f};
    if (rows_in) {
        up = *reinterpret_cast<const f4 *>(rp - (int64_t)A * f.stride + x0);
        dn = *reinterpret_cast<const f4 *>(rp + (int64_t)A * f.stride + x0);
    }
    const float upv[4] = {up.x, up.y, up.z, up.w};
    const float dnv[4] = {dn.x, dn.y, dn.z, dn.w};
    const float yc = (float)y - f.cy;
    float nv[12];
    uint32_t codes = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t x = x0 + j;
        const bool inside = rows_in & (x >= (uint32_t)A) & (x + A < (uint32_t)f.W);
        const float xc = (float)x - f.cx;
        const int c = 4 * R + j;
        const PixelOut o = eval_pixel(inside, row[c], row[c + A], dnv[j], row[c - A], upv[j],
                                      xc, yc, f);
        nv[3 * j + 0] = o.nx;
        nv[3 * j + 1] = o.ny;
        nv[3 * j + 2] = o.nz;
        codes |= o.code << (8 * j);
    }
    const int64_t p = (int64_t)y * f.W + x0;
    f4 *np = reinterpret_cast<f4 *>(f.normals + 3 * p);
    __builtin_nontemporal_store(f4{nv[0], nv[1], nv[2], nv[3]}, np + 0);
    __builtin_nontemporal_store(f4{nv[4], nv[5], nv[6], nv[7]}, np + 1);
    __builtin_nontemporal_store(f4{nv[8], nv[9], nv[10], nv[11]}, np + 2);
    __builtin_nontemporal_store(codes, reinterpret_cast<uint32_t *>(f.mask + p));
    codes_out = codes;
}

// Per-wave counts of the four codes packed in `codes` (one byte each).
__device__ __forceinline__ void count_codes(bool live, uint32_t codes, uint32_t &cv, uint32_t &cb,
                                            uint32_t &ci) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t c = (codes >> (8 * j)) & 0xffu;
        cv += wave_count(live & (c == BN_VALID));
        cb += wave_count(live & (c == BN_BOUNDARY));
        ci += wave_count(live & (c == BN_INVALID));
    }
}

template <int A, int G>
__global__ __launch_bounds__(kBlock) void k_vec4(FrameArgs f) {
    // G groups of 4 pixels per thread, kBlock groups apart (coalesced).
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    uint32_t cv = 0, cb = 0, ci = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t i = (tile * G + g) * kBlock + threadIdx.x;
        const bool live = i < f.nitems;
        uint32_t codes = 0;
        if (live) {
            const uint32_t y = row_of(i, f.inv_gpr);
            const uint32_t x0 = (i - y * f.gpr) * 4;
            process_group4<A>(f, y, x0, codes);
        }
        if (f.stats) count_codes(live, codes, cv, cb, ci);
    }
    if (f.stats) flush_counts(f.stats, cv, cb, ci);
}

// ---------------------------------------------------------------------------
// Launch table
// ---------------------------------------------------------------------------
typedef void (*KernelFn)(FrameArgs);

template <template <int> class K>
struct AlphaTable {
    static KernelFn get(int a) {
        switch (a) {
            case 1: return K<1>::fn;
            case 2: return K<2>::fn;
            case 3: return K<3>::fn;
            case 4: return K<4>::fn;
            case 5: return K<5>::fn;
            case 6: return K<6>::fn;
            case 7: return K<7>::fn;
            case 8: return K<8>::fn;
        }
        return nullptr;
    }
};

template <int A> struct ScalarK { static constexpr KernelFn fn = k_scalar<A>; };
template <int A> struct Vec4G1 { static constexpr KernelFn fn = k_vec4<A, 1>; };
template <int A> struct Vec4G2 { static constexpr KernelFn fn = k_vec4<A, 2>; };
template <int A> struct Vec4G4 { static constexpr KernelFn fn = k_vec4<A, 4>; };

const VariantInfo kVariants[] = {
    {VAR_SCALAR, "scalar", 1, 1},
    {VAR_VEC4, "vec4", 4, 1},
    {VAR_VEC4_G2, "vec4x2", 4, 2},
    {VAR_VEC4_G4, "vec4x4", 4, 4},
};

const VariantInfo *variant_info(int v) {
    for (const auto &vi : kVariants)
        if (vi.id == v) return &vi;
    return nullptr;
}

hipError_t launch_plain(int variant, const FrameArgs &f, hipStream_t stream) {
    const VariantInfo *vi = variant_info(variant);
    if (!vi) return hipErrorInvalidValue;
    KernelFn fn = nullptr;
    switch (variant) {
        case VAR_SCALAR: fn = AlphaTable<ScalarK>::get((int)f.af); break;
        case VAR_VEC4: fn = AlphaTable<Vec4G1>::get((int)f.af); break;
        case VAR_VEC4_G2: fn = AlphaTable<Vec4G2>::get((int)f.af); break;
        case VAR_VEC4_G4: fn = AlphaTable<Vec4G4>::get((int)f.af); break;
    }
    if (!fn) return hipErrorInvalidValue;
    const uint64_t per_block = (uint64_t)kBlock * vi->groups_per_thread;
    const uint64_t nblocks = (f.nitems + per_block - 1) / per_block;
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(kBlock), 0, stream, f);
    return hipGetLastError();
}

}  // namespace bn
