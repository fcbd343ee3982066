// Plain (one frame per launch) kernels for gfx950.
//
// The estimator is a memory-bound 5-point stencil: 4 bytes of depth in,
// 12 bytes of normal and 1 byte of code out per pixel, about 40 binary32
// operations in between.  The kernels therefore aim at full-width coalesced
// HBM traffic:
//   * a workgroup owns a run of consecutive pixels; the normals it computes
//     go through LDS so that every global store instruction of a wavefront
//     writes one contiguous KiB (interleaved 12-byte records stored straight
//     from registers would scatter each instruction over 3 KiB);
//   * depth is read with 16-byte loads; the horizontal taps come from the
//     neighbouring lanes through DPP wave shifts, the vertical taps from the
//     rows alpha above and below, which the workgroups of the same XCD read
//     as their own rows (L2 hits);
//   * per-frame counts are reduced in registers (wavefront ballots), in LDS,
//     then across the grid with one packed atomic per workgroup.
#include "bn_device.h"
#include "bn_internal.h"

#pragma clang fp contract(off)

namespace bn {

// ---------------------------------------------------------------------------
// Scalar kernel: one pixel per thread, any row stride and alignment.
// ---------------------------------------------------------------------------
template <int A>
__global__ __launch_bounds__(kBlock) void k_scalar(FrameArgs f) {
    __shared__ float s_out[3 * kBlock];
    const uint32_t blk = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t base = blk * kBlock;
    const uint32_t i = base + threadIdx.x;
    const bool live = i < f.nitems;
    uint32_t code = BN_INVALID;
    float nx = 0.f, ny = 0.f, nz = 0.f;
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
        nx = o.nx;
        ny = o.ny;
        nz = o.nz;
        code = o.code;
        f.mask[i] = (uint8_t)code;
    }
    s_out[3 * threadIdx.x + 0] = nx;
    s_out[3 * threadIdx.x + 1] = ny;
    s_out[3 * threadIdx.x + 2] = nz;
    __syncthreads();
    const uint32_t n = min((uint32_t)kBlock, f.nitems - base) * 3u;
    float *out = f.normals + 3 * (int64_t)base;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint32_t j = k * kBlock + threadIdx.x;
        if (j < n) out[j] = s_out[j];
    }
    if (f.stats) {
        const uint32_t cv = wave_count(live & (code == BN_VALID));
        const uint32_t cb = wave_count(live & (code == BN_BOUNDARY));
        block_counts(f.stats, blk, gridDim.x, cv, cb, f.npix);
    }
}

// ---------------------------------------------------------------------------
// Vector kernel: four consecutive pixels of a row per thread, 256 groups
// (1024 pixels) per tile, G tiles per workgroup.  Requires width % 4 == 0,
// stride % 4 == 0, 16-byte aligned depth and normals, 4-byte aligned mask.
// ---------------------------------------------------------------------------
template <int A>
struct Win {
    static constexpr int R = (A + 3) / 4;  // float4s needed on each side
    static constexpr int N = 4 * (2 * R + 1);
};

// Evaluate the group of thread threadIdx.x in `tile`: its 12 normal floats
// go to s_out[3t .. 3t+2], its four codes to the mask (one 32-bit store) and
// are returned packed one per byte.
template <int A>
__device__ __forceinline__ uint32_t vec4_group(const FrameArgs &f, uint32_t tile, f4 *s_out,
                                               bool &live) {
    constexpr int R = Win<A>::R;
    const uint32_t t = threadIdx.x;
    const uint32_t lane = t & 63u;
    const uint32_t i = tile * kBlock + t;
    live = i < f.nitems;
    uint32_t y = 0, x0 = 0;
    if (live) {
        y = row_of(i, f.inv_gpr);
        x0 = (i - y * f.gpr) * 4u;
    }
    const float *rp = f.depth + (int64_t)y * f.stride;
    const bool rows_in = live & (y >= (uint32_t)A) & (y + A < (uint32_t)f.H);
    f4 c = {0.f, 0.f, 0.f, 0.f}, up = {0.f, 0.f, 0.f, 0.f}, dn = {0.f, 0.f, 0.f, 0.f};
    if (live) c = *reinterpret_cast<const f4 *>(rp + x0);
    if (rows_in) {
        up = *reinterpret_cast<const f4 *>(rp - (int64_t)A * f.stride + x0);
        dn = *reinterpret_cast<const f4 *>(rp + (int64_t)A * f.stride + x0);
    }
    // row window x0-4R .. x0+4+4R-1; neighbours from adjacent lanes, the
    // first / last lane of the wave loads its missing float4 itself.  Values
    // taken across a row end only feed border pixels, which are INVALID.
    float row[Win<A>::N];
    row[4 * R + 0] = c.x;
    row[4 * R + 1] = c.y;
    row[4 * R + 2] = c.z;
    row[4 * R + 3] = c.w;
    f4 lk = c, rk = c;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lk = from_left(lk);
        rk = from_right(rk);
        if (lane == 0) {
            const int xs = (int)x0 - 4 * k;
            lk = (live && xs >= 0) ? *reinterpret_cast<const f4 *>(rp + xs) : f4{0.f, 0.f, 0.f, 0.f};
        }
        if (lane == 63) {
            const int xs = (int)x0 + 4 * k;
            rk = (live && xs < f.W) ? *reinterpret_cast<const f4 *>(rp + xs) : f4{0.f, 0.f, 0.f, 0.f};
        }
        row[4 * (R - k) + 0] = lk.x;
        row[4 * (R - k) + 1] = lk.y;
        row[4 * (R - k) + 2] = lk.z;
        row[4 * (R - k) + 3] = lk.w;
        row[4 * (R + k) + 0] = rk.x;
        row[4 * (R + k) + 1] = rk.y;
        row[4 * (R + k) + 2] = rk.z;
        row[4 * (R + k) + 3] = rk.w;
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
        const int cI = 4 * R + j;
        const PixelOut o = eval_pixel(inside, row[cI], row[cI + A], dnv[j], row[cI - A], upv[j],
                                      xc, yc, f);
        nv[3 * j + 0] = o.nx;
        nv[3 * j + 1] = o.ny;
        nv[3 * j + 2] = o.nz;
        codes |= o.code << (8 * j);
    }
    s_out[3 * t + 0] = f4{nv[0], nv[1], nv[2], nv[3]};
    s_out[3 * t + 1] = f4{nv[4], nv[5], nv[6], nv[7]};
    s_out[3 * t + 2] = f4{nv[8], nv[9], nv[10], nv[11]};
    if (live) __builtin_nontemporal_store(codes, reinterpret_cast<uint32_t *>(f.mask) + i);
    return codes;
}

// Contiguous store of the tile's normals from LDS: 12 floats per group.
__device__ __forceinline__ void store_tile_normals(const FrameArgs &f, uint32_t tile,
                                                   const f4 *s_out) {
    const uint32_t ngr = min((uint32_t)kBlock, f.nitems - tile * kBlock);
    f4 *out = reinterpret_cast<f4 *>(f.normals) + 3 * (int64_t)tile * kBlock;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint32_t j = k * kBlock + threadIdx.x;
        if (j < 3 * ngr) __builtin_nontemporal_store(s_out[j], out + j);
    }
}

__device__ __forceinline__ void count_codes(bool live, uint32_t codes, uint32_t &cv,
                                            uint32_t &cb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t c = (codes >> (8 * j)) & 0xffu;
        cv += wave_count(live & (c == BN_VALID));
        cb += wave_count(live & (c == BN_BOUNDARY));
    }
}

template <int A, int G>
__global__ __launch_bounds__(kBlock) void k_vec4(FrameArgs f) {
    __shared__ f4 s_out[3 * kBlock];
    const uint32_t blk = xcd_tile(blockIdx.x, gridDim.x);
    uint32_t cv = 0, cb = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t tile = blk * G + g;
        if (tile * kBlock >= f.nitems) break;  // uniform over the workgroup
        if (g > 0) __syncthreads();             // LDS reuse
        bool live;
        const uint32_t codes = vec4_group<A>(f, tile, s_out, live);
        if (f.stats) count_codes(live, codes, cv, cb);
        __syncthreads();
        store_tile_normals(f, tile, s_out);
    }
    if (f.stats) block_counts(f.stats, blk, gridDim.x, cv, cb, f.npix);
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
