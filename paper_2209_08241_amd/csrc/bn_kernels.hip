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
#include "bn_tiles.h"

#pragma clang fp contract(off)

namespace bn {

// Scalar kernel: one pixel per thread, any row stride and alignment; one
// tile per workgroup.  M: the method (the multi-scale one ignores A).
template <int A, int M>
__global__ __launch_bounds__(kBlock) void k_scalar(FrameArgs f) {
    __shared__ TileLds lds;
    const uint32_t blk = xcd_tile(blockIdx.x, gridDim.x);
    scalar_tile_counted<A, M>(f, blk, blockIdx.x, gridDim.x, lds);
}

// Vector kernel: four consecutive pixels of a row per thread, G tiles of
// 1024 pixels per workgroup.  Requires width % 4 == 0, stride % 4 == 0,
// 16-byte aligned depth and normals, 4-byte aligned mask.
template <int A, int G, int M>
__global__ __launch_bounds__(kBlock) void k_vec4(FrameArgs f) {
    __shared__ TileLds lds;
    const uint32_t blk = xcd_tile(blockIdx.x, gridDim.x);
    uint32_t cv = 0, cb = 0;
    if (G == 1) {
        vec4_tile_counted<A, M>(f, blk, blockIdx.x, gridDim.x, lds);
        return;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t tile = blk * G + g;
        if (tile * kBlock >= f.nitems) break;  // uniform over the workgroup
        run_tile<A, M>(f, true, tile, lds, cv, cb);
    }
    if (f.stats) block_counts(f, blockIdx.x, gridDim.x, cv, cb);
}

// Vector kernel, two tiles per workgroup, software-pipelined (the second
// tile's loads in flight during the first tile's arithmetic and stores); the
// five-tap methods only.
template <int A, int M>
__global__ __launch_bounds__(kBlock) void k_vec4p(FrameArgs f) {
    __shared__ TileLds lds;
    const uint32_t blk = xcd_tile(blockIdx.x, gridDim.x);
    vec4_tile_pair_counted<A, M>(f, 2 * blk, 2 * blk + 1, blockIdx.x, gridDim.x, lds);
}

// Vector kernel with workgroups of TB = 64 or 128 threads (tiles of 256 or
// 512 pixels): more, smaller workgroups for small frames; the five-tap
// methods only.
template <int A, int M, int TB>
__global__ __launch_bounds__(TB) void k_vec4w(FrameArgs f) {
    __shared__ TileLdsT<TB> lds;
    const uint32_t blk = xcd_tile(blockIdx.x, gridDim.x);
    vec4_tile_counted<A, M, TB>(f, blk, blockIdx.x, gridDim.x, lds);
}

// ---------------------------------------------------------------------------
// Launch table
// ---------------------------------------------------------------------------
typedef void (*KernelFn)(FrameArgs);

template <template <int, int> class K, int M>
struct AlphaTable {
    static KernelFn get(int a) {
        switch (a) {
            case 1: return K<1, M>::fn;
            case 2: return K<2, M>::fn;
            case 3: return K<3, M>::fn;
            case 4: return K<4, M>::fn;
            case 5: return K<5, M>::fn;
            case 6: return K<6, M>::fn;
            case 7: return K<7, M>::fn;
            case 8: return K<8, M>::fn;
        }
        return nullptr;
    }
};

template <int A, int M> struct ScalarK { static constexpr KernelFn fn = k_scalar<A, M>; };
template <int A, int M> struct Vec4G1 { static constexpr KernelFn fn = k_vec4<A, 1, M>; };
template <int A, int M> struct Vec4G2 { static constexpr KernelFn fn = k_vec4<A, 2, M>; };
template <int A, int M> struct Vec4G4 { static constexpr KernelFn fn = k_vec4<A, 4, M>; };
template <int A, int M> struct Vec4P2 { static constexpr KernelFn fn = k_vec4p<A, M>; };
template <int A, int M> struct Vec4W128 { static constexpr KernelFn fn = k_vec4w<A, M, 128>; };
template <int A, int M> struct Vec4W64 { static constexpr KernelFn fn = k_vec4w<A, M, 64>; };

template <int M>
static KernelFn plain_kernel(int variant, int alpha) {
    switch (variant) {
        case VAR_SCALAR: return AlphaTable<ScalarK, M>::get(alpha);
        case VAR_VEC4: return AlphaTable<Vec4G1, M>::get(alpha);
        case VAR_VEC4_G2: return AlphaTable<Vec4G2, M>::get(alpha);
        case VAR_VEC4_G4: return AlphaTable<Vec4G4, M>::get(alpha);
        case VAR_VEC4_P2:
            if constexpr (!is_multiscale(M)) return AlphaTable<Vec4P2, M>::get(alpha);
            return nullptr;
        case VAR_VEC4_W128:
            if constexpr (!is_multiscale(M)) return AlphaTable<Vec4W128, M>::get(alpha);
            return nullptr;
        case VAR_VEC4_W64:
            if constexpr (!is_multiscale(M)) return AlphaTable<Vec4W64, M>::get(alpha);
            return nullptr;
    }
    return nullptr;
}

const VariantInfo kVariants[] = {
    {VAR_SCALAR, "scalar", 1, 1, kBlock},
    {VAR_VEC4, "vec4", 4, 1, kBlock},
    {VAR_VEC4_G2, "vec4x2", 4, 2, kBlock},
    {VAR_VEC4_G4, "vec4x4", 4, 4, kBlock},
    {VAR_VEC4_P2, "vec4p2", 4, 2, kBlock},
    {VAR_VEC4_W128, "vec4w128", 4, 1, 128},
    {VAR_VEC4_W64, "vec4w64", 4, 1, 64},
};

const VariantInfo *variant_info(int v) {
    for (const auto &vi : kVariants)
        if (vi.id == v) return &vi;
    return nullptr;
}

hipError_t launch_plain(int variant, int method, const FrameArgs &f, hipStream_t stream) {
    const VariantInfo *vi = variant_info(variant);
    if (!vi) return hipErrorInvalidValue;
    KernelFn fn = nullptr;
    if (method == kFourPair) {
        fn = plain_kernel<kFourPair>(variant, f.alpha);
    } else if (method == kPairRemoval) {
        fn = plain_kernel<kPairRemoval>(variant, f.alpha);
    } else if (method == kMultiScale) {
        // scalar tiles take any offsets at run time; vector tiles serve
        // alpha * scales <= kMsVecReach, in two instantiations
        fn = variant == VAR_SCALAR ? k_scalar<1, kMultiScale>
             : kernel_method(method, f.alpha, f.scales) == kMultiScaleLong
                 ? plain_kernel<kMultiScaleLong>(variant, f.alpha)
                 : plain_kernel<kMultiScale>(variant, f.alpha);
    }
    if (!fn) return hipErrorInvalidValue;
    const uint64_t per_block = (uint64_t)vi->block * vi->groups_per_thread;
    const uint64_t nblocks = (f.nitems + per_block - 1) / per_block;
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(vi->block), 0, stream, f);
    return hipGetLastError();
}

}  // namespace bn
