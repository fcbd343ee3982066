// Stacks: n frames of one size in one launch, each with its own intrinsics.
//
// Workgroup b (in the XCD-aware numbering) takes tile b % T of frame b / T,
// T = tiles per frame, so a stack is one grid of n * T workgroups: a batch of
// small frames fills the chip where n separate launches would each ramp up
// and drain.  The per-frame values travel in the kernel arguments, so a call
// needs no upload and allocates nothing.  Each tile is exactly the tile of
// the single-frame kernels, and the counts go through the same per-frame
// reduction with the frame's T tiles as its parts.
#include <cmath>
#include <cstring>

#include "bn_device.h"
#include "bn_internal.h"
#include "bn_tiles.h"

#pragma clang fp contract(off)

namespace bn {

template <int A, int M>
__global__ __launch_bounds__(kBlock) void k_stack(const StackArgs s) {
    __shared__ TileLds lds;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t k = b / s.tiles_per_frame;
    const uint32_t tile = b - k * s.tiles_per_frame;
    const FrameArgs f = stack_frame(s, k);
    if (s.vec) {
        vec4_tile_counted<A, M>(f, tile, tile, s.tiles_per_frame, lds);
        return;
    }
    scalar_tile_counted<A, M>(f, tile, tile, s.tiles_per_frame, lds);
}

typedef void (*StackFn)(const StackArgs);

template <int M>
static StackFn stack_kernel_m(int alpha) {
    switch (alpha) {
        case 1: return k_stack<1, M>;
        case 2: return k_stack<2, M>;
        case 3: return k_stack<3, M>;
        case 4: return k_stack<4, M>;
        case 5: return k_stack<5, M>;
        case 6: return k_stack<6, M>;
        case 7: return k_stack<7, M>;
        case 8: return k_stack<8, M>;
    }
    return nullptr;
}

static StackFn stack_kernel(int method, int alpha, int scales, bool vec) {
    if (method == kFourPair) return stack_kernel_m<kFourPair>(alpha);
    if (method == kPairRemoval) return stack_kernel_m<kPairRemoval>(alpha);
    // multi-scale scalar tiles take the offsets at run time
    if (method == kMultiScale && !vec) return k_stack<1, kMultiScale>;
    if (kernel_method(method, alpha, scales) == kMultiScaleLong)
        return stack_kernel_m<kMultiScaleLong>(alpha);
    if (method == kMultiScale) return stack_kernel_m<kMultiScale>(alpha);
    return nullptr;
}

int stack_args(StackArgs &s, const float *depth, int32_t n, int32_t H, int32_t W,
               int64_t stride, int64_t fstride, const bn_intrinsics *intr, const bn_params *p,
               float *normals, uint8_t *mask, bn_frame_stats *stats, int px_per_item) {
    std::memset(&s, 0, sizeof(s));
    if (n < 0 || (n > 0 && !intr)) return BN_ERR_INVALID_ARG;
    if (n > BN_MAX_STACK) return BN_ERR_UNSUPPORTED;
    for (int32_t k = 0; k < n; ++k) {
        const bn_intrinsics &c = intr[k];
        const int rc = check_frame_args(depth, H, W, stride, c.fx, c.fy, c.cx, c.cy, normals,
                                        mask);
        if (rc != BN_OK) return rc;
    }
    if (n > 1 && H > 0 && W > 0 && fstride < (int64_t)H * stride) return BN_ERR_INVALID_ARG;
    if (fstride < 0) return BN_ERR_INVALID_ARG;
    if (fstride > ((int64_t)1 << 40)) return BN_ERR_UNSUPPORTED;
    if (n == 0 || H == 0 || W == 0) return BN_OK;
    fill_frame_args(s.f, depth, H, W, stride, intr[0].fx, intr[0].fy, intr[0].cx, intr[0].cy, p,
                    normals, mask, stats, px_per_item);
    for (int32_t k = 0; k < n; ++k) {
        FrameArgs fk;
        fill_frame_args(fk, depth, H, W, stride, intr[k].fx, intr[k].fy, intr[k].cx, intr[k].cy,
                        p, normals, mask, stats, px_per_item);
        s.fr[k] = StackFrame{fk.fx, fk.fy, fk.cx, fk.cy, fk.hconst};
    }
    s.depth_fstride = fstride;
    s.n = (uint32_t)n;
    return BN_OK;
}

}  // namespace bn

using namespace bn;

extern "C" int bn_estimate_normals_stack(const float *depth, int32_t n, int32_t height,
                                         int32_t width, int64_t depth_stride,
                                         int64_t depth_frame_stride,
                                         const bn_intrinsics *intrinsics,
                                         const bn_params *params, float *normals, uint8_t *mask,
                                         bn_frame_stats *stats, void *stream) {
    int rc = check_params_args(params);
    if (rc != BN_OK) return rc;
    rc = check_stats_arg(stats);
    if (rc != BN_OK) return rc;
    const int v = (int)params->variant;
    if (v != VAR_AUTO && v != VAR_SCALAR && v != VAR_VEC4) {
        return variant_info(v) ? BN_ERR_UNSUPPORTED : BN_ERR_INVALID_ARG;
    }
    StackArgs s;
    rc = stack_args(s, depth, n, height, width, depth_stride, depth_frame_stride, intrinsics,
                    params, normals, mask, stats, 1);
    if (rc != BN_OK || s.n == 0) return rc;
    const bool vec_ok = method_has_vec4(params) && (n == 1 || depth_frame_stride % 4 == 0) &&
                        vec4_layout(depth, width, depth_stride, normals, mask);
    if (v == VAR_VEC4 && !vec_ok) return BN_ERR_UNSUPPORTED;
    const bool vec = v == VAR_VEC4 || (v == VAR_AUTO && vec_ok);
    if (vec) {
        rc = stack_args(s, depth, n, height, width, depth_stride, depth_frame_stride, intrinsics,
                        params, normals, mask, stats, 4);
        if (rc != BN_OK) return rc;
    }
    StackFn fn = stack_kernel(params->method, params->alpha, params->scales, vec);
    if (!fn) return BN_ERR_UNSUPPORTED;
    if (stats) {
        rc = stream_work_areas((hipStream_t)stream, &s.f.work);
        if (rc != BN_OK) return rc;
    }
    s.vec = vec ? 1u : 0u;
    s.tiles_per_frame = (s.f.nitems + kBlock - 1) / kBlock;
    const uint64_t grid = (uint64_t)s.tiles_per_frame * s.n;
    hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kBlock), 0, (hipStream_t)stream, s);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}
