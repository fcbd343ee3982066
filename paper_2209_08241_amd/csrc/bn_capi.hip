// Host side of the C ABI declared in include/bnormals.h: argument
// validation (before any launch), per-frame constants, variant choice and
// launch on the caller's stream.
#include <cfloat>
#include <cmath>
#include <cstdint>

#include "bn_internal.h"
#include "bnormals.h"

#pragma clang fp contract(off)

using namespace bn;

namespace bn {

static bool finite(float v) { return std::isfinite(v); }

int check_params_args(const bn_params *p) {
    if (!p) return BN_ERR_INVALID_ARG;
    if (p->alpha < 1) return BN_ERR_INVALID_ARG;
    if (p->alpha > BN_MAX_ALPHA) return BN_ERR_UNSUPPORTED;
    if (p->mask_mode != BN_MASK_REL && p->mask_mode != BN_MASK_ABS &&
        p->mask_mode != BN_MASK_NONE)
        return BN_ERR_INVALID_ARG;
    if (p->mask_mode != BN_MASK_NONE && !(finite(p->tau) && p->tau > 0.0f))
        return BN_ERR_INVALID_ARG;
    if (p->variant > (uint32_t)VAR_COUNT) return BN_ERR_INVALID_ARG;
    if (p->method == BN_METHOD_FOUR_PAIR || p->method == BN_METHOD_PAIR_REMOVAL) {
        if (p->scales != 0 && p->scales != 1) return BN_ERR_INVALID_ARG;
    } else if (p->method == BN_METHOD_MULTISCALE) {
        if (p->scales < 1) return BN_ERR_INVALID_ARG;
        if (p->scales > BN_MAX_SCALES) return BN_ERR_UNSUPPORTED;
    } else {
        return BN_ERR_INVALID_ARG;
    }
    if ((p->flags & ~BN_FLAG_COUNTS_ACCUMULATE) != 0u || p->reserved != 0u)
        return BN_ERR_INVALID_ARG;
    return BN_OK;
}

bool method_has_vec4(const bn_params *p) {
    return p->method != BN_METHOD_MULTISCALE || p->alpha * p->scales <= kMsVecReach;
}

// A small frame has few tiles: at 1024 pixels a tile, a 640x480 frame is
// 1200 wavefronts, about one per SIMD, and its launch is one chain of
// latencies; at one pixel a thread it is 4800 wavefronts whose latencies
// overlap.  Four-pair, graph-replayed: 320x240 3.19 against 3.60-3.81 us,
// 640x480 3.77 against 4.25-4.37 us for the vector shapes; 1280x720 the
// same within 1.5%; 1920x1080 9.2 against 7.5 us.
int default_plain_variant(const bn_params *p, uint64_t pixels, bool vec_layout) {
    if (!vec_layout || !method_has_vec4(p)) return VAR_SCALAR;
    if (p->method == BN_METHOD_FOUR_PAIR && pixels <= kSmallFrame) return VAR_SCALAR;
    return VAR_VEC4;
}

int check_frame_args(const float *depth, int32_t H, int32_t W, int64_t stride, float fx,
                     float fy, float cx, float cy, const float *normals, const uint8_t *mask) {
    if (H < 0 || W < 0) return BN_ERR_INVALID_ARG;
    if (W > BN_MAX_WIDTH) return BN_ERR_UNSUPPORTED;
    if ((int64_t)H * (int64_t)W > BN_MAX_PIXELS) return BN_ERR_UNSUPPORTED;
    if (!(finite(fx) && fx > 0.0f) || !(finite(fy) && fy > 0.0f)) return BN_ERR_INVALID_ARG;
    if (!finite(cx) || !finite(cy)) return BN_ERR_INVALID_ARG;
    if (H == 0 || W == 0) return BN_OK;
    if (stride < W) return BN_ERR_INVALID_ARG;
    if (stride > (int64_t)1 << 40) return BN_ERR_UNSUPPORTED;
    if (!depth || !normals || !mask) return BN_ERR_INVALID_ARG;
    if ((uintptr_t)depth % 4 || (uintptr_t)normals % 4) return BN_ERR_INVALID_ARG;
    return BN_OK;
}

int check_stats_arg(const bn_frame_stats *stats) {
    return ((uintptr_t)stats % 4) ? BN_ERR_INVALID_ARG : BN_OK;
}

static bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

bool vec4_layout(const float *depth, int32_t W, int64_t stride, const float *normals,
                 const uint8_t *mask) {
    return (W % 4 == 0) && (stride % 4 == 0) && aligned(depth, 16) && aligned(normals, 16) &&
           aligned(mask, 4);
}

static bool variant_ok(int v, const float *depth, int32_t W, int64_t stride,
                       const float *normals, const uint8_t *mask) {
    const VariantInfo *vi = variant_info(v);
    if (!vi) return false;
    if (vi->px_per_item == 4) return vec4_layout(depth, W, stride, normals, mask);
    return true;
}

static bool method_variant_ok(const bn_params *p, int v, const float *depth, int32_t W,
                              int64_t stride, const float *normals, const uint8_t *mask) {
    const VariantInfo *vi = variant_info(v);
    if (!vi) return false;
    if (vi->px_per_item == 4 && !method_has_vec4(p)) return false;
    // the pipelined pair of tiles and the small workgroups serve the
    // five-tap methods
    if ((v == VAR_VEC4_P2 || v == VAR_VEC4_W128 || v == VAR_VEC4_W64) &&
        p->method == BN_METHOD_MULTISCALE)
        return false;
    return variant_ok(v, depth, W, stride, normals, mask);
}

// The ABS test on the method's binary32 |m|^2 scale, computed in double in
// this order and rounded once:
//   four-pair    r = |n|   = alpha |m| / (4 fx fy)  ->  ((((4 fx) fy) tau) / alpha)^2
//   pair removal r = |n_p| = alpha |m_p| / (fx fy)  ->  (((fx fy) tau) / alpha)^2
//   multi-scale  r = |avg| = |M| / (K fx fy)        ->  (((K fx) fy) tau)^2
static float abs_threshold(int method, int scales, float fx, float fy, float tau, int alpha) {
    double k;
    if (method == BN_METHOD_PAIR_REMOVAL) {
        k = (double)fx;
        k = k * (double)fy;
        k = k * (double)tau;
        k = k / (double)alpha;
    } else if (method == BN_METHOD_MULTISCALE) {
        k = (double)scales;
        k = k * (double)fx;
        k = k * (double)fy;
        k = k * (double)tau;
    } else {
        k = 4.0 * (double)fx;
        k = k * (double)fy;
        k = k * (double)tau;
        k = k / (double)alpha;
    }
    k = k * k;
    return (float)k;
}

static int pick_variant(const float *depth, int32_t H, int32_t W, int64_t stride,
                        const float *normals, const uint8_t *mask, const bn_params *p) {
    const int tuned = tuned_plain_variant(p->method, p->alpha, (uint64_t)H * (uint64_t)W);
    if (tuned > 0 && method_variant_ok(p, tuned, depth, W, stride, normals, mask)) return tuned;
    return default_plain_variant(p, (uint64_t)H * (uint64_t)W,
                                 vec4_layout(depth, W, stride, normals, mask));
}

void fill_frame_args(FrameArgs &f, const float *depth, int32_t H, int32_t W, int64_t stride,
                     float fx, float fy, float cx, float cy, const bn_params *p, float *normals,
                     uint8_t *mask, bn_frame_stats *stats, int px_per_item) {
    f.depth = depth;
    f.normals = normals;
    f.mask = mask;
    f.stats = stats;
    f.work = nullptr;
    f.stride = stride;
    f.H = H;
    f.W = W;
    f.fx = fx;
    f.fy = fy;
    f.cx = cx;
    f.cy = cy;
    f.af = (float)p->alpha;
    f.rel = p->mask_mode == BN_MASK_REL ? 1 : 0;
    f.tt = p->tau * p->tau;
    f.hconst = p->mask_mode == BN_MASK_ABS
                   ? abs_threshold(p->method, p->scales, fx, fy, p->tau, p->alpha)
                   : INFINITY;
    f.gpr = (uint32_t)(W / px_per_item);
    f.nitems = f.gpr * (uint32_t)H;
    f.npix = (uint32_t)H * (uint32_t)W;
    f.alpha = p->alpha;
    f.scales = p->method == BN_METHOD_MULTISCALE ? p->scales : 1;
    f.overwrite = (p->flags & BN_FLAG_COUNTS_ACCUMULATE) ? 0u : 1u;
    f.inv_gpr = 1.0 / (double)f.gpr;
}

}  // namespace bn

extern "C" {

int bn_estimate_normals(const float *depth, int32_t height, int32_t width, int64_t depth_stride,
                        float fx, float fy, float cx, float cy, const bn_params *params,
                        float *normals, uint8_t *mask, bn_frame_stats *stats, void *stream) {
    int rc = check_params_args(params);
    if (rc != BN_OK) return rc;
    rc = check_frame_args(depth, height, width, depth_stride, fx, fy, cx, cy, normals, mask);
    if (rc != BN_OK) return rc;
    rc = check_stats_arg(stats);
    if (rc != BN_OK) return rc;
    if (height == 0 || width == 0) return BN_OK;
    int v = (int)params->variant;
    if (v == VAR_AUTO) {
        v = pick_variant(depth, height, width, depth_stride, normals, mask, params);
    } else if (!method_variant_ok(params, v, depth, width, depth_stride, normals, mask)) {
        return BN_ERR_UNSUPPORTED;
    }
    FrameArgs f;
    fill_frame_args(f, depth, height, width, depth_stride, fx, fy, cx, cy, params, normals, mask,
                    stats, variant_info(v)->px_per_item);
    if (stats) {
        rc = stream_work_areas((hipStream_t)stream, &f.work);
        if (rc != BN_OK) return rc;
    }
    hipError_t e = launch_plain(v, params->method, f, (hipStream_t)stream);
    return e == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

int bn_variant_count(void) { return VAR_COUNT; }

const char *bn_variant_name(int variant) {
    const VariantInfo *vi = variant_info(variant);
    return vi ? vi->name : nullptr;
}

int bn_variant_supported(int variant, const float *depth, int32_t height, int32_t width,
                         int64_t depth_stride, const float *normals, const uint8_t *mask) {
    (void)height;
    return variant_ok(variant, depth, width, depth_stride, normals, mask) ? 1 : 0;
}

const char *bn_status_string(int status) {
    switch (status) {
        case BN_OK: return "ok";
        case BN_ERR_INVALID_ARG: return "invalid argument";
        case BN_ERR_UNSUPPORTED: return "unsupported argument";
        case BN_ERR_DEVICE: return "device error";
        case BN_ERR_OOM: return "out of device memory";
        case BN_ERR_TIMEOUT: return "timed out";
    }
    return "unknown status";
}

int bn_version(void) { return BN_VERSION; }

}  // extern "C"
