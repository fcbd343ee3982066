// Internal interface between the host side of the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "bn_device.h"

namespace bn {

enum Variant {
    VAR_AUTO = 0,
    VAR_SCALAR = 1,   // one pixel per thread, any layout
    VAR_VEC4 = 2,     // 4 pixels per thread, 16-byte vector loads/stores
    VAR_VEC4_G2 = 3,  // 2 groups of 4 pixels per thread
    VAR_VEC4_G4 = 4,  // 4 groups of 4 pixels per thread
    VAR_VEC4_P2 = 5,  // 2 groups of 4 pixels per thread, second tile's loads ahead
    VAR_VEC4_W128 = 6,  // 4 pixels per thread, workgroups of 128 threads
    VAR_VEC4_W64 = 7,   // 4 pixels per thread, workgroups of 64 threads
    VAR_COUNT = 7
};

struct VariantInfo {
    int id;
    const char *name;
    int px_per_item;        // pixels per work item (1 or 4)
    int groups_per_thread;  // work items per thread
    int block;              // threads per workgroup
};

const VariantInfo *variant_info(int v);

// Argument checks shared by the entry points (bn status codes).
int check_params_args(const bn_params *p);
int check_frame_args(const float *depth, int32_t H, int32_t W, int64_t stride, float fx,
                     float fy, float cx, float cy, const float *normals, const uint8_t *mask);
// A bn_frame_stats pointer: NULL or 4-byte aligned.
int check_stats_arg(const bn_frame_stats *stats);
// The count work areas (BN_MAX_STACK of them) of the current device's
// `stream` (bn_workspace.hip); BN_ERR_UNSUPPORTED beyond BN_MAX_STREAMS
// streams of a device.
int stream_work_areas(hipStream_t stream, WorkArea **out);
// True when the frame can use the 4-pixel vector tiles.
bool vec4_layout(const float *depth, int32_t W, int64_t stride, const float *normals,
                 const uint8_t *mask);
// True when the method can take vector tiles (multi-scale: alpha * scales
// <= kMsVecReach).
bool method_has_vec4(const bn_params *p);
// The plain entry point's tile shape when nothing is tuned for the frame:
// vector tiles where the method and the layout allow them, except four-pair
// frames of at most kSmallFrame pixels, which take the scalar tiles.
constexpr uint64_t kSmallFrame = 1u << 19;
int default_plain_variant(const bn_params *p, uint64_t pixels, bool vec_layout);
// Per-frame kernel arguments (derived constants included); work = NULL (the
// caller sets the count work area when stats is given).
void fill_frame_args(FrameArgs &f, const float *depth, int32_t H, int32_t W, int64_t stride,
                     float fx, float fy, float cx, float cy, const bn_params *p, float *normals,
                     uint8_t *mask, bn_frame_stats *stats, int px_per_item);

// Checked arguments of a stack of n frames (bn_stack.hip); s.n == 0 when
// there is nothing to do.  normals / mask stand for the outputs in the
// checks (the adjoint passes its gradients).
int stack_args(StackArgs &s, const float *depth, int32_t n, int32_t H, int32_t W,
               int64_t stride, int64_t fstride, const bn_intrinsics *intr, const bn_params *p,
               float *normals, uint8_t *mask, bn_frame_stats *stats, int px_per_item);

// True when the plan's current list went to the device through an upload
// on the update's stream (false for small lists, whose descriptors travel in
// the kernel arguments).
bool batch_plan_uploads(const bn_batch_plan *plan);

// Autotuning table (bn_autotune.hip): 0 when nothing is recorded.
int tuned_plain_variant(int method, int alpha, uint64_t pixels);
// batch grid shape as recorded: -1 flat, -2 / -4 flat with 2 / 4 tiles per
// workgroup, k > 0 persistent workgroups per compute unit
int tuned_batch_shape(int method, int alpha, uint64_t pixels);
void record_tuning(int kind, int method, int alpha, uint64_t pixels, int value, float us);

// Launch one frame with the given variant and method.  FrameArgs.gpr /
// nitems / inv_gpr must match the variant's pixels per work item.
hipError_t launch_plain(int variant, int method, const FrameArgs &f, hipStream_t stream);

}  // namespace bn
