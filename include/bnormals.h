/*
 * bnormals.h -- C ABI of the MI355X (gfx950) boundary-aware surface-normal
 * library.
 *
 * Method: Moradi, Memarmoghadam, Laurendeau, "Fast, Accurate and Object
 * Boundary-Aware Surface Normal Estimation from Depth Maps".
 *   - Per pixel, the average of the normals of the four perpendicular
 *     tangent pairs around the pixel (Section 3.1, Eq. 7), evaluated in the
 *     paper's reformulated single-cross-product form 0.25 s24 x s35
 *     (Eqs. 8-12).  Stencil at pixel distance alpha: tap 2 = (x+alpha, y),
 *     3 = (x, y+alpha), 4 = (x-alpha, y), 5 = (x, y-alpha), x the column,
 *     y the row; u = (x - cx)/fx, v = (y - cy)/fy; depth is z-depth.
 *   - Boundary test (Section 3.2, Eq. 13): the length r = |n| grows with
 *     the tangent lengths, so pixels whose r exceeds a threshold are
 *     masked out of the normal map.
 *
 * Output per pixel: a code (BN_VALID, BN_BOUNDARY, BN_INVALID) and a normal
 * that is the camera-facing unit vector -n/|n| when the code is BN_VALID and
 * (0, 0, 0) otherwise.
 *
 * Methods (bn_params.method):
 *   BN_METHOD_FOUR_PAIR (default) the paper's estimator as above: the
 *       four-pair average, the whole pixel removed by the test.
 *   BN_METHOD_PAIR_REMOVAL each of the four perpendicular-pair normals that
 *       Eq. 7 averages, n23 = s12 x s13, n34, n45, n52, is tested on its
 *       own; the normal is the average of the pairs that pass, and the pixel
 *       is BOUNDARY only when none passes.  Only the tangent pairs that
 *       cross a depth discontinuity are dropped.  With all four passing, the
 *       result is the four-pair one.
 *   BN_METHOD_MULTISCALE the authors' earlier single-pair estimator
 *       (Section 2, Eqs. 1-3: the pair (2, 3) only) at offsets alpha_i =
 *       i*alpha, i = 1..scales, averaged over i as in Eqs. 4-6, with the
 *       test on the average.  Reads (x + alpha_i, y) and (x, y + alpha_i).
 *
 * Codes:
 *   BN_INVALID  the stencil leaves the image (four-pair and pair removal:
 *               a border of alpha on every side; multi-scale: scales*alpha
 *               on the right and bottom); or a tap read is not a finite
 *               depth > 0 (holes are 0); or a binary32 squared length below
 *               is not a finite number >= FLT_MIN.
 *   BN_BOUNDARY otherwise, when the threshold test fires (pair removal:
 *               for all four pairs);
 *   BN_VALID    otherwise.
 *
 * The four-pair threshold test is decided in IEEE binary32, with this exact
 * order of operations (no fused multiply-add), on m = -(4 fx fy / alpha) n:
 *     P=d2-d4  S=d2+d4  Q=d3-d5  T=d3+d5   a=T*P  b=S*Q  c=S*T
 *     mx=fx*a  my=fy*b  xc=(float)x-cx  yc=(float)y-cy
 *     t3=(xc*a)+(yc*b)  w=(float)alpha*c  mz=t3+w
 *     q=((mx*mx)+(my*my))+(mz*mz)
 *   BN_MASK_REL : fires iff q > (tau*tau)*(w*w)    i.e. r/(n.(u,v,1)) > tau
 *   BN_MASK_ABS : fires iff q > K,  K = (float)((4 fx fy tau / alpha)^2)
 *                 evaluated in double as ((((4*fx)*fy)*tau)/alpha)^2;
 *                 i.e. r = |n| > tau, tau in squared depth units
 *   BN_MASK_NONE: never fires.
 * so the mask is reproducible bit for bit by any IEEE binary32 evaluation
 * of the same sequence.  The normal itself is (mx, my, -mz)/sqrt(q) in
 * binary32 (within 1e-5 per component of the FP64 value for intrinsics of
 * ordinary cameras, |x - cx|/fx and |y - cy|/fy up to about 2).
 *
 * Pair removal, per pair p in Eq. 7's order (h, v) = (2,3), (4,3), (4,5),
 * (2,5), with directions (sh, sv) = (+,+), (-,+), (-,-), (+,-):
 *     eh=dh-d1  ev=dv-d1  A=eh*dv  B=dh*ev  (negated where sh, sv is -)
 *     w=((float)alpha*dh)*dv   mx=fx*A  my=fy*B
 *     mz=fma(xc, A, fma(yc, B, w))   q=fma(mx, mx, fma(my, my, mz*mz))
 *   (m_p = -(fx fy / alpha) n_p; each fma is one IEEE fused multiply-add,
 *   rounded once).  Any pair's q not a finite number >= FLT_MIN: INVALID.
 *   REL fires for the pair iff q > ((tau*tau)*w)*w; ABS iff
 *   q > (float)(((fx*fy)*tau)/alpha)^2 (double), i.e. |n_p| > tau.  The
 *   passing pairs' mx, my, mz are summed in pair order from +0 (sx, sy,
 *   sz); Q=fma(sx, sx, fma(sy, sy, sz*sz)) not a finite number >= FLT_MIN:
 *   INVALID.  Normal (sx, sy, -sz)/sqrt(Q).  When all four pairs pass, the
 *   sum is the four-pair m (Eq. 7) and is taken in its closed form instead,
 *   in which d1 cancels exactly rather than through rounded sums: (sx, sy)
 *   = (mx, my) of the four-pair sequence, sz = fma(xc, a, fma(yc, b, w))
 *   with its a, b, w, and Q as above.
 * Multi-scale: for i = 1..K, a=(float)(i*alpha), taps d2 = (x+i*alpha, y),
 *   d3 = (x, y+i*alpha): e2=d2-d1 e3=d3-d1 A=e2*d3 B=d2*e3 C=d2*d3, then
 *   mx, my, w=a*C and mz as for one pair of pair removal; Mx=fma(a, mx, Mx)
 *   and likewise My, Mz, Wt with my, mz, w (from +0, in scale order);
 *   q=fma(Mx, Mx, fma(My, My, Mz*Mz)).  REL
 *   fires iff q > (tau*tau)*(Wt*Wt); ABS iff q > (float)((((K*fx)*fy)*tau)^2)
 *   (double), i.e. |average of Eqs. 4-6| > tau.  Normal (Mx, My, -Mz)/sqrt(q).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer (HBM of the current HIP
 *     device) unless its name ends in _host.  The caller owns all buffers;
 *     the plain entry point allocates nothing.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream; results are visible after the
 *     caller synchronises it.
 *   - Argument errors return synchronously, before any launch, and nothing
 *     is written.  A launch failure returns BN_ERR_DEVICE.  Faults inside a
 *     kernel surface at the caller's next synchronisation.
 *   - No C++ exception crosses this interface.  Calls on distinct streams
 *     may run from several threads at once.
 */
#ifndef BNORMALS_H
#define BNORMALS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BN_VERSION 3

/* status codes */
#define BN_OK 0
#define BN_ERR_INVALID_ARG 1
#define BN_ERR_UNSUPPORTED 2
#define BN_ERR_DEVICE 3
#define BN_ERR_OOM 4
#define BN_ERR_TIMEOUT 5

/* boundary-test modes */
#define BN_MASK_REL 0
#define BN_MASK_ABS 1
#define BN_MASK_NONE 2

/* per-pixel codes written to the mask */
#define BN_VALID 0
#define BN_BOUNDARY 1
#define BN_INVALID 2

/* methods */
#define BN_METHOD_FOUR_PAIR 0
#define BN_METHOD_PAIR_REMOVAL 1
#define BN_METHOD_MULTISCALE 2

/* flags */
#define BN_FLAG_COUNTS_ACCUMULATE 1u /* counts are added to n_valid/n_boundary/n_invalid */

/* limits */
#define BN_MAX_ALPHA 8
#define BN_MAX_SCALES 8
#define BN_MAX_STACK 64
#define BN_SMALL_BATCH 16
#define BN_MAX_WIDTH 65536
#define BN_MAX_PIXELS (1LL << 28)
#define BN_MAX_STREAMS 64 /* streams per device with a count work area at a time */

typedef struct bn_params {
    int32_t alpha;     /* stencil pixel distance, 1..BN_MAX_ALPHA (Section 3.1) */
    int32_t mask_mode; /* BN_MASK_REL, BN_MASK_ABS or BN_MASK_NONE (Section 3.2) */
    float tau;         /* threshold, finite and > 0 (ignored by BN_MASK_NONE) */
    uint32_t variant;  /* 0 = library's choice (the autotuner's entry for
                          the frame's size class, else vector tiles where the
                          method and layout allow them, except four-pair
                          frames of at most 2^19 pixels, which take the
                          scalar tiles); else a kernel variant id
                          (bn_variant_count / bn_variant_name), for tests and
                          tuning: every variant writes identical output */
    int32_t method;    /* BN_METHOD_*; 0 = the paper's four-pair estimator */
    int32_t scales;    /* BN_METHOD_MULTISCALE: K, 1..BN_MAX_SCALES; others: 0 or 1 */
    uint32_t flags;    /* 0 or BN_FLAG_COUNTS_ACCUMULATE */
    uint32_t reserved; /* 0 */
} bn_params;          /* 32 bytes; a zeroed structure plus alpha, mode and tau
                         selects the paper's method */

/* Per-frame pixel counts by code (16 bytes, 4-byte aligned, device memory).
 *
 * A call that is given one STORES the frame's counts in it (n_invalid =
 * pixels - n_valid - n_boundary, reserved = 0), or, with
 * BN_FLAG_COUNTS_ACCUMULATE in params->flags, ADDS them to the three
 * counters (for totals over many calls; the caller zeroes them first).  No
 * other bytes are written.
 *
 * The counts are reduced inside the launch that produces them, on a device
 * work area that the library owns (never in this structure): the
 * single-frame and stack calls take the work area of the calling stream -
 * one per (device, stream), from a fixed pool of BN_MAX_STREAMS per device
 * held by the library until the process ends - and a batch plan owns one per
 * frame of its capacity.  Calls on one stream run one after another, so they
 * share its work area safely.  Streams are told apart by their handle: a
 * stream destroyed while a counted launch on it is pending must not be
 * followed, before that launch completes, by a counted launch on a new
 * stream that takes over its handle value.  When a further stream needs a
 * work area and all BN_MAX_STREAMS are taken, the call first waits for the
 * whole device (hipDeviceSynchronize) and then hands the work areas out
 * afresh; during graph capture it returns BN_ERR_UNSUPPORTED instead, and a
 * host thread that is between another counted call and its launch at that
 * moment may race with it (so programs that count on more than
 * BN_MAX_STREAMS streams from several threads at once should not).  A launch
 * captured into a graph keeps the work area of the stream it was captured
 * on, so its replays must not overlap other calls on that stream (or replays
 * of other graphs captured on it). */
typedef struct bn_frame_stats {
    uint32_t n_valid;
    uint32_t n_boundary;
    uint32_t n_invalid;
    uint32_t reserved;
} bn_frame_stats; /* 16 bytes */

/* One frame of a batch.  depth: [height][depth_stride] binary32, row-major,
 * depth_stride >= width (elements), 4-byte aligned.  normals:
 * [height][width][3] binary32, dense, 4-byte aligned.  mask: [height][width]
 * uint8, dense.  stats: nullable, 4-byte aligned. */
typedef struct bn_frame {
    const float *depth;
    int32_t height;
    int32_t width;
    int64_t depth_stride;
    float fx, fy, cx, cy;
    float *normals;
    uint8_t *mask;
    bn_frame_stats *stats;
} bn_frame;

/*
 * One frame: normals, mask and (if stats != NULL) counts.
 *   depth     [height][depth_stride] binary32 depth (z, > 0; 0 = hole),
 *             4-byte aligned (as are normals)
 *   fx, fy    focal lengths in pixels (finite, > 0); cx, cy principal point
 *   params    alpha, mode, tau, variant, method, scales, flags (host
 *             pointer, read during the call)
 *   normals   [height][width][3] binary32 out
 *   mask      [height][width] uint8 out (BN_VALID / BN_BOUNDARY / BN_INVALID)
 *   stats     one bn_frame_stats: the frame's counts, stored (or added, with
 *             BN_FLAG_COUNTS_ACCUMULATE); nullable
 * height or width 0: nothing to do, BN_OK.  Limits: width <= BN_MAX_WIDTH,
 * height*width <= BN_MAX_PIXELS.  Returns BN_OK, BN_ERR_INVALID_ARG,
 * BN_ERR_UNSUPPORTED (alpha > BN_MAX_ALPHA, scales > BN_MAX_SCALES, a
 * forced variant that the method or the buffers' layout does not allow:
 * the multi-scale method takes the vector variants only when alpha * scales
 * <= 16; or counts asked, during graph capture, on a stream beyond the
 * BN_MAX_STREAMS that hold work areas)
 * or BN_ERR_DEVICE.
 */
int bn_estimate_normals(const float *depth, int32_t height, int32_t width,
                        int64_t depth_stride, float fx, float fy, float cx, float cy,
                        const bn_params *params, float *normals, uint8_t *mask,
                        bn_frame_stats *stats, void *stream);

/*
 * Adjoint of bn_estimate_normals with respect to the depth (the
 * vector-Jacobian product), with every pixel's code held fixed:
 *   grad_depth[j] = sum over VALID pixels p of (d normal_p / d depth_j) . grad_normals[p]
 * The codes are recomputed exactly as bn_estimate_normals decides them; the
 * entries of grad_normals at masked pixels are ignored (their normal is the
 * constant 0).  d1 does not enter Eqs. 10-12, so a pixel's own depth gets
 * gradient only through its four neighbours' normals.
 *   grad_normals [height][width][3] binary32, dense
 *   grad_depth   [height][width] binary32 out, dense, 4-byte aligned, overwritten
 * Same argument rules and errors as bn_estimate_normals (params->variant 0);
 * BN_ERR_UNSUPPORTED for a method other than BN_METHOD_FOUR_PAIR.  Width and
 * depth_stride multiples of 4, the three arrays 16-byte aligned and alpha
 * <= 4 take a vector kernel; any other layout takes scalar tiles.  Both sum
 * each gradient's four contributions in the same order: the same bits.
 */
int bn_normals_vjp(const float *depth, int32_t height, int32_t width, int64_t depth_stride,
                   float fx, float fy, float cx, float cy, const bn_params *params,
                   const float *grad_normals, float *grad_depth, void *stream);

/*
 * Stacks: n frames of one size in one launch, each with its own intrinsics
 * (a training or evaluation batch).  Frame k is what bn_estimate_normals /
 * bn_normals_vjp compute for it, bit for bit.
 *   depth        frame k at depth + k * depth_frame_stride (elements), rows
 *                of depth_stride elements; depth_frame_stride >=
 *                height * depth_stride
 *   intrinsics   host array of n bn_intrinsics, read during the call
 *   normals      [n][height][width][3] out;  mask [n][height][width] out
 *   stats        [n] bn_frame_stats, frame k's counts stored in entry k
 *                (added with BN_FLAG_COUNTS_ACCUMULATE); nullable
 *   grad_normals [n][height][width][3];  grad_depth [n][height][width] out
 * 1 <= n <= BN_MAX_STACK (n = 0, height 0 or width 0: nothing to do).
 * params->variant: 0 (vector tiles when the layout allows them, which
 * needs depth_frame_stride % 4 == 0 besides the single-frame rules), 1
 * ("scalar") or 2 ("vec4") for the forward; 0 for the adjoint.
 * Errors as for the single-frame calls; BN_ERR_UNSUPPORTED for n >
 * BN_MAX_STACK.  Nothing is allocated; the arguments travel in the launch.
 */
typedef struct bn_intrinsics {
    float fx, fy, cx, cy;
} bn_intrinsics;

int bn_estimate_normals_stack(const float *depth, int32_t n, int32_t height, int32_t width,
                              int64_t depth_stride, int64_t depth_frame_stride,
                              const bn_intrinsics *intrinsics, const bn_params *params,
                              float *normals, uint8_t *mask, bn_frame_stats *stats,
                              void *stream);
int bn_normals_vjp_stack(const float *depth, int32_t n, int32_t height, int32_t width,
                         int64_t depth_stride, int64_t depth_frame_stride,
                         const bn_intrinsics *intrinsics, const bn_params *params,
                         const float *grad_normals, float *grad_depth, void *stream);

/*
 * Batches: many frames of any mix of sizes, one launch.
 *
 * A plan holds the frame descriptors in device memory and a HIP graph of two
 * kernel nodes: one processes every tile of every frame (one workgroup per
 * tile of 1024 pixels by default), the other sums each frame's counts (in
 * chunks of 4096 tiles for large frames); running the plan replays the
 * graph.  A list of at most BN_SMALL_BATCH
 * frames instead carries its descriptors in the kernel arguments and reduces
 * its counts inside the one kernel (on a zeroed work area of the plan): an
 * update of such a list uploads nothing, and a run is a single kernel, its
 * own one-node graph.  Frames are described by bn_frame (device
 * pointers, owned by the caller, which must stay valid while the plan runs).
 * All frames share `params` (alpha, mode, tau, method, scales, flags;
 * params->variant must be 0);
 * each frame has its own size, stride, intrinsics and outputs, and its
 * counts go to its own bn_frame_stats or nowhere (stats = NULL).  Each frame's outputs are identical to those of
 * bn_estimate_normals on that frame.
 *
 * bn_batch_plan_create: validates every frame (the checks of
 *   bn_estimate_normals), allocates the plan (device descriptor table of
 *   n_frames entries, a tile-to-frame table, a table of 4 counts per tile,
 *   two pinned staging copies, n_frames count work areas) and instantiates
 *   the graph.
 *   Capacity = n_frames.  Returns BN_OK, BN_ERR_INVALID_ARG,
 *   BN_ERR_UNSUPPORTED, BN_ERR_OOM or BN_ERR_DEVICE; *out_plan is NULL on
 *   error.  Synchronous.
 * bn_batch_plan_update: replaces the frame list (n_frames <= capacity) with
 *   an asynchronous copy on `stream`, ordered after earlier work and before
 *   later runs on that stream.  The instantiated graph is kept; its kernel
 *   nodes' launch parameters (grid, table sizes) are updated in place by the
 *   next bn_batch_run.  A list with more tiles than the plan's tables hold
 *   grows them, which first synchronises `stream` (the plan's earlier runs
 *   must have finished).
 * bn_batch_run: one replay of the plan's graph over the current frame list
 *   on `stream`.
 * bn_batch_launch: the same kernels (two, or one for a small list), with
 *   the same output, as ordinary launches on `stream` instead of a graph
 *   replay.  Costs less host time per call (a graph replay costs tens of
 *   microseconds), so it suits small, latency-bound batches such as a
 *   server's; a long batch is the same either way.  Runs of one plan must
 *   not overlap (they share its descriptors and count work areas).
 * bn_batch_plan_info: pixels, tiles and workgroups of the current list.
 * bn_batch_plan_destroy: frees the plan; the caller makes sure no run of it
 *   is still in flight.
 */
typedef struct bn_batch_plan bn_batch_plan;
int bn_batch_plan_create(const bn_frame *frames_host, int32_t n_frames, const bn_params *params,
                         bn_batch_plan **out_plan);
int bn_batch_plan_update(bn_batch_plan *plan, const bn_frame *frames_host, int32_t n_frames,
                         void *stream);
int bn_batch_run(bn_batch_plan *plan, void *stream);
int bn_batch_launch(bn_batch_plan *plan, void *stream);
int bn_batch_plan_info(const bn_batch_plan *plan, int64_t *n_pixels, int64_t *n_tiles,
                       int32_t *n_workgroups);
void bn_batch_plan_destroy(bn_batch_plan *plan);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * small-list launch of bn_batch_launch without a plan.  Allocates nothing
 * (no hipMalloc / hipFree, no allocating library routine): the frame
 * descriptors travel in the kernel arguments and the per-frame count work
 * areas are a fixed array in device memory, BN_NOALLOC_MAX_FRAMES areas of
 * 4224 bytes (67.6 KB), which each GPU the library runs on holds until the
 * process ends.
 *   frames_host  [n_frames] frames as for a plan (device pointers, validated
 *                as by bn_batch_plan_create), 1 <= n_frames <=
 *                BN_NOALLOC_MAX_FRAMES (more: BN_ERR_UNSUPPORTED)
 *   params       as for a plan (variant 0)
 * Each frame's outputs and counts are those of bn_estimate_normals.  Two
 * kernels on `stream`: a fill kernel that zeroes the work areas, then the
 * batch.  Every call on a GPU shares that GPU's array (it keeps the last
 * call's contents), so calls that overlap in time on one GPU - on different
 * streams, or graph replays - race and must not be issued.
 */
#define BN_NOALLOC_MAX_FRAMES 16
int bn_estimate_normals_batch_noalloc(const bn_frame *frames_host, int32_t n_frames,
                                      const bn_params *params, void *stream);

/*
 * Autotuning.  Choices are kept per process in a table keyed by GPU
 * architecture, alpha and frame-size class (bit length of the pixel count);
 * when the environment variable BN_AUTOTUNE_CACHE names a file, the table
 * is loaded from it on first use and saved to it after each tuning.
 *
 * bn_autotune_plain: times every kernel variant (tile shape) of
 *   bn_estimate_normals that the method and layout allow - scalar or vector
 *   work items; workgroups of 256, 128 or 64 threads; one, two or four tiles
 *   per workgroup or a software-pipelined pair - on a ring of scratch frames
 *   of height x width (allocated and freed here, about 512 MiB, a synthetic
 *   scene with steps, noise and holes) and records the fastest; later calls
 *   with params->variant == 0 on frames of that size class use it.
 *   Synchronous.
 * bn_batch_plan_autotune: times the plan's launch over its grid shapes - a
 *   flat grid of one tile per workgroup (*best_shape = 0), of two or four
 *   consecutive tiles per workgroup (-2, -4), or 2, 4 or 8 persistent
 *   workgroups per compute unit (2, 4, 8) - keeps the fastest for this plan
 *   and records it for new plans of the same size class.  It RUNS the plan
 *   (outputs and counts are rewritten; with BN_FLAG_COUNTS_ACCUMULATE the
 *   counts accumulate).
 * bn_autotune_save / _load: write / read the table as JSON.
 * bn_autotune_reset: forget every entry.  bn_autotune_entries: table size.
 */
int bn_autotune_plain(int32_t height, int32_t width, const bn_params *params,
                      int32_t *best_variant, float *best_us);
int bn_batch_plan_autotune(bn_batch_plan *plan, void *stream, int32_t *best_shape,
                           float *best_us);
int bn_autotune_save(const char *path);
int bn_autotune_load(const char *path);
void bn_autotune_reset(void);
int bn_autotune_entries(void);

/*
 * Serving: continuous batching of frames of mixed sizes.
 *
 * Requests are queued first come, first served.  A request is admitted when
 * its slot - normals (12 B/px), mask (1 B/px), a bn_frame_stats and, for a
 * depth in host memory, a copy of the depth (4 B/px) - fits in the HBM
 * budget; admission starts the host-to-device copy of a host depth on a
 * copy stream (a device depth is used in place).  Launches store each
 * request's counts (BN_FLAG_COUNTS_ACCUMULATE is ignored).  Whenever fewer than max_batches_in_flight launches are
 * queued on the GPU, all admitted requests whose input is on the device (up
 * to max_batch) form one batched launch (bn_batch_plan) on a compute
 * stream.  New requests are therefore admitted and copied while earlier
 * batches run.  Outputs stay in device memory until the client releases the
 * request, which returns its slot to the budget.  Each request's outputs are
 * those of bn_estimate_normals on its frame, whatever it was batched with.
 *
 * The HIP backend runs the scheduler on a worker thread.  The fake backend
 * (tests, CPU only) runs nothing: bn_server_progress schedules what the
 * current time allows, bn_server_fake_advance moves a virtual clock, and copies and
 * launches take fake_copy_gbs / fake_launch_ns + fake_ns_per_pixel of
 * virtual time; bn_server_fake_fail makes one request's result fail.
 */
#define BN_BACKEND_HIP 0
#define BN_BACKEND_FAKE 1

#define BN_REQ_PENDING 0
#define BN_REQ_ADMITTED 1
#define BN_REQ_READY 2
#define BN_REQ_RUNNING 3
#define BN_REQ_DONE 4
#define BN_REQ_FAILED 5

typedef struct bn_server_config {
    int64_t hbm_budget_bytes;      /* device memory for request slots, > 0 */
    int32_t max_batch;             /* frames per launch, >= 1 */
    int32_t max_batches_in_flight; /* launches queued on the GPU at once, >= 1 */
    bn_params params;              /* shared by all requests (variant 0) */
    int32_t backend;               /* BN_BACKEND_HIP or BN_BACKEND_FAKE */
    int32_t reserved;
    double fake_ns_per_pixel;      /* fake backend: kernel time per pixel */
    double fake_launch_ns;         /* fake backend: time per launch */
    double fake_copy_gbs;          /* fake backend: host-to-device GB/s */
} bn_server_config;

typedef struct bn_request_info {
    int32_t state;       /* BN_REQ_* */
    int32_t status;      /* BN_OK, or the error of a failed request */
    int32_t batch_size;  /* frames in its launch */
    int32_t reserved;
    uint64_t batch;      /* launch id */
    double t_submit, t_admit, t_launch, t_done;  /* seconds, monotonic clock */
    float *normals;      /* device outputs, valid until release */
    uint8_t *mask;
    bn_frame_stats *stats;
} bn_request_info;

typedef struct bn_server_stats {
    int64_t submitted, completed, failed, released, batches, pending, in_flight_batches;
    int64_t bytes_in_use, peak_bytes_in_use, max_batch_seen;
} bn_server_stats;

typedef struct bn_server bn_server;
/* Errors: BN_ERR_INVALID_ARG, BN_ERR_UNSUPPORTED, BN_ERR_OOM (budget not
 * allocatable), BN_ERR_DEVICE. */
int bn_server_create(const bn_server_config *config, bn_server **out_server);
/* depth: device memory (depth_on_host = 0; must stay valid until the
 * request completes) or host memory (copied at admission; must stay valid
 * until then).  BN_ERR_OOM when the request can never fit the budget.
 * Thread-safe. */
int bn_server_submit(bn_server *server, const float *depth, int32_t depth_on_host,
                     int32_t height, int32_t width, int64_t depth_stride, float fx, float fy,
                     float cx, float cy, uint64_t *request_id);
int bn_server_query(bn_server *server, uint64_t request_id, bn_request_info *info);
/* Blocks until the request is done or failed (HIP backend), or
 * BN_ERR_TIMEOUT after timeout_s (< 0: no limit). */
int bn_server_wait(bn_server *server, uint64_t request_id, double timeout_s,
                   bn_request_info *info);
/* Returns a done or failed request's slot to the budget; its outputs are
 * no longer valid. */
int bn_server_release(bn_server *server, uint64_t request_id);
/* Scheduling passes until nothing changes at the current time (fake
 * backend; the HIP backend's worker does this continuously); returns the
 * number of state changes. */
int bn_server_progress(bn_server *server);
int bn_server_get_stats(bn_server *server, bn_server_stats *stats);
int bn_server_fake_advance(bn_server *server, double seconds);
int bn_server_fake_fail(bn_server *server, uint64_t request_id);
/* Waits for queued GPU work, then frees everything. */
void bn_server_destroy(bn_server *server);
/* Open-loop load: n_requests frames drawn uniformly from `pool` (device
 * depths), Poisson arrivals at rate_hz, each released on completion.
 * latency_s[i] = completion - scheduled arrival (n_requests entries). */
int bn_server_run_poisson(bn_server *server, const bn_frame *pool, int32_t n_pool,
                          double rate_hz, int32_t n_requests, uint64_t seed, double *latency_s,
                          double *wall_s, int64_t *pixels);

/*
 * Evaluation tools (Section 4).  All pointers are device pointers; nothing
 * is allocated; asynchronous on `stream`.
 *
 * bn_normal_angles: the spherical angle images of a normal map [H][W][3]
 *   binary32 (Eqs. 14-15, with the quadrant-aware arctangent):
 *     phi   = atan2(ny, nx), taken into [0, 2 pi)
 *     theta = atan2(sqrt(nx^2 + ny^2), nz), in [0, pi]
 *   evaluated in FP64 and stored as binary32 [H][W]; a zero vector gives 0, 0.
 * bn_angle_mse: mean squared error of the theta and of the phi images of
 *   two normal maps over the pixels whose code is BN_VALID in both (a NULL
 *   mask counts as all valid); result (device, 3 doubles): MSE theta, MSE
 *   phi, pixel count.  workspace: BN_MSE_WORKSPACE_DOUBLES doubles of device
 *   memory, owned by the caller, not shared by overlapping calls.  The sums
 *   run in FP64 in a fixed order (deterministic).
 * bn_plane_fit_normals: local plane fit over the (2 radius + 1)^2 window of
 *   each pixel (radius 2: the 25-neighbour fit used as ground truth on real
 *   depth, Section 4): the camera-facing eigenvector of the smallest
 *   eigenvalue of the scatter matrix of the back-projected window points
 *   (Eqs. 8-9), in FP64, stored as binary32 normals [H][W][3] and codes
 *   [H][W] (BN_VALID; BN_INVALID when the window leaves the image, holds a
 *   depth that is not finite and > 0, or has no unique smallest direction).
 *   radius 1..BN_MAX_FIT_RADIUS.  Frame arguments as bn_estimate_normals.
 */
#define BN_MSE_WORKSPACE_DOUBLES (3 * 2048)
#define BN_MAX_FIT_RADIUS 3
int bn_normal_angles(const float *normals, int32_t height, int32_t width, float *theta,
                     float *phi, void *stream);
int bn_angle_mse(const float *normals_a, const uint8_t *mask_a, const float *normals_b,
                 const uint8_t *mask_b, int32_t height, int32_t width, double *workspace,
                 double *result, void *stream);
int bn_plane_fit_normals(const float *depth, int32_t height, int32_t width, int64_t depth_stride,
                         float fx, float fy, float cx, float cy, int32_t radius, float *normals,
                         uint8_t *mask, void *stream);

/* Number of kernel variants of the plain entry point, and a name for each
 * id 1..count (NULL for an unknown id). */
int bn_variant_count(void);
const char *bn_variant_name(int variant);
/* 1 if `variant` can run this frame layout, 0 if not. */
int bn_variant_supported(int variant, const float *depth, int32_t height, int32_t width,
                         int64_t depth_stride, const float *normals, const uint8_t *mask);

const char *bn_status_string(int status);
int bn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BNORMALS_H */
