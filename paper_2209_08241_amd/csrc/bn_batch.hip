// Batched execution: every tile of every frame of a batch in one kernel
// launch, instantiated once as a HIP graph.
//
// Frames of different sizes are cut into tiles of 256 work items (1024
// pixels for vector frames).  Workgroup b owns the contiguous tile range
// [b*chunk, (b+1)*chunk) of the concatenated tile sequence, so the load is
// balanced whatever the frame mix, a workgroup touches few frames (one count
// reduction per frame segment), and - through the XCD-contiguous numbering
// of workgroups - neighbouring tiles, which share stencil rows, are
// processed by the same XCD.  Two grid shapes, picked by the autotuner:
//   * flat (default): one tile per workgroup, as many workgroups as tiles;
//     a workgroup retires with its stores still in flight and the
//     dispatcher refills the compute unit at once;
//   * persistent: k workgroups per compute unit, all resident, each looping
//     over its chunk.  On gfx9 one counter tracks loads and stores, so a
//     wait for the next tile's loads also waits for the previous tile's
//     stores; this shape wins only when launch work dominates.
// The frame descriptors live in device memory, so a plan's graph is
// replayed as is when the frames change (the grid of the flat shape is
// updated in place).
//
// Lists of at most kSmallFrames frames take another route: their
// descriptors travel in the kernel arguments (an update uploads nothing)
// and the counts go through the plain kernels' in-launch reduction on a
// zeroed scratch work area of the plan, so a launch is a single kernel.
// This is the latency path of a server's small batches.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "bn_device.h"
#include "bn_internal.h"
#include "bn_tiles.h"

#pragma clang fp contract(off)

namespace bn {

struct BatchFrame {
    FrameArgs a;
    uint32_t tile_begin;  // first tile in the batch-wide tile sequence
    uint32_t ntiles;
    uint32_t vec;         // 1: vector tiles, 0: scalar tiles
    uint32_t pad;
};

struct BatchHeader {
    uint32_t nframes;
    uint32_t ntiles;  // total over the batch
    uint32_t chunk;   // tiles per workgroup
    uint32_t pad;
};

// tile_frame[t] is the index of the frame that holds tile t, so that a
// workgroup finds its first frame with one load (a search over the frame
// descriptors is a chain of dependent loads, long next to a 1024-pixel tile).
//
// Counts: each wavefront stores the VALID / BOUNDARY counts of its quarter
// of a tile (VALID | BOUNDARY << 16, at most 256 pixels each) into
// wave_counts[4 t + w]; a second kernel of the same graph sums them per
// frame.  The main kernel thus has neither atomics nor workgroup barriers.
// At most 80 scalar registers: left alone the compiler takes 92 (allocated
// as 96), which it counts as fitting 8 wavefronts per SIMD, but the
// measured mean occupancy was 6.5 against 7.6 for the kernels of 61-67
// registers; capped at 80 (a few spills to VGPR lanes) the 256-frame mix
// runs 540 -> 527 us (72 and 64 spill more and are slower).
template <int A, int M>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_num_sgpr(80))) void k_batch(
    const BatchFrame *__restrict__ frames,
                                                  const uint32_t *__restrict__ tile_frame,
                                                  uint32_t *__restrict__ wave_counts,
                                                  uint32_t ntiles, uint32_t chunk,
                                                  uint32_t nframes) {
    __shared__ TileLds lds;
    const uint32_t blk = xcd_tile(blockIdx.x, gridDim.x);
    uint32_t t = blk * chunk;
    if (chunk == 0 || t >= ntiles) return;  // uniform: this workgroup has no tiles
    const uint32_t tend = min(t + chunk, ntiles);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    uint32_t fi = tile_frame[t];
    while (fi < nframes) {
        FrameArgs f = frames[fi].a;
        frame_pointers_global(f, &frames[fi].a);
        const uint32_t tb = frames[fi].tile_begin;
        const uint32_t nt = frames[fi].ntiles;
        const bool vec = frames[fi].vec != 0;
        const uint32_t seg_end = min(tend, tb + nt);
        for (; t < seg_end; ++t) {
            uint32_t cv = 0, cb = 0;
            run_tile<A, M>(f, vec, t - tb, lds, cv, cb);
            if (f.stats && lane == 0) wave_counts[4 * (int64_t)t + wave] = cv | (cb << 16);
        }
        // done (always so in the flat shape) before looking at the next
        // frame's descriptor, which would hold the workgroup for one more load
        if (t >= tend) break;
        do {
            ++fi;
        } while (fi < nframes && frames[fi].ntiles == 0);
    }
}

// Sums of the wavefront counts: workgroup (f, c) takes chunk c of
// kCountChunk tiles of frame f.  A frame of one chunk adds its totals to its
// bn_frame_stats (or adds them, BN_FLAG_COUNTS_ACCUMULATE) at once; the
// chunks of a larger frame combine through the in-launch reduction of the
// plain kernels, on the plan's work area for the frame, so that one huge
// frame is not summed by a single workgroup.
constexpr uint32_t kCountChunk = 4096;

__global__ __launch_bounds__(kBlock) void k_batch_counts(const BatchFrame *__restrict__ frames,
                                                         const uint32_t *__restrict__ wave_counts,
                                                         uint32_t nframes) {
    __shared__ uint32_t s_sum[kBlock / 64][2];
    const uint32_t fi = blockIdx.x;
    if (fi >= nframes) return;
    FrameArgs f = frames[fi].a;
    frame_pointers_global(f, &frames[fi].a);
    const uint32_t nt = frames[fi].ntiles;
    const uint32_t nchunks = (nt + kCountChunk - 1) / kCountChunk;
    const uint32_t c = blockIdx.y;
    if (!f.stats || c >= nchunks) return;  // uniform over the workgroup
    const uint32_t kb = c * kCountChunk, ke = min(nt, kb + kCountChunk);
    // the 4 wavefront counts of a tile are one 16-byte load; unrolled so that
    // several loads are in flight per thread
    const uint4 *wc = reinterpret_cast<const uint4 *>(wave_counts) + frames[fi].tile_begin;
    uint32_t v = 0, b = 0;
#pragma unroll 8
    for (uint32_t k = kb + threadIdx.x; k < ke; k += kBlock) {
        const uint4 q = wc[k];
        v += (q.x & 0xffffu) + (q.y & 0xffffu) + (q.z & 0xffffu) + (q.w & 0xffffu);
        b += (q.x >> 16) + (q.y >> 16) + (q.z >> 16) + (q.w >> 16);
    }
    // wavefront sums through DPP-free shuffles, then across the 4 wavefronts
    for (int off = 32; off > 0; off >>= 1) {
        v += __shfl_xor(v, off);
        b += __shfl_xor(b, off);
    }
    if ((threadIdx.x & 63u) == 0) {
        s_sum[threadIdx.x >> 6][0] = v;
        s_sum[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t vt = 0, bt = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            vt += s_sum[w][0];
            bt += s_sum[w][1];
        }
        if (nchunks == 1)
            put_counts(f.stats, vt, bt, f.npix, f.overwrite);
        else
            reduce_counts(f.work, f.stats, c, nchunks, vt, bt, f.npix, f.overwrite);
    }
}

constexpr int kSmallFrames = BN_SMALL_BATCH;

struct SmallBatch {
    uint32_t nframes;
    uint32_t ntiles;
    uint32_t vec_bits;                       // bit k: frame k takes vector tiles
    uint32_t pad;
    uint32_t tile_begin[kSmallFrames];       // unused entries: UINT32_MAX
    uint32_t tile_count[kSmallFrames];
    FrameArgs f[kSmallFrames];               // work = the plan's scratch for frame k
};

// Workgroup b takes tile b of the concatenated sequence; its frame is the
// last one whose first tile is <= b (a scan of uniform scalar values).
template <int A, int M>
__global__ __launch_bounds__(kBlock) void k_batch_small(const SmallBatch s) {
    __shared__ TileLds lds;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= s.ntiles) return;
    uint32_t k = 0;
#pragma unroll
    for (uint32_t j = 1; j < (uint32_t)kSmallFrames; ++j)
        if (s.tile_begin[j] <= b) k = j;
    const FrameArgs f = s.f[k];
    const uint32_t tile = b - s.tile_begin[k];
    const uint32_t nparts = s.tile_count[k];
    if ((s.vec_bits >> k) & 1u) {
        vec4_tile_counted<A, M>(f, tile, tile, nparts, lds);
        return;
    }
    scalar_tile_counted<A, M>(f, tile, tile, nparts, lds);
}

typedef void (*BatchKernelFn)(const BatchFrame *, const uint32_t *, uint32_t *, uint32_t,
                              uint32_t, uint32_t);
typedef void (*SmallKernelFn)(const SmallBatch);

template <int M>
static SmallKernelFn small_kernel_m(int alpha) {
    switch (alpha) {
        case 1: return k_batch_small<1, M>;
        case 2: return k_batch_small<2, M>;
        case 3: return k_batch_small<3, M>;
        case 4: return k_batch_small<4, M>;
        case 5: return k_batch_small<5, M>;
        case 6: return k_batch_small<6, M>;
        case 7: return k_batch_small<7, M>;
        case 8: return k_batch_small<8, M>;
    }
    return nullptr;
}

static SmallKernelFn small_kernel(int method, int alpha, int scales) {
    method = kernel_method(method, alpha, scales);
    if (method == kFourPair) return small_kernel_m<kFourPair>(alpha);
    if (method == kPairRemoval) return small_kernel_m<kPairRemoval>(alpha);
    if (method == kMultiScale) return small_kernel_m<kMultiScale>(alpha);
    if (method == kMultiScaleLong) return small_kernel_m<kMultiScaleLong>(alpha);
    return nullptr;
}

template <int M>
static BatchKernelFn batch_kernel_m(int alpha) {
    switch (alpha) {
        case 1: return k_batch<1, M>;
        case 2: return k_batch<2, M>;
        case 3: return k_batch<3, M>;
        case 4: return k_batch<4, M>;
        case 5: return k_batch<5, M>;
        case 6: return k_batch<6, M>;
        case 7: return k_batch<7, M>;
        case 8: return k_batch<8, M>;
    }
    return nullptr;
}

static BatchKernelFn batch_kernel(int method, int alpha, int scales) {
    method = kernel_method(method, alpha, scales);
    if (method == kFourPair) return batch_kernel_m<kFourPair>(alpha);
    if (method == kPairRemoval) return batch_kernel_m<kPairRemoval>(alpha);
    if (method == kMultiScale) return batch_kernel_m<kMultiScale>(alpha);
    if (method == kMultiScaleLong) return batch_kernel_m<kMultiScaleLong>(alpha);
    return nullptr;
}

}  // namespace bn

using namespace bn;

struct bn_batch_plan {
    int device = -1;
    bn_params params{};
    int32_t capacity = 0;          // frames
    uint64_t tile_capacity = 0;    // entries of the tile -> frame table
    int cus = 0;
    int32_t shape = 0;             // grid shape (kFlat, -2, -4: tiles per workgroup; k > 0:
                                   // k persistent workgroups per compute unit)
    uint32_t grid = 0;
    size_t buf_bytes = 0;
    // device buffer and two pinned host images of it:
    //   BatchHeader | BatchFrame[capacity] | uint32 tile_frame[tile_capacity]
    void *dbuf = nullptr;
    void *staging[2] = {nullptr, nullptr};
    hipEvent_t staged[2] = {nullptr, nullptr};
    int next = 0;                  // staging copy the next update writes
    uint32_t *dcounts = nullptr;   // 4 wavefront counts per tile (tile_capacity tiles)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node = nullptr;         // the tile kernel
    hipGraphNode_t count_node = nullptr;   // the per-frame count sums
    BatchKernelFn fn = nullptr;
    BatchHeader hdr{};                     // current header (kernel arguments)
    bool graph_stale = false;              // node parameters behind the frame list
    uint64_t total_tiles = 0;
    uint64_t total_pixels = 0;
    // small lists (at most kSmallFrames frames): descriptors in the kernel
    // arguments, counts reduced on `work`, one kernel (graph sgraph/sexec)
    bool small_mode = false;
    SmallBatch small{};
    SmallKernelFn small_fn = nullptr;
    // one count work area per frame of the capacity, zero between launches
    // (the small lists' in-kernel reductions, the large frames' count sums)
    WorkArea *work = nullptr;
    uint32_t count_chunks = 1;             // grid.y of the count sums
    hipGraph_t sgraph = nullptr;
    hipGraphExec_t sexec = nullptr;
    hipGraphNode_t snode = nullptr;
    bool small_stale = false;
};

namespace {

constexpr int32_t kFlat = 0;  // shape of the flat grid, one tile per workgroup

size_t table_offset(int32_t capacity) {
    return sizeof(BatchHeader) + sizeof(BatchFrame) * (size_t)capacity;
}

size_t buffer_bytes(int32_t capacity, uint64_t tile_capacity) {
    return table_offset(capacity) + sizeof(uint32_t) * (size_t)tile_capacity;
}

// Vector tiles for this frame under these parameters?
bool frame_vec(const bn_frame &s, const bn_params *p) {
    return method_has_vec4(p) && vec4_layout(s.depth, s.width, s.depth_stride, s.normals, s.mask);
}

// Validate the frames; total tiles and pixels.
int count_frames(const bn_frame *frames, int32_t n, const bn_params *p, uint64_t *tiles,
                 uint64_t *pixels) {
    uint64_t t = 0, px = 0;
    for (int32_t k = 0; k < n; ++k) {
        const bn_frame &s = frames[k];
        int rc = check_frame_args(s.depth, s.height, s.width, s.depth_stride, s.fx, s.fy, s.cx,
                                  s.cy, s.normals, s.mask);
        if (rc == BN_OK) rc = check_stats_arg(s.stats);
        if (rc != BN_OK) return rc;
        if (s.height > 0 && s.width > 0) {
            const bool vec = frame_vec(s, p);
            const uint64_t items = (uint64_t)s.height * (uint64_t)(vec ? s.width / 4 : s.width);
            t += (items + kBlock - 1) / kBlock;
            px += (uint64_t)s.height * (uint64_t)s.width;
        }
    }
    if (t > 0x7fffffffull) return BN_ERR_UNSUPPORTED;
    *tiles = t;
    *pixels = px;
    return BN_OK;
}

// Workgroups of a grid shape: shape <= 0 is a flat grid of max(1, -shape)
// consecutive tiles per workgroup; shape > 0 is `shape` persistent
// workgroups per compute unit.
uint32_t grid_for(uint64_t tiles, int cus, int32_t shape) {
    if (shape <= 0) {
        const uint64_t per = shape < -1 ? (uint64_t)(-shape) : 1u;
        return tiles ? (uint32_t)((tiles + per - 1) / per) : 1u;
    }
    return (uint32_t)cus * (uint32_t)shape;
}

// Host image of the descriptors of `frames` (already validated) in `base`.
int build_table(const bn_frame *frames, int32_t n, const bn_params *p, int32_t capacity,
                uint32_t grid, WorkArea *work, uint32_t *count_chunks, void *base) {
    auto *hdr = static_cast<BatchHeader *>(base);
    auto *fr = reinterpret_cast<BatchFrame *>(hdr + 1);
    auto *tf = reinterpret_cast<uint32_t *>(static_cast<char *>(base) + table_offset(capacity));
    uint64_t tiles = 0;
    *count_chunks = 1;
    for (int32_t k = 0; k < n; ++k) {
        const bn_frame &s = frames[k];
        const bool vec = frame_vec(s, p);
        BatchFrame b;
        std::memset(&b, 0, sizeof(b));
        uint64_t nt = 0;
        if (s.height > 0 && s.width > 0) {
            fill_frame_args(b.a, s.depth, s.height, s.width, s.depth_stride, s.fx, s.fy, s.cx,
                            s.cy, p, s.normals, s.mask, s.stats, vec ? 4 : 1);
            b.a.work = work + k;
            nt = ((uint64_t)b.a.nitems + kBlock - 1) / kBlock;
        }
        const uint32_t nc = (uint32_t)((nt + kCountChunk - 1) / kCountChunk);
        if (nc > *count_chunks) *count_chunks = nc;
        b.tile_begin = (uint32_t)tiles;
        b.ntiles = (uint32_t)nt;
        b.vec = vec ? 1u : 0u;
        for (uint64_t t = 0; t < nt; ++t) tf[tiles + t] = (uint32_t)k;
        tiles += nt;
        fr[k] = b;
    }
    hdr->nframes = (uint32_t)n;
    hdr->ntiles = (uint32_t)tiles;
    hdr->chunk = tiles ? (uint32_t)((tiles + grid - 1) / grid) : 0;
    hdr->pad = 0;
    if (hdr->chunk > 4096) return BN_ERR_UNSUPPORTED;  // parts stay below 2^22 pixels
    return BN_OK;
}

// The kernel-argument image of a small list (already validated); frame k
// reduces its counts on work[k].
void fill_small(SmallBatch &sb, const bn_frame *frames, int32_t n, const bn_params *params,
                WorkArea *work) {
    std::memset(&sb, 0, sizeof(sb));
    uint32_t tiles = 0;
    for (int k = 0; k < kSmallFrames; ++k) sb.tile_begin[k] = UINT32_MAX;
    for (int32_t k = 0; k < n; ++k) {
        const bn_frame &s = frames[k];
        const bool vec = frame_vec(s, params);
        uint32_t nt = 0;
        if (s.height > 0 && s.width > 0) {
            fill_frame_args(sb.f[k], s.depth, s.height, s.width, s.depth_stride, s.fx, s.fy, s.cx,
                            s.cy, params, s.normals, s.mask, s.stats, vec ? 4 : 1);
            sb.f[k].work = work + k;
            nt = (sb.f[k].nitems + kBlock - 1) / kBlock;
        }
        sb.tile_begin[k] = tiles;
        sb.tile_count[k] = nt;
        if (vec) sb.vec_bits |= 1u << k;
        tiles += nt;
    }
    sb.nframes = (uint32_t)n;
    sb.ntiles = tiles;
}

void build_small(bn_batch_plan *pl, const bn_frame *frames, int32_t n) {
    fill_small(pl->small, frames, n, &pl->params, pl->work);
}

hipKernelNodeParams kernel_params(void *func, dim3 grid, void **args) {
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = func;
    kp.gridDim = grid;
    kp.blockDim = dim3(kBlock);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return kp;
}

// The two kernels' arguments for the plan's current buffers and header.
struct BatchArgs {
    const BatchFrame *frames;
    const uint32_t *tile_frame;
    uint32_t *wave_counts;
    const uint32_t *wave_counts_c;
    uint32_t ntiles, chunk, nframes;
    void *main[6];
    void *counts[3];
    explicit BatchArgs(const bn_batch_plan *pl)
        : frames(reinterpret_cast<const BatchFrame *>(static_cast<const char *>(pl->dbuf) +
                                                      sizeof(BatchHeader))),
          tile_frame(reinterpret_cast<const uint32_t *>(static_cast<const char *>(pl->dbuf) +
                                                        table_offset(pl->capacity))),
          wave_counts(pl->dcounts),
          wave_counts_c(pl->dcounts),
          ntiles(pl->hdr.ntiles),
          chunk(pl->hdr.chunk),
          nframes(pl->hdr.nframes),
          main{(void *)&frames, (void *)&tile_frame, (void *)&wave_counts,
               (void *)&ntiles, (void *)&chunk,      (void *)&nframes},
          counts{(void *)&frames, (void *)&wave_counts_c, (void *)&nframes} {}
    BatchArgs(const BatchArgs &) = delete;
    BatchArgs &operator=(const BatchArgs &) = delete;
    dim3 count_grid(const bn_batch_plan *pl) const { return dim3(nframes ? nframes : 1u, pl->count_chunks); }
};

// Kernel node parameters (buffer pointers, header values, grids) into the
// graph, or a fresh graph [tile kernel] -> [count sums] when none exists.
int refresh_node(bn_batch_plan *pl) {
    BatchArgs a(pl);
    hipKernelNodeParams kp = kernel_params(reinterpret_cast<void *>(pl->fn), pl->grid, a.main);
    hipKernelNodeParams cp = kernel_params(reinterpret_cast<void *>(k_batch_counts),
                                           a.count_grid(pl), a.counts);
    pl->graph_stale = false;
    if (!pl->exec) {
        if (hipGraphCreate(&pl->graph, 0) != hipSuccess ||
            hipGraphAddKernelNode(&pl->node, pl->graph, nullptr, 0, &kp) != hipSuccess ||
            hipGraphAddKernelNode(&pl->count_node, pl->graph, &pl->node, 1, &cp) != hipSuccess ||
            hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess)
            return BN_ERR_DEVICE;
        return BN_OK;
    }
    if (hipGraphExecKernelNodeSetParams(pl->exec, pl->node, &kp) != hipSuccess ||
        hipGraphExecKernelNodeSetParams(pl->exec, pl->count_node, &cp) != hipSuccess)
        return BN_ERR_DEVICE;
    return BN_OK;
}

void free_buffers(bn_batch_plan *pl) {
    for (int k = 0; k < 2; ++k) {
        if (pl->staging[k]) (void)hipHostFree(pl->staging[k]);
        pl->staging[k] = nullptr;
    }
    if (pl->dbuf) (void)hipFree(pl->dbuf);
    pl->dbuf = nullptr;
    if (pl->dcounts) (void)hipFree(pl->dcounts);
    pl->dcounts = nullptr;
}

int alloc_buffers(bn_batch_plan *pl, uint64_t tile_capacity) {
    pl->tile_capacity = tile_capacity;
    pl->buf_bytes = buffer_bytes(pl->capacity, tile_capacity);
    for (int k = 0; k < 2; ++k)
        if (hipHostMalloc(&pl->staging[k], pl->buf_bytes, hipHostMallocDefault) != hipSuccess)
            return BN_ERR_OOM;
    if (hipMalloc(&pl->dbuf, pl->buf_bytes) != hipSuccess) return BN_ERR_OOM;
    if (hipMalloc(&pl->dcounts, sizeof(uint32_t) * 4 * (size_t)tile_capacity) != hipSuccess)
        return BN_ERR_OOM;
    return BN_OK;
}

void free_plan(bn_batch_plan *pl) {
    if (!pl) return;
    for (int k = 0; k < 2; ++k) {
        if (pl->staged[k]) {
            (void)hipEventSynchronize(pl->staged[k]);
            (void)hipEventDestroy(pl->staged[k]);
        }
    }
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->sexec) (void)hipGraphExecDestroy(pl->sexec);
    if (pl->sgraph) (void)hipGraphDestroy(pl->sgraph);
    if (pl->work) (void)hipFree(pl->work);
    free_buffers(pl);
    delete pl;
}

// The small list's graph: one kernel node, created on first use, its
// arguments rewritten after each update.
int refresh_small_node(bn_batch_plan *pl) {
    void *args[1] = {(void *)&pl->small};
    hipKernelNodeParams kp =
        kernel_params(reinterpret_cast<void *>(pl->small_fn), pl->small.ntiles, args);
    pl->small_stale = false;
    if (!pl->sexec) {
        if (hipGraphCreate(&pl->sgraph, 0) != hipSuccess ||
            hipGraphAddKernelNode(&pl->snode, pl->sgraph, nullptr, 0, &kp) != hipSuccess ||
            hipGraphInstantiate(&pl->sexec, pl->sgraph, nullptr, nullptr, 0) != hipSuccess)
            return BN_ERR_DEVICE;
        return BN_OK;
    }
    return hipGraphExecKernelNodeSetParams(pl->sexec, pl->snode, &kp) == hipSuccess
               ? BN_OK
               : BN_ERR_DEVICE;
}

// Write `frames` into the staging copy `k` and send it to the device on
// `stream` (header, descriptors and the used part of the tile table).
int upload(bn_batch_plan *pl, const bn_frame *frames, int32_t n, int k, hipStream_t stream,
           uint64_t tiles) {
    int rc = build_table(frames, n, &pl->params, pl->capacity, pl->grid, pl->work,
                         &pl->count_chunks, pl->staging[k]);
    if (rc != BN_OK) return rc;
    pl->hdr = *static_cast<const BatchHeader *>(pl->staging[k]);
    const size_t bytes = table_offset(pl->capacity) + sizeof(uint32_t) * (size_t)tiles;
    if (hipMemcpyAsync(pl->dbuf, pl->staging[k], bytes, hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipEventRecord(pl->staged[k], stream) != hipSuccess)
        return BN_ERR_DEVICE;
    return BN_OK;
}

}  // namespace

namespace bn {
bool batch_plan_uploads(const bn_batch_plan *plan) { return plan && !plan->small_mode; }
}  // namespace bn

extern "C" {

int bn_batch_plan_create(const bn_frame *frames_host, int32_t n_frames, const bn_params *params,
                         bn_batch_plan **out_plan) {
    if (!out_plan) return BN_ERR_INVALID_ARG;
    *out_plan = nullptr;
    if (!frames_host || n_frames < 1) return BN_ERR_INVALID_ARG;
    int rc = check_params_args(params);
    if (rc != BN_OK) return rc;
    if (params->variant != VAR_AUTO) return BN_ERR_UNSUPPORTED;
    BatchKernelFn fn = batch_kernel(params->method, params->alpha, params->scales);
    SmallKernelFn sfn = small_kernel(params->method, params->alpha, params->scales);
    if (!fn || !sfn) return BN_ERR_UNSUPPORTED;
    uint64_t tiles = 0, pixels = 0;
    rc = count_frames(frames_host, n_frames, params, &tiles, &pixels);
    if (rc != BN_OK) return rc;

    bn_batch_plan *pl = new (std::nothrow) bn_batch_plan();
    if (!pl) return BN_ERR_OOM;
    pl->params = *params;
    pl->capacity = n_frames;
    pl->fn = fn;
    pl->small_fn = sfn;
    if (hipGetDevice(&pl->device) != hipSuccess) {
        free_plan(pl);
        return BN_ERR_DEVICE;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) !=
            hipSuccess ||
        cus <= 0)
        cus = 256;
    pl->cus = cus;
    // the grid shape tuned for this alpha and batch size class, if recorded
    // (the table stores the flat shape as -1)
    const int tuned = tuned_batch_shape(params->method, params->alpha, pixels);
    pl->shape = tuned == -1 ? kFlat : tuned;
    pl->grid = grid_for(tiles, cus, pl->shape);
    pl->total_tiles = tiles;
    pl->total_pixels = pixels;
    for (int k = 0; k < 2; ++k) {
        if (hipEventCreateWithFlags(&pl->staged[k], hipEventDisableTiming) != hipSuccess) {
            free_plan(pl);
            return BN_ERR_DEVICE;
        }
    }
    // the counts' work areas, one per frame of the capacity, zero from here on
    const size_t work_bytes = sizeof(WorkArea) * (size_t)n_frames;
    if (hipMalloc(&pl->work, work_bytes) != hipSuccess) {
        free_plan(pl);
        return BN_ERR_OOM;
    }
    if (hipMemsetAsync(pl->work, 0, work_bytes, nullptr) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess) {
        free_plan(pl);
        return BN_ERR_DEVICE;
    }
    rc = alloc_buffers(pl, tiles > 0 ? tiles : 1);
    if (rc == BN_OK) rc = build_table(frames_host, n_frames, params, pl->capacity, pl->grid,
                                      pl->work, &pl->count_chunks, pl->staging[0]);
    if (rc == BN_OK) pl->hdr = *static_cast<const BatchHeader *>(pl->staging[0]);
    if (rc == BN_OK &&
        hipMemcpy(pl->dbuf, pl->staging[0], pl->buf_bytes, hipMemcpyHostToDevice) != hipSuccess)
        rc = BN_ERR_DEVICE;
    if (rc == BN_OK) rc = refresh_node(pl);
    if (rc != BN_OK) {
        free_plan(pl);
        return rc;
    }
    pl->next = 1;  // staging[0] holds the current table
    if (n_frames <= kSmallFrames) {
        build_small(pl, frames_host, n_frames);
        pl->small_mode = true;
        pl->small_stale = true;
    }
    *out_plan = pl;
    return BN_OK;
}

int bn_batch_plan_update(bn_batch_plan *plan, const bn_frame *frames_host, int32_t n_frames,
                         void *stream) {
    if (!plan || !frames_host || n_frames < 1) return BN_ERR_INVALID_ARG;
    if (n_frames > plan->capacity) return BN_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    uint64_t tiles = 0, pixels = 0;
    int rc = count_frames(frames_host, n_frames, &plan->params, &tiles, &pixels);
    if (rc != BN_OK) return rc;
    if (n_frames <= kSmallFrames) {
        // descriptors in the kernel arguments: nothing to upload
        build_small(plan, frames_host, n_frames);
        plan->small_mode = true;
        plan->small_stale = true;
        plan->total_tiles = tiles;
        plan->total_pixels = pixels;
        return BN_OK;
    }
    plan->small_mode = false;
    const uint32_t grid = grid_for(tiles, plan->cus, plan->shape);
    if (tiles > 0 && (tiles + grid - 1) / grid > 4096) return BN_ERR_UNSUPPORTED;
    if (tiles > plan->tile_capacity) {
        // a larger tile table: wait for every use of the old buffers first
        if (hipStreamSynchronize(s) != hipSuccess ||
            hipEventSynchronize(plan->staged[0]) != hipSuccess ||
            hipEventSynchronize(plan->staged[1]) != hipSuccess)
            return BN_ERR_DEVICE;
        // allocate the new buffers before releasing the old ones, so that a
        // failed allocation leaves the plan as it was
        bn_batch_plan fresh;
        fresh.capacity = plan->capacity;
        rc = alloc_buffers(&fresh, tiles + tiles / 4);
        if (rc != BN_OK) {
            free_buffers(&fresh);
            return rc;
        }
        free_buffers(plan);
        for (int j = 0; j < 2; ++j) {
            plan->staging[j] = fresh.staging[j];
            fresh.staging[j] = nullptr;
        }
        plan->dbuf = fresh.dbuf;
        plan->dcounts = fresh.dcounts;
        plan->buf_bytes = fresh.buf_bytes;
        plan->tile_capacity = fresh.tile_capacity;
        fresh.dbuf = nullptr;
        fresh.dcounts = nullptr;
    }
    const int k = plan->next;
    // the staging copy may still feed the upload issued two updates ago
    if (hipEventSynchronize(plan->staged[k]) != hipSuccess) return BN_ERR_DEVICE;
    plan->grid = grid;
    rc = upload(plan, frames_host, n_frames, k, s, tiles);
    if (rc != BN_OK) return rc;
    plan->next = 1 - k;
    plan->total_tiles = tiles;
    plan->total_pixels = pixels;
    // new header values, grids and pointers reach the graph at its next run
    plan->graph_stale = true;
    return BN_OK;
}

int bn_batch_run(bn_batch_plan *plan, void *stream) {
    if (!plan || !plan->exec) return BN_ERR_INVALID_ARG;
    if (plan->small_mode) {
        if (plan->small.ntiles == 0) return BN_OK;  // only empty frames
        if (plan->small_stale) {
            const int rc = refresh_small_node(plan);
            if (rc != BN_OK) return rc;
        }
        return hipGraphLaunch(plan->sexec, (hipStream_t)stream) == hipSuccess ? BN_OK
                                                                              : BN_ERR_DEVICE;
    }
    if (plan->graph_stale) {
        const int rc = refresh_node(plan);
        if (rc != BN_OK) return rc;
    }
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

int bn_batch_launch(bn_batch_plan *plan, void *stream) {
    if (!plan || !plan->exec) return BN_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (plan->small_mode) {
        if (plan->small.ntiles == 0) return BN_OK;  // only empty frames
        void *args[1] = {(void *)&plan->small};
        return hipLaunchKernel(reinterpret_cast<const void *>(plan->small_fn),
                               dim3(plan->small.ntiles), dim3(kBlock), args, 0, s) == hipSuccess
                   ? BN_OK
                   : BN_ERR_DEVICE;
    }
    BatchArgs a(plan);
    if (hipLaunchKernel(reinterpret_cast<const void *>(plan->fn), dim3(plan->grid),
                        dim3(kBlock), a.main, 0, s) != hipSuccess ||
        hipLaunchKernel(reinterpret_cast<const void *>(k_batch_counts), a.count_grid(plan),
                        dim3(kBlock), a.counts, 0, s) != hipSuccess)
        return BN_ERR_DEVICE;
    return BN_OK;
}

int bn_batch_plan_info(const bn_batch_plan *plan, int64_t *n_pixels, int64_t *n_tiles,
                       int32_t *n_workgroups) {
    if (!plan) return BN_ERR_INVALID_ARG;
    if (n_pixels) *n_pixels = (int64_t)plan->total_pixels;
    if (n_tiles) *n_tiles = (int64_t)plan->total_tiles;
    if (n_workgroups)
        *n_workgroups = (int32_t)(plan->small_mode ? plan->small.ntiles : plan->grid);
    return BN_OK;
}

// Re-grid the plan: new chunk and workgroup count in the graph's kernel
// arguments (they take effect at the next run).
static int set_grid(bn_batch_plan *plan, int32_t shape, hipStream_t stream) {
    (void)stream;
    const uint32_t grid = grid_for(plan->hdr.ntiles, plan->cus, shape);
    const uint32_t chunk = plan->hdr.ntiles ? (plan->hdr.ntiles + grid - 1) / grid : 0;
    if (chunk > 4096) return BN_ERR_UNSUPPORTED;
    plan->shape = shape;
    plan->grid = grid;
    plan->hdr.chunk = chunk;
    return refresh_node(plan);
}

int bn_batch_plan_autotune(bn_batch_plan *plan, void *stream, int32_t *best_shape,
                           float *best_us) {
    if (!plan || !plan->exec) return BN_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return BN_ERR_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return BN_ERR_DEVICE;
    }
    if (plan->small_mode) {
        // one shape only (a workgroup per tile): time it, record nothing
        int rc = bn_batch_run(plan, s);
        (void)hipEventRecord(e0, s);
        const int reps = 3;
        for (int r = 0; r < reps && rc == BN_OK; ++r) rc = bn_batch_run(plan, s);
        (void)hipEventRecord(e1, s);
        if (rc == BN_OK && hipEventSynchronize(e1) != hipSuccess) rc = BN_ERR_DEVICE;
        float ms = 0.f;
        if (rc == BN_OK) (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != BN_OK) return rc;
        if (best_shape) *best_shape = kFlat;
        if (best_us) *best_us = 1000.f * ms / reps;
        return BN_OK;
    }
    const int32_t cands[] = {kFlat, -2, -4, 2, 4, 8};
    int32_t best = kFlat;
    bool found = false;
    float best_t = 1e30f;
    int rc = BN_OK;
    for (int32_t c : cands) {
        rc = set_grid(plan, c, s);
        if (rc == BN_ERR_UNSUPPORTED) continue;
        if (rc != BN_OK) break;
        if (hipGraphLaunch(plan->exec, s) != hipSuccess) {
            rc = BN_ERR_DEVICE;
            break;
        }
        (void)hipEventRecord(e0, s);
        const int reps = 3;
        for (int r = 0; r < reps; ++r) (void)hipGraphLaunch(plan->exec, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = BN_ERR_DEVICE;
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const float us = 1000.f * ms / reps;
        if (us < best_t) {
            best_t = us;
            best = c;
            found = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != BN_OK && rc != BN_ERR_UNSUPPORTED) return rc;
    if (!found) return BN_ERR_UNSUPPORTED;
    rc = set_grid(plan, best, s);
    if (rc != BN_OK) return rc;
    // the table stores the flat shape as -1 (0 means "nothing recorded")
    record_tuning(1, plan->params.method, plan->params.alpha, plan->total_pixels,
                  best == kFlat ? -1 : (int)best, best_t);
    if (best_shape) *best_shape = best;
    if (best_us) *best_us = best_t;
    return BN_OK;
}

void bn_batch_plan_destroy(bn_batch_plan *plan) { free_plan(plan); }

}  // extern "C"

// ---------------------------------------------------------------------------
// The allocation-free batched launch: the small-list kernel of
// bn_batch_launch, with its count work areas in a fixed device array
// instead of a plan's allocation.
// ---------------------------------------------------------------------------
namespace {

// One count work area per frame of a list of at most BN_NOALLOC_MAX_FRAMES;
// each GPU holds its own copy until the process ends.
__device__ __align__(256) WorkArea scratch[BN_NOALLOC_MAX_FRAMES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
WorkArea *g_scratch[kMaxDevices];  // scratch's device address, per device

__global__ __launch_bounds__(256) void k_clear_words(unsigned long long *p, uint32_t words) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < words) p[i] = 0ull;
}

// scratch's address on the current device, looked up once per device with
// that device current (the array's name is only a host-side stand-in).
int scratch_for_current_device(WorkArea **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BN_ERR_DEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return BN_ERR_DEVICE;
        g_scratch[dev] = static_cast<WorkArea *>(p);
    }
    *out = g_scratch[dev];
    return BN_OK;
}

}  // namespace

extern "C" int bn_estimate_normals_batch_noalloc(const bn_frame *frames_host, int32_t n_frames,
                                                 const bn_params *params, void *stream) {
    if (!frames_host || n_frames < 1) return BN_ERR_INVALID_ARG;
    int rc = check_params_args(params);
    if (rc != BN_OK) return rc;
    if (n_frames > BN_NOALLOC_MAX_FRAMES) return BN_ERR_UNSUPPORTED;
    if (params->variant != VAR_AUTO) return BN_ERR_UNSUPPORTED;
    SmallKernelFn fn = small_kernel(params->method, params->alpha, params->scales);
    if (!fn) return BN_ERR_UNSUPPORTED;
    uint64_t tiles = 0, pixels = 0;
    rc = count_frames(frames_host, n_frames, params, &tiles, &pixels);
    if (rc != BN_OK) return rc;
    if (tiles == 0) return BN_OK;  // only empty frames
    WorkArea *work = nullptr;
    rc = scratch_for_current_device(&work);
    if (rc != BN_OK) return rc;
    SmallBatch sb;
    fill_small(sb, frames_host, n_frames, params, work);
    hipStream_t s = (hipStream_t)stream;
    // the work areas must start at zero: a fill kernel (graph-capture safe)
    const uint32_t words = (uint32_t)((size_t)n_frames * sizeof(WorkArea) / 8);
    hipLaunchKernelGGL(k_clear_words, dim3((words + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long *>(work), words);
    if (hipGetLastError() != hipSuccess) return BN_ERR_DEVICE;
    void *args[1] = {(void *)&sb};
    return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(sb.ntiles), dim3(kBlock), args,
                           0, s) == hipSuccess
               ? BN_OK
               : BN_ERR_DEVICE;
}
