// Batched execution: every tile of every frame of a batch in one launch of
// a persistent kernel, instantiated once as a HIP graph.
//
// Frames of different sizes are cut into tiles of 256 work items (1024
// pixels for vector frames).  The grid is sized to the machine (8 workgroups
// per compute unit, all resident at once); workgroup b owns the contiguous
// tile range [b*chunk, (b+1)*chunk) of the concatenated tile sequence, so the
// load is balanced whatever the frame mix, a workgroup touches few frames
// (one count reduction per frame segment), and - through the XCD-contiguous
// numbering of workgroups - neighbouring tiles, which share stencil rows,
// are processed by the same XCD.  The frame descriptors live in device
// memory, so a plan's graph is replayed unchanged when the frames change.
#include <cmath>
#include <cstring>
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

// Index of the frame that holds tile t: the last frame whose tile_begin is
// <= t (frames without tiles share their tile_begin with the next frame).
__device__ __forceinline__ uint32_t find_frame(const BatchFrame *fr, uint32_t nf, uint32_t t) {
    uint32_t lo = 0, hi = nf;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (fr[mid].tile_begin <= t)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <int A>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchHeader *__restrict__ hdr,
                                                  const BatchFrame *__restrict__ frames) {
    __shared__ TileLds lds;
    const uint32_t T = hdr->ntiles;
    const uint32_t c = hdr->chunk;
    const uint32_t nf = hdr->nframes;
    const uint32_t blk = xcd_tile(blockIdx.x, gridDim.x);
    uint32_t t = blk * c;
    if (c == 0 || t >= T) return;  // uniform: this workgroup has no tiles
    const uint32_t tend = min(t + c, T);
    uint32_t fi = find_frame(frames, nf, t);
    bool first = true;
    while (t < tend && fi < nf) {
        const FrameArgs f = frames[fi].a;
        const uint32_t tb = frames[fi].tile_begin;
        const uint32_t nt = frames[fi].ntiles;
        const bool vec = frames[fi].vec != 0;
        const uint32_t seg_end = min(tend, tb + nt);
        uint32_t cv = 0, cb = 0;
        for (; t < seg_end; ++t) {
            if (!first) __syncthreads();  // LDS reuse
            first = false;
            run_tile<A>(f, vec, t - tb, lds, cv, cb);
        }
        if (f.stats) {
            // the frame's parts are the workgroups whose chunks meet it
            const uint32_t b_first = tb / c;
            const uint32_t b_last = (tb + nt - 1) / c;
            block_counts(f.stats, blk - b_first, b_last - b_first + 1, cv, cb, f.npix);
        }
        do {
            ++fi;
        } while (fi < nf && frames[fi].ntiles == 0);
    }
}

typedef void (*BatchKernelFn)(const BatchHeader *, const BatchFrame *);

static BatchKernelFn batch_kernel(int alpha) {
    switch (alpha) {
        case 1: return k_batch<1>;
        case 2: return k_batch<2>;
        case 3: return k_batch<3>;
        case 4: return k_batch<4>;
        case 5: return k_batch<5>;
        case 6: return k_batch<6>;
        case 7: return k_batch<7>;
        case 8: return k_batch<8>;
    }
    return nullptr;
}

}  // namespace bn

using namespace bn;

struct bn_batch_plan {
    int device = -1;
    bn_params params{};
    int32_t capacity = 0;
    uint32_t grid = 0;
    void *dbuf = nullptr;            // BatchHeader followed by BatchFrame[capacity]
    size_t table_bytes = 0;
    void *staging[2] = {nullptr, nullptr};  // pinned host copies for updates
    hipEvent_t staged[2] = {nullptr, nullptr};
    int next = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t total_tiles = 0;
    uint64_t total_pixels = 0;
};

namespace {

constexpr uint32_t kBlocksPerCU = 8;

// Host image of the descriptor table for `frames`; returns a bn status.
int build_table(const bn_frame *frames, int32_t n, const bn_params *p, uint32_t grid,
                void *out, uint64_t *tiles_out, uint64_t *pixels_out) {
    auto *hdr = static_cast<BatchHeader *>(out);
    auto *fr = reinterpret_cast<BatchFrame *>(hdr + 1);
    uint64_t tiles = 0, pixels = 0;
    for (int32_t k = 0; k < n; ++k) {
        const bn_frame &s = frames[k];
        int rc = check_frame_args(s.depth, s.height, s.width, s.depth_stride, s.fx, s.fy, s.cx,
                                  s.cy, s.normals, s.mask);
        if (rc != BN_OK) return rc;
        const bool vec = vec4_layout(s.depth, s.width, s.depth_stride, s.normals, s.mask);
        BatchFrame b;
        std::memset(&b, 0, sizeof(b));
        if (s.height > 0 && s.width > 0) {
            fill_frame_args(b.a, s.depth, s.height, s.width, s.depth_stride, s.fx, s.fy, s.cx,
                            s.cy, p, s.normals, s.mask, s.stats, vec ? 4 : 1);
        }
        const uint64_t nt = (s.height > 0 && s.width > 0)
                                ? ((uint64_t)b.a.nitems + kBlock - 1) / kBlock
                                : 0;
        b.tile_begin = (uint32_t)tiles;
        b.ntiles = (uint32_t)nt;
        b.vec = vec ? 1u : 0u;
        tiles += nt;
        pixels += (uint64_t)s.height * (uint64_t)s.width;
        if (tiles > 0xFFF00000ull) return BN_ERR_UNSUPPORTED;
        fr[k] = b;
    }
    hdr->nframes = (uint32_t)n;
    hdr->ntiles = (uint32_t)tiles;
    hdr->chunk = tiles ? (uint32_t)((tiles + grid - 1) / grid) : 0;
    hdr->pad = 0;
    if (hdr->chunk > 4096) return BN_ERR_UNSUPPORTED;  // parts stay below 2^22 pixels
    *tiles_out = tiles;
    *pixels_out = pixels;
    return BN_OK;
}

void free_plan(bn_batch_plan *pl) {
    if (!pl) return;
    for (int k = 0; k < 2; ++k) {
        if (pl->staged[k]) {
            (void)hipEventSynchronize(pl->staged[k]);
            (void)hipEventDestroy(pl->staged[k]);
        }
        if (pl->staging[k]) (void)hipHostFree(pl->staging[k]);
    }
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->dbuf) (void)hipFree(pl->dbuf);
    delete pl;
}

}  // namespace

extern "C" {

int bn_batch_plan_create(const bn_frame *frames_host, int32_t n_frames, const bn_params *params,
                         bn_batch_plan **out_plan) {
    if (!out_plan) return BN_ERR_INVALID_ARG;
    *out_plan = nullptr;
    if (!frames_host || n_frames < 1) return BN_ERR_INVALID_ARG;
    int rc = check_params_args(params);
    if (rc != BN_OK) return rc;
    if (params->variant != VAR_AUTO) return BN_ERR_UNSUPPORTED;
    BatchKernelFn fn = batch_kernel(params->alpha);
    if (!fn) return BN_ERR_UNSUPPORTED;

    bn_batch_plan *pl = new (std::nothrow) bn_batch_plan();
    if (!pl) return BN_ERR_OOM;
    pl->params = *params;
    pl->capacity = n_frames;
    if (hipGetDevice(&pl->device) != hipSuccess) {
        free_plan(pl);
        return BN_ERR_DEVICE;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) !=
            hipSuccess ||
        cus <= 0)
        cus = 256;
    pl->grid = (uint32_t)cus * kBlocksPerCU;
    pl->table_bytes = sizeof(BatchHeader) + sizeof(BatchFrame) * (size_t)n_frames;

    for (int k = 0; k < 2; ++k) {
        if (hipHostMalloc(&pl->staging[k], pl->table_bytes, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&pl->staged[k], hipEventDisableTiming) != hipSuccess) {
            free_plan(pl);
            return BN_ERR_OOM;
        }
    }
    rc = build_table(frames_host, n_frames, params, pl->grid, pl->staging[0], &pl->total_tiles,
                     &pl->total_pixels);
    if (rc != BN_OK) {
        free_plan(pl);
        return rc;
    }
    if (hipMalloc(&pl->dbuf, pl->table_bytes) != hipSuccess) {
        free_plan(pl);
        return BN_ERR_OOM;
    }
    if (hipMemcpy(pl->dbuf, pl->staging[0], pl->table_bytes, hipMemcpyHostToDevice) !=
        hipSuccess) {
        free_plan(pl);
        return BN_ERR_DEVICE;
    }

    // one kernel node: the persistent launch over the whole batch
    const BatchHeader *d_hdr = static_cast<const BatchHeader *>(pl->dbuf);
    const BatchFrame *d_frames = reinterpret_cast<const BatchFrame *>(d_hdr + 1);
    void *args[2] = {(void *)&d_hdr, (void *)&d_frames};
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = reinterpret_cast<void *>(fn);
    kp.gridDim = dim3(pl->grid);
    kp.blockDim = dim3(kBlock);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    if (hipGraphCreate(&pl->graph, 0) != hipSuccess ||
        hipGraphAddKernelNode(&node, pl->graph, nullptr, 0, &kp) != hipSuccess ||
        hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess) {
        free_plan(pl);
        return BN_ERR_DEVICE;
    }
    *out_plan = pl;
    return BN_OK;
}

int bn_batch_plan_update(bn_batch_plan *plan, const bn_frame *frames_host, int32_t n_frames,
                         void *stream) {
    if (!plan || !frames_host || n_frames < 1) return BN_ERR_INVALID_ARG;
    if (n_frames > plan->capacity) return BN_ERR_UNSUPPORTED;
    const int k = plan->next;
    // the staging buffer may still feed the copy issued two updates ago
    if (hipEventSynchronize(plan->staged[k]) != hipSuccess) return BN_ERR_DEVICE;
    uint64_t tiles = 0, pixels = 0;
    int rc = build_table(frames_host, n_frames, &plan->params, plan->grid, plan->staging[k],
                         &tiles, &pixels);
    if (rc != BN_OK) return rc;
    const size_t bytes = sizeof(BatchHeader) + sizeof(BatchFrame) * (size_t)n_frames;
    if (hipMemcpyAsync(plan->dbuf, plan->staging[k], bytes, hipMemcpyHostToDevice,
                       (hipStream_t)stream) != hipSuccess ||
        hipEventRecord(plan->staged[k], (hipStream_t)stream) != hipSuccess)
        return BN_ERR_DEVICE;
    plan->next = 1 - k;
    plan->total_tiles = tiles;
    plan->total_pixels = pixels;
    return BN_OK;
}

int bn_batch_run(bn_batch_plan *plan, void *stream) {
    if (!plan || !plan->exec) return BN_ERR_INVALID_ARG;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

int bn_batch_plan_info(const bn_batch_plan *plan, int64_t *n_pixels, int64_t *n_tiles,
                       int32_t *n_workgroups) {
    if (!plan) return BN_ERR_INVALID_ARG;
    if (n_pixels) *n_pixels = (int64_t)plan->total_pixels;
    if (n_tiles) *n_tiles = (int64_t)plan->total_tiles;
    if (n_workgroups) *n_workgroups = (int32_t)plan->grid;
    return BN_OK;
}

void bn_batch_plan_destroy(bn_batch_plan *plan) { free_plan(plan); }

}  // extern "C"
