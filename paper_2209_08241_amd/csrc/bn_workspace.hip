// Count work areas of the single-frame and stack calls.
//
// The per-frame counts are reduced inside the launch on device words that
// must be zero when the launch starts (the reduction leaves them zero again).
// Those words belong to the library, not to the caller's 16-byte
// bn_frame_stats: one set of BN_MAX_STACK work areas per (device, stream),
// taken from a pool in device memory that each device holds from the
// library's first use until the process ends.  Launches on one stream run
// one after another, so they can share the stream's set; launches on
// distinct streams get distinct sets.  Streams are told apart by their
// handle.  When every set of a device is taken, the next new stream waits
// for the whole device (outside graph capture) and the sets are handed out
// afresh: every launch that used them has then completed.
#include <map>
#include <mutex>
#include <utility>

#include "bn_internal.h"

namespace bn {
namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kSetAreas = BN_MAX_STACK;  // one area per frame of a stack

// BN_MAX_STREAMS sets of kSetAreas work areas (17.3 MB); each set is zeroed
// on the stream it is given to before that stream's first launch uses it.
__device__ __align__(256) WorkArea g_pool[BN_MAX_STREAMS * kSetAreas];

std::mutex g_mu;
WorkArea *g_base[kMaxDevices];                          // g_pool's address on each device
std::map<std::pair<int, uintptr_t>, int> g_set_of;      // (device, stream) -> set
int g_sets_used[kMaxDevices];

__global__ __launch_bounds__(256) void k_zero_set(unsigned long long *p, uint32_t words) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < words) p[i] = 0ull;
}

}  // namespace

int stream_work_areas(hipStream_t stream, WorkArea **out) {
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BN_ERR_DEVICE;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_base[dev]) {
        // the array's name is a host-side stand-in: the device address comes
        // from the runtime, per device, with that device current
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_pool)) != hipSuccess || !p) return BN_ERR_DEVICE;
        g_base[dev] = static_cast<WorkArea *>(p);
    }
    const auto key = std::make_pair(dev, (uintptr_t)stream);
    const auto it = g_set_of.find(key);
    if (it != g_set_of.end()) {
        *out = g_base[dev] + (size_t)it->second * kSetAreas;
        return BN_OK;
    }
    if (g_sets_used[dev] >= BN_MAX_STREAMS) {
        // every set is taken: once the device is idle, none is in use
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return BN_ERR_DEVICE;
        if (cs != hipStreamCaptureStatusNone) return BN_ERR_UNSUPPORTED;
        if (hipDeviceSynchronize() != hipSuccess) return BN_ERR_DEVICE;
        for (auto e = g_set_of.begin(); e != g_set_of.end();) {
            if (e->first.first == dev) {
                e = g_set_of.erase(e);
            } else {
                ++e;
            }
        }
        g_sets_used[dev] = 0;
    }
    WorkArea *set = g_base[dev] + (size_t)g_sets_used[dev] * kSetAreas;
    // zero the set on its stream, ahead of the launch that will use it (a
    // fill kernel, so that a graph captured from this stream replays it
    // correctly)
    const uint32_t words = (uint32_t)(kSetAreas * sizeof(WorkArea) / 8);
    hipLaunchKernelGGL(k_zero_set, dim3((words + 255) / 256), dim3(256), 0, stream,
                       reinterpret_cast<unsigned long long *>(set), words);
    if (hipGetLastError() != hipSuccess) return BN_ERR_DEVICE;
    g_set_of.emplace(key, g_sets_used[dev]++);
    *out = set;
    return BN_OK;
}

}  // namespace bn
