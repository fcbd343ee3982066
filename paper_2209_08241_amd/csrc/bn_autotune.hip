// Autotuner: measured choice of the plain kernel's tile shape (variant:
// scalar or vector work items; 64, 128 or 256 threads per workgroup; one,
// two or four tiles per workgroup, or a software-pipelined pair) per (method,
// alpha, frame size class), and of the grid shape of batch plans (a flat
// grid of one, two or four tiles per workgroup, or 2, 4 or 8 persistent
// workgroups per compute unit).  Choices live in a process-wide table keyed by the GPU
// architecture name; the table can be saved to and loaded from a small JSON
// file, and is loaded from $BN_AUTOTUNE_CACHE on first use when that is set.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bn_internal.h"
#include "bnormals.h"

namespace bn {

namespace {

struct Entry {
    std::string arch;
    int kind;   // 0 plain, 1 batch
    int method;
    int alpha;
    int cls;    // bit length of the pixel count
    int value;  // variant id, or batch grid shape (-1, -2, -4 flat; k > 0 persistent)
    float us;
};

std::mutex g_mu;
std::vector<Entry> g_table;
bool g_env_loaded = false;

std::string current_arch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

int bit_length(uint64_t v) {
    int n = 0;
    while (v) {
        ++n;
        v >>= 1;
    }
    return n;
}

int load_locked(const char *path);

void ensure_env_loaded_locked() {
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char *p = std::getenv("BN_AUTOTUNE_CACHE");
    if (p && *p) (void)load_locked(p);
}

void put_locked(const Entry &e) {
    for (auto &x : g_table) {
        if (x.arch == e.arch && x.kind == e.kind && x.method == e.method && x.alpha == e.alpha &&
            x.cls == e.cls) {
            x = e;
            return;
        }
    }
    g_table.push_back(e);
}

const Entry *find_locked(const std::string &arch, int kind, int method, int alpha, int cls) {
    for (const auto &x : g_table)
        if (x.arch == arch && x.kind == kind && x.method == method && x.alpha == alpha &&
            x.cls == cls)
            return &x;
    return nullptr;
}

// Minimal reader for the file written by save_locked: one entry object per
// line, fields in a fixed order.
int load_locked(const char *path) {
    FILE *fh = std::fopen(path, "r");
    if (!fh) return BN_ERR_INVALID_ARG;
    char line[512];
    while (std::fgets(line, sizeof(line), fh)) {
        char arch[64], kind[16];
        int method, alpha, cls, value;
        float us;
        if (std::sscanf(line,
                        " {\"arch\": \"%63[^\"]\", \"kind\": \"%15[^\"]\", \"method\": %d, "
                        "\"alpha\": %d, \"class\": %d, \"value\": %d, \"us\": %f}",
                        arch, kind, &method, &alpha, &cls, &value, &us) == 7) {
            Entry e{arch, std::strcmp(kind, "batch") == 0 ? 1 : 0, method, alpha, cls, value, us};
            put_locked(e);
        }
    }
    std::fclose(fh);
    return BN_OK;
}

int save_locked(const char *path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *fh = std::fopen(tmp.c_str(), "w");
    if (!fh) return BN_ERR_INVALID_ARG;
    std::fprintf(fh, "{\"entries\": [\n");
    for (size_t i = 0; i < g_table.size(); ++i) {
        const Entry &e = g_table[i];
        std::fprintf(fh,
                     " {\"arch\": \"%s\", \"kind\": \"%s\", \"method\": %d, \"alpha\": %d, "
                     "\"class\": %d, \"value\": %d, \"us\": %.3f}%s\n",
                     e.arch.c_str(), e.kind ? "batch" : "plain", e.method, e.alpha, e.cls, e.value,
                     e.us,
                     i + 1 < g_table.size() ? "," : "");
    }
    std::fprintf(fh, "]}\n");
    std::fclose(fh);
    return std::rename(tmp.c_str(), path) == 0 ? BN_OK : BN_ERR_INVALID_ARG;
}

}  // namespace

int tuned_plain_variant(int method, int alpha, uint64_t pixels) {
    std::lock_guard<std::mutex> g(g_mu);
    ensure_env_loaded_locked();
    if (g_table.empty()) return 0;
    const Entry *e = find_locked(current_arch(), 0, method, alpha, bit_length(pixels));
    return e ? e->value : 0;
}

int tuned_batch_shape(int method, int alpha, uint64_t pixels) {
    std::lock_guard<std::mutex> g(g_mu);
    ensure_env_loaded_locked();
    if (g_table.empty()) return 0;
    const Entry *e = find_locked(current_arch(), 1, method, alpha, bit_length(pixels));
    return e ? e->value : 0;
}

void record_tuning(int kind, int method, int alpha, uint64_t pixels, int value, float us) {
    std::lock_guard<std::mutex> g(g_mu);
    ensure_env_loaded_locked();
    put_locked(Entry{current_arch(), kind, method, alpha, bit_length(pixels), value, us});
    const char *p = std::getenv("BN_AUTOTUNE_CACHE");
    if (p && *p) (void)save_locked(p);
}

}  // namespace bn

using namespace bn;

namespace {

// Timing frames with the cost structure of real scenes: a tilted, rippled
// surface 1.5 - 3 m away with step edges, depth noise growing as z^2 and 2%
// holes, so that every branch of each method is taken where it would be.
__global__ __launch_bounds__(256) void k_tune_scene(float *d, int32_t H, int32_t W,
                                                    uint32_t seed) {
    const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (i >= (uint64_t)H * (uint64_t)W) return;
    const uint32_t y = (uint32_t)(i / (uint32_t)W), x = (uint32_t)(i % (uint32_t)W);
    float z = 2.2f + 0.3f * __sinf(0.011f * (float)x + (float)seed) +
              0.2f * __cosf(0.017f * (float)y) + 0.0002f * (float)x;
    if ((x / 131u + y / 97u + seed) % 4u == 0u) z -= 0.6f;  // step edges
    uint32_t h = x * 0x9e3779b1u ^ (y + 0x7f4a7c15u * (seed + 1u)) * 0x85ebca77u;
    h ^= h >> 15;
    h *= 0x2c1b3c6du;
    h ^= h >> 12;
    // noise of spread 0.001 z^2 (sum of two uniforms, mean 0)
    const float u = (float)(h & 0xffffu) * (1.0f / 65536.0f) +
                    (float)((h >> 16) & 0x7fffu) * (1.0f / 32768.0f) - 1.0f;
    z += 0.001f * z * z * 1.7f * u;
    d[i] = (h % 50u == 7u) ? 0.0f : z;  // 2% holes
}

struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    void *alloc(size_t bytes) {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
};

}  // namespace

extern "C" {

int bn_autotune_plain(int32_t height, int32_t width, const bn_params *params, int32_t *best_variant,
                      float *best_us) {
    int rc = check_params_args(params);
    if (rc != BN_OK) return rc;
    if (height < 1 || width < 1 || width > BN_MAX_WIDTH ||
        (int64_t)height * width > BN_MAX_PIXELS)
        return BN_ERR_INVALID_ARG;
    const uint64_t px = (uint64_t)height * (uint64_t)width;
    // a ring of distinct frames of about 512 MiB, so that timings see HBM
    const uint64_t per = px * 17 + sizeof(bn_frame_stats);
    int ring = (int)((512ull << 20) / per);
    if (ring < 1) ring = 1;
    if (ring > 64) ring = 64;
    Scratch s;
    std::vector<float *> d(ring), n(ring);
    std::vector<uint8_t *> m(ring);
    bn_frame_stats *st = static_cast<bn_frame_stats *>(s.alloc(sizeof(bn_frame_stats) * ring));
    if (!st) return BN_ERR_OOM;
    for (int k = 0; k < ring; ++k) {
        d[k] = static_cast<float *>(s.alloc(px * 4));
        n[k] = static_cast<float *>(s.alloc(px * 12));
        m[k] = static_cast<uint8_t *>(s.alloc(px));
        if (!d[k] || !n[k] || !m[k]) return BN_ERR_OOM;
        hipLaunchKernelGGL(k_tune_scene, dim3((uint32_t)((px + 255) / 256)), dim3(256), 0,
                           nullptr, d[k], height, width, (uint32_t)k);
        if (hipGetLastError() != hipSuccess) return BN_ERR_DEVICE;
    }
    if (hipMemset(st, 0, sizeof(bn_frame_stats) * ring) != hipSuccess) return BN_ERR_DEVICE;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return BN_ERR_DEVICE;
    const float cx = 0.5f * (float)(width - 1), cy = 0.5f * (float)(height - 1);
    const float f = 525.0f * (float)width / 640.0f;
    // The library's default variant is kept unless another one is faster by
    // more than kMargin (choices within run-to-run noise would otherwise flip
    // between runs).
    constexpr float kMargin = 0.97f;
    const int dflt =
        default_plain_variant(params, px, vec4_layout(d[0], width, width, n[0], m[0]));
    int best = 0;
    float best_t = 1e30f, dflt_t = 1e30f;
    const int reps = ring * ((px < (1u << 20)) ? 8 : 3);
    for (int v = 1; v <= (int)VAR_COUNT; ++v) {
        bn_params p = *params;
        p.variant = (uint32_t)v;
        if (!bn_variant_supported(v, d[0], height, width, width, n[0], m[0])) continue;
        bool ok = true;
        for (int k = 0; k < ring && ok; ++k)  // warm-up
            ok = bn_estimate_normals(d[k], height, width, width, f, f, cx, cy, &p, n[k], m[k],
                                     st + k, nullptr) == BN_OK;
        if (!ok) continue;
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps; ++r) {
            const int k = r % ring;
            (void)bn_estimate_normals(d[k], height, width, width, f, f, cx, cy, &p, n[k], m[k],
                                      st + k, nullptr);
        }
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return BN_ERR_DEVICE;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const float us = 1000.f * ms / (float)reps;
        if (v == dflt) dflt_t = us;
        if (us < best_t) {
            best_t = us;
            best = v;
        }
    }
    if (best && best != dflt && dflt_t < 1e30f && best_t > kMargin * dflt_t) {
        best = dflt;
        best_t = dflt_t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!best) return BN_ERR_UNSUPPORTED;
    record_tuning(0, params->method, params->alpha, px, best, best_t);
    if (best_variant) *best_variant = best;
    if (best_us) *best_us = best_t;
    return BN_OK;
}

int bn_autotune_save(const char *path) {
    if (!path) return BN_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(g_mu);
    return save_locked(path);
}

int bn_autotune_load(const char *path) {
    if (!path) return BN_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(g_mu);
    g_env_loaded = true;
    return load_locked(path);
}

void bn_autotune_reset(void) {
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
    g_env_loaded = true;
}

int bn_autotune_entries(void) {
    std::lock_guard<std::mutex> g(g_mu);
    return (int)g_table.size();
}

}  // extern "C"
