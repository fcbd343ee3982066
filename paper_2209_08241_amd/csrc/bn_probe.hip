// Bandwidth probes: the HBM rates this GPU reaches for plain streaming
// traffic, as the achievable reference next to the 8 TB/s peak.
//   * a copy with 16-byte non-temporal loads and streaming device-scope
//     stores (the stores of the estimator's outputs);
//   * the estimator's traffic shape without its arithmetic: 16 bytes of
//     depth in per thread (4 pixels), 48 bytes of "normals" out through the
//     same LDS staging as the vector tiles (three contiguous KiB per
//     wavefront) and 4 bytes of "codes" out;
//   * the vector ALUs: independent binary32 multiply chains in registers.
#include "bn_internal.h"
#include "bn_probe.h"
#include "bn_tiles.h"
#include "bnormals.h"

namespace bn {
namespace {

__global__ __launch_bounds__(256) void k_stream_copy(const f4 *__restrict__ src,
                                                     f4 *__restrict__ dst, uint64_t n16) {
    const uint64_t b0 = (uint64_t)blockIdx.x * 256u;
    const uint64_t i = b0 + threadIdx.x;
    const uint32_t nb = n16 - b0 < 256u ? (uint32_t)(n16 - b0) : 256u;
    if (i < n16) out_store(__builtin_nontemporal_load(src + i), out_buf(dst + b0, 16u * nb),
                           16u * threadIdx.x);
}

__global__ __launch_bounds__(256) void k_stream_pattern(const f4 *__restrict__ depth,
                                                        f4 *__restrict__ normals,
                                                        uint32_t *__restrict__ mask) {
    __shared__ TileLds lds;
    const uint32_t t = threadIdx.x, lane = t & 63u, w = wave_id();
    const uint64_t i = (uint64_t)blockIdx.x * 256u + t;
    const f4 c = depth[i];
    out_store(__float_as_uint(c.x) & 0x01010101u,
              out_buf(mask + (uint64_t)blockIdx.x * 256u + 64u * w, 256u), 4u * lane);
    f4 *slice = lds.v + 192 * w;
    wave_lds_sync();
    slice[3 * lane + 0] = c;
    slice[3 * lane + 1] = c * 2.0f;
    slice[3 * lane + 2] = c * 3.0f;
    wave_lds_sync();
    const OutBuf nb = out_buf(normals + 3 * ((uint64_t)blockIdx.x * 256u + 64u * w), 3072u);
    out_store(slice[lane], nb, 16u * lane);
    out_store(slice[64 + lane], nb, 16u * lane + 1024u);
    out_store(slice[128 + lane], nb, 16u * lane + 2048u);
}

// Eight independent chains keep every SIMD's issue slot busy at 8 wavefronts
// per SIMD (a multiply's result is not needed for the next 7 instructions).
__global__ __launch_bounds__(256) void k_alu_chain(float *__restrict__ out, float m,
                                                   uint32_t iters) {
    float x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = 1.0f + 1e-3f * (float)(threadIdx.x + c);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = x[c] * m;
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s = s + x[c];
    out[(uint64_t)blockIdx.x * 256u + threadIdx.x] = s;
}

}  // namespace
}  // namespace bn

using namespace bn;

extern "C" {

int bn_stream_copy(void *dst, const void *src, uint64_t bytes, void *stream) {
    if (bytes % 16 || (uintptr_t)dst % 16 || (uintptr_t)src % 16) return BN_ERR_INVALID_ARG;
    if (bytes == 0) return BN_OK;
    if (!dst || !src) return BN_ERR_INVALID_ARG;
    const uint64_t n16 = bytes / 16;
    const uint64_t blocks = (n16 + 255) / 256;
    if (blocks > 0xffffffffull) return BN_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_stream_copy, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const f4 *>(src), static_cast<f4 *>(dst), n16);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

int bn_stream_pattern(const float *depth, float *normals, uint8_t *mask, uint64_t pixels,
                      void *stream) {
    if (pixels % 1024 || (uintptr_t)depth % 16 || (uintptr_t)normals % 16 || (uintptr_t)mask % 4)
        return BN_ERR_INVALID_ARG;
    if (pixels == 0) return BN_OK;
    if (!depth || !normals || !mask) return BN_ERR_INVALID_ARG;
    const uint64_t blocks = pixels / 1024;
    if (blocks > 0xffffffffull) return BN_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_stream_pattern, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const f4 *>(depth), reinterpret_cast<f4 *>(normals),
                       reinterpret_cast<uint32_t *>(mask));
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

int bn_alu_probe(float *out, uint32_t workgroups, uint32_t iters, float m, void *stream) {
    if (workgroups == 0) return BN_OK;
    if (!out || (uintptr_t)out % 4) return BN_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_alu_chain, dim3(workgroups), dim3(256), 0, (hipStream_t)stream, out, m,
                       iters);
    return hipGetLastError() == hipSuccess ? BN_OK : BN_ERR_DEVICE;
}

}  // extern "C"
