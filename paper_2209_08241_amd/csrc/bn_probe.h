// Bandwidth probes: what this GPU's HBM delivers to plain streaming kernels,
// the achievable rate next to the published peak.  Measurement helpers, not
// part of the estimator's interface (include/bnormals.h): the benchmark and
// its probe test call them through the library's exported symbols.  Device
// pointers, asynchronous on `stream`, nothing allocated.
//   bn_stream_copy: bytes (a multiple of 16, 16-byte aligned buffers) from
//     src to dst with 16-byte non-temporal loads and stores.
//   bn_stream_pattern: the estimator's traffic without its arithmetic: reads
//     4 B of depth and writes 12 B of normals and 1 B of code per pixel
//     through the same LDS staging; pixels a multiple of 1024, depth and
//     normals 16-byte and mask 4-byte aligned.  Output values are
//     meaningless.
#pragma once

#include <stdint.h>

extern "C" {
int bn_stream_copy(void *dst, const void *src, uint64_t bytes, void *stream);
int bn_stream_pattern(const float *depth, float *normals, uint8_t *mask, uint64_t pixels,
                      void *stream);
}
