// Bandwidth probes: what this GPU's HBM delivers to plain streaming kernels,
// the achievable rate next to the published peak.  Measurement helpers, not
// part of the estimator's interface (include/bnormals.h): the benchmark and
// its probe test call them through the library's exported symbols.  Device
// pointers, asynchronous on `stream`, nothing allocated.
//   bn_stream_copy: bytes (a multiple of 16, 16-byte aligned buffers) from
//     src to dst with 16-byte non-temporal loads and the estimator's
//     streaming device-scope stores.
//   bn_stream_pattern: the estimator's traffic without its arithmetic: reads
//     4 B of depth and writes 12 B of normals and 1 B of code per pixel
//     through the same LDS staging and stores; pixels a multiple of 1024, depth and
//     normals 16-byte and mask 4-byte aligned.  Output values are
//     meaningless.
//   bn_alu_probe: the vector ALUs' issue rate for unpacked binary32
//     instructions: each of workgroups x 256 threads runs 8 independent
//     chains x <- x * m of `iters` steps (8 iters multiplies, no memory
//     traffic in the loop) and writes the sum of its chains to out[thread]
//     (out holds workgroups x 256 floats).  Chain c of thread t starts at
//     1 + 1e-3 (t % 256 + c).
#pragma once

#include <stdint.h>

extern "C" {
int bn_stream_copy(void *dst, const void *src, uint64_t bytes, void *stream);
int bn_stream_pattern(const float *depth, float *normals, uint8_t *mask, uint64_t pixels,
                      void *stream);
int bn_alu_probe(float *out, uint32_t workgroups, uint32_t iters, float m, void *stream);
}
