// Tile bodies shared by the plain and the batched kernels.
//
// A tile is kBlock = 256 consecutive work items of one frame, one per
// thread: 4 consecutive pixels of a row (vector tiles, width % 4 == 0 and
// 16-byte aligned rows) or 1 pixel (scalar tiles, any layout).  Each
// wavefront stages the normals of its 64 work items in its own slice of LDS
// and writes them back with contiguous stores: a wavefront's LDS accesses
// execute in program order, so no workgroup barrier is needed - a barrier
// would also carry a release fence that waits for the previous tile's
// global stores, serialising the tiles of a persistent workgroup.
#pragma once

#include "bn_device.h"

#pragma clang fp contract(off)

namespace bn {

// LDS staging area of one tile of TB work items: 3 float4 (12 floats) per
// vector work item, or 3 floats per scalar work item; wavefront w owns
// v[192w .. 192w+191].  Tiles are kBlock = 256 work items except in the
// plain kernels' smaller-workgroup variants (TB = 64 or 128).
template <int TB = kBlock>
struct TileLdsT {
    f4 v[3 * TB];
};
using TileLds = TileLdsT<kBlock>;

// Orders this wavefront's LDS accesses for the compiler; the hardware
// already executes them in order.  Emits no wait instruction.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int A>
struct Win {
    static constexpr int R = (A + 3) / 4;  // float4s needed on each side
    static constexpr int N = 4 * (2 * R + 1);
};

// ---------------------------------------------------------------------------
// Vector tile, first half: evaluate the group of thread threadIdx.x (pixels
// 4i .. 4i+3 of the frame, i = tile*256 + t) into registers.  Every lane of
// the workgroup must call this (DPP lane shifts).
// ---------------------------------------------------------------------------
struct Vec4Out {
    float nv[12];
    uint32_t codes;  // one per byte
    bool live;
};

// Methods whose tile writes each pixel's normal into the wavefront's LDS
// slice as soon as it is computed, instead of holding the 12 floats of the
// thread's four pixels in registers until the stores (pair removal: its
// per-pixel working set would otherwise push the kernel past 64 VGPRs, below
// eight wavefronts per SIMD).
template <int M>
constexpr bool kEarlyStage = M == kPairRemoval;

// The loads of a vector work item, kept apart from its arithmetic so that a
// workgroup can issue one tile's loads before another tile's arithmetic.
// edge[k]: lane 0's float4 k to the left of the wavefront's row segment,
// lane 63's float4 k to the right (other lanes: unused).
template <int A>
struct Vec4In {
    f4 c, up, dn;
    f4 edge[Win<A>::R];
    uint32_t y, x0;
    bool live, rows_in;
};

template <int A, int TB = kBlock>
__device__ __forceinline__ void vec4_load(const FrameArgs &f, uint32_t tile, Vec4In<A> &in) {
    constexpr int R = Win<A>::R;
    const uint32_t t = threadIdx.x;
    const uint32_t lane = t & 63u;
    const uint32_t i = tile * TB + t;
    const bool live = i < f.nitems;
    in.live = live;
    // Every load is unconditional: a lane past the frame's last item takes
    // the last item's position, and a row A above or below that leaves the
    // frame is replaced by row y itself.  What such a load brings in only
    // reaches pixels that are not inside (or not live), whose codes are
    // INVALID whatever it holds.
    const uint32_t il = live ? i : f.nitems - 1u;
    const uint32_t y = row_of(il, f.inv_gpr);
    const uint32_t x0 = (il - y * f.gpr) * 4u;
    in.y = y;
    in.x0 = x0;
    const float *rp = f.depth + (int64_t)y * f.stride;
    in.rows_in = live & (y >= (uint32_t)A) & (y + A < (uint32_t)f.H);
    const int64_t su = y >= (uint32_t)A ? (int64_t)A * f.stride : 0;
    const int64_t sd = y + A < (uint32_t)f.H ? (int64_t)A * f.stride : 0;
    in.c = *reinterpret_cast<const f4 *>(rp + x0);
    in.up = *reinterpret_cast<const f4 *>(rp - su + x0);
    in.dn = *reinterpret_cast<const f4 *>(rp + sd + x0);
    // the first / last lane of the wave loads the float4s its neighbours
    // cannot pass it (clamped into the row)
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        in.edge[k - 1] = f4{0.f, 0.f, 0.f, 0.f};
        if (lane == 0) in.edge[k - 1] = *reinterpret_cast<const f4 *>(rp + max((int)x0 - 4 * k, 0));
        if (lane == 63)
            in.edge[k - 1] = *reinterpret_cast<const f4 *>(rp + min((int)x0 + 4 * k, f.W - 4));
    }
}

// The arithmetic of a vector work item from its loads.  Every lane of the
// workgroup must call this (DPP lane shifts).
template <int A, int M, int TB = kBlock>
__device__ __forceinline__ void vec4_compute(const FrameArgs &f, const Vec4In<A> &in, Vec4Out &o,
                                             TileLdsT<TB> &lds) {
    constexpr int R = Win<A>::R;
    const uint32_t t = threadIdx.x;
    const uint32_t lane = t & 63u;
    o.live = in.live;
    const uint32_t y = in.y, x0 = in.x0;
    const f4 c = in.c, up = in.up, dn = in.dn;
    // Row window x0-4R .. x0+4+4R-1.  Neighbouring float4s come from the
    // adjacent lanes; the first / last lane of the wave takes its loaded
    // edge.  Values taken across a row end only feed border pixels, which
    // are INVALID whatever they hold.
    float row[Win<A>::N];
    row[4 * R + 0] = c.x;
    row[4 * R + 1] = c.y;
    row[4 * R + 2] = c.z;
    row[4 * R + 3] = c.w;
    f4 lk = c, rk = c;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lk = from_left(lk);
        rk = from_right(rk);
        if (lane == 0) lk = in.edge[k - 1];
        if (lane == 63) rk = in.edge[k - 1];
        row[4 * (R - k) + 0] = lk.x;
        row[4 * (R - k) + 1] = lk.y;
        row[4 * (R - k) + 2] = lk.z;
        row[4 * (R - k) + 3] = lk.w;
        row[4 * (R + k) + 0] = rk.x;
        row[4 * (R + k) + 1] = rk.y;
        row[4 * (R + k) + 2] = rk.z;
        row[4 * (R + k) + 3] = rk.w;
    }
    const float upv[4] = {up.x, up.y, up.z, up.w};
    const float dnv[4] = {dn.x, dn.y, dn.z, dn.w};
    const float yc = (float)y - f.cy;
    uint32_t codes = 0;
    // early staging: this lane's 12 floats of the wavefront's LDS slice
    float *st = reinterpret_cast<float *>(lds.v + 192 * (t >> 6)) + 12 * lane;
    if (kEarlyStage<M>) wave_lds_sync();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t x = x0 + j;
        const bool inside = in.rows_in & (x >= (uint32_t)A) & (x + A < (uint32_t)f.W);
        const float xc = (float)x - f.cx;
        const int cI = 4 * R + j;
        const PixelOut p = eval_method<M>(inside, row[cI], row[cI + A], dnv[j], row[cI - A],
                                          upv[j], xc, yc, f);
        if (kEarlyStage<M>) {
            st[3 * j + 0] = p.nx;
            st[3 * j + 1] = p.ny;
            st[3 * j + 2] = p.nz;
        } else {
            o.nv[3 * j + 0] = p.nx;
            o.nv[3 * j + 1] = p.ny;
            o.nv[3 * j + 2] = p.nz;
        }
        codes |= p.code << (8 * j);
    }
    o.codes = codes;
}

template <int A, int M, int TB = kBlock>
__device__ __forceinline__ void vec4_eval(const FrameArgs &f, uint32_t tile, Vec4Out &o,
                                          TileLdsT<TB> &lds) {
    Vec4In<A> in;
    vec4_load<A, TB>(f, tile, in);
    vec4_compute<A, M, TB>(f, in, o, lds);
}

// Multi-scale vector tile (alpha * scales <= REACH): the taps lie right of and
// below each pixel, so the row window extends to the right only and the
// vertical taps are the float4s of rows y + i alpha.  Same arithmetic per
// scale as the scalar tile.
template <int A, int REACH>
__device__ __forceinline__ void vec4_eval_ms(const FrameArgs &f, uint32_t tile, Vec4Out &o) {
    constexpr int KMAX = REACH / A < BN_MAX_SCALES ? REACH / A : BN_MAX_SCALES;
    constexpr int RR = (A * KMAX + 3) / 4;  // float4s needed on the right
    const uint32_t t = threadIdx.x;
    const uint32_t lane = t & 63u;
    const uint32_t i = tile * kBlock + t;
    const bool live = i < f.nitems;
    o.live = live;
    // Every load is unconditional and in the frame: a lane past the last item
    // takes the last item's position, a lane whose taps below leave the frame
    // reads them from rows that are in it, and the right-hand float4s are
    // clamped into the row.  What such a load brings in only reaches pixels
    // that are not inside (or not live), whose codes are INVALID whatever it
    // holds.  (Conditional loads had to zero their registers first, and the
    // compiler waited for the centre load before issuing the rows below.)
    const uint32_t il = live ? i : f.nitems - 1u;
    const uint32_t y = row_of(il, f.inv_gpr);
    const uint32_t x0 = (il - y * f.gpr) * 4u;
    const int K = f.scales;
    const uint32_t reach = (uint32_t)(K * A);
    const float *rp = f.depth + (int64_t)y * f.stride;
    const bool rows_in = live & (y + reach < (uint32_t)f.H);
    const f4 c = *reinterpret_cast<const f4 *>(rp + x0);
    // The rows below: from row y, or, where they would leave the frame, from
    // the last rows that keep all K in it.  On a frame no taller than the
    // reach no pixel is inside, and every "row below" is row y itself.
    const bool fits = reach < (uint32_t)f.H;
    const int64_t rstep = fits ? (int64_t)A * f.stride : 0;
    const uint32_t yb = (fits && !rows_in) ? (uint32_t)f.H - 1u - reach : y;
    const float *bp = f.depth + (int64_t)yb * f.stride + x0;
    f4 dn[KMAX];
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        if (s < K) dn[s] = *reinterpret_cast<const f4 *>(bp + (int64_t)(s + 1) * rstep);
    }
    // The row window to the right: float4 k of lane l is lane l+k's centre;
    // lane 63 loads its own (clamped into the row) before any lane shift, so
    // that no shift waits for a load issued after the rows below.
    f4 edge[RR];
#pragma unroll
    for (int k = 1; k <= RR; ++k) {
        if (lane == 63)
            edge[k - 1] = *reinterpret_cast<const f4 *>(rp + min((int)x0 + 4 * k, f.W - 4));
    }
    float row[4 * (RR + 1)];
    row[0] = c.x;
    row[1] = c.y;
    row[2] = c.z;
    row[3] = c.w;
    f4 rk = c;
#pragma unroll
    for (int k = 1; k <= RR; ++k) {
        rk = from_right(rk);
        if (lane == 63) rk = edge[k - 1];
        row[4 * k + 0] = rk.x;
        row[4 * k + 1] = rk.y;
        row[4 * k + 2] = rk.z;
        row[4 * k + 3] = rk.w;
    }
    const float yc = (float)y - f.cy;
    uint32_t codes = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t x = x0 + j;
        const bool inside = rows_in & (x + reach < (uint32_t)f.W);
        const float xc = (float)x - f.cx;
        const float d1 = row[j];
        uint32_t ok = (inside ? 1u : 0u) & tap_ok(d1);
        float Mx = 0.0f, My = 0.0f, Mz = 0.0f, Wt = 0.0f;
#pragma unroll
        for (int s = 0; s < KMAX; ++s) {
            if (s < K) {
                const float d2 = row[j + (s + 1) * A];
                const float dv[4] = {dn[s].x, dn[s].y, dn[s].z, dn[s].w};
                const float d3 = dv[j];
                ok &= tap_ok(d2) & tap_ok(d3);
                ms_accumulate(d1, d2, d3, (float)((s + 1) * A), xc, yc, f, Mx, My, Mz, Wt);
            }
        }
        const PixelOut p = ms_finish(ok, Mx, My, Mz, Wt, f);
        o.nv[3 * j + 0] = p.nx;
        o.nv[3 * j + 1] = p.ny;
        o.nv[3 * j + 2] = p.nz;
        codes |= p.code << (8 * j);
    }
    o.codes = codes;
}

// The vector tile of method M.
template <int A, int M>
__device__ __forceinline__ void vec4_eval_method(const FrameArgs &f, uint32_t tile, Vec4Out &o,
                                                 TileLds &lds) {
    if constexpr (is_multiscale(M)) {
        vec4_eval_ms<A, M == kMultiScaleLong ? kMsVecReach : kMsShortReach>(f, tile, o);
    } else {
        vec4_eval<A, M>(f, tile, o, lds);
    }
}

// Vector tile, second half: the four codes with one 32-bit store, the 12
// normal floats through the wavefront's LDS slice with contiguous 16-byte
// stores (lane l holds groups 3l..3l+2 of the slice; store k writes
// float4s 64k .. 64k+63 of it, one contiguous KiB).  The stores stream at
// device scope (out_store); the wavefront's share of the frame bounds them,
// so the lanes past the frame's last work item store nothing.
template <int M, int TB = kBlock>
__device__ __forceinline__ void vec4_write(const FrameArgs &f, uint32_t tile, TileLdsT<TB> &lds,
                                           const Vec4Out &o) {
    const uint32_t t = threadIdx.x;
    const uint32_t lane = t & 63u;
    const float *nv = o.nv;
    const uint32_t w = wave_id();
    const uint32_t g0 = tile * TB + 64 * w;  // first work item of this wavefront
    // A wavefront past the frame's end has a resource of size 0, which
    // drops every store.  The stores are unconditional, so a count ticket
    // issued before them is waited for by its own position in the counter
    // (loads, stores and atomics complete in issue order), not by a wait for
    // all of them.
    const uint32_t ng = g0 < f.nitems ? min(64u, f.nitems - g0) : 0u;
    {
        const OutBuf mb = out_buf(reinterpret_cast<uint32_t *>(f.mask) + g0, 4 * ng);
        out_store(o.codes, mb, 4 * lane);
    }
    f4 *slice = lds.v + 192 * w;
    if (!kEarlyStage<M>) {
        wave_lds_sync();
        slice[3 * lane + 0] = f4{nv[0], nv[1], nv[2], nv[3]};
        slice[3 * lane + 1] = f4{nv[4], nv[5], nv[6], nv[7]};
        slice[3 * lane + 2] = f4{nv[8], nv[9], nv[10], nv[11]};
    }
    wave_lds_sync();
    {
        const OutBuf nb = out_buf(reinterpret_cast<f4 *>(f.normals) + 3 * (int64_t)g0, 48 * ng);
#pragma unroll
        for (int k = 0; k < 3; ++k) out_store(slice[64 * k + lane], nb, 16 * lane + 1024 * k);
    }
}

// Ballots of the compares and a scalar AND with the live lanes.
__device__ __forceinline__ void vec4_count(const Vec4Out &o, uint32_t &cv, uint32_t &cb) {
    const uint64_t lm = __builtin_amdgcn_ballot_w64(o.live);
    const uint32_t codes = o.codes;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t c = (codes >> (8 * j)) & 0xffu;
        cv += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(c == BN_VALID) & lm);
        cb += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(c == BN_BOUNDARY) &
                                             lm);
    }
}

// ---------------------------------------------------------------------------
// Scalar tile: pixel i = tile*256 + t, any stride and alignment; outputs
// written like the vector tile's.
// ---------------------------------------------------------------------------
struct ScalarOut {
    float nx, ny, nz;
    uint32_t code;
    bool live;
};

template <int A, int M>
__device__ __forceinline__ void scalar_eval(const FrameArgs &f, uint32_t tile, ScalarOut &r) {
    const uint32_t i = tile * kBlock + threadIdx.x;
    const bool live = i < f.nitems;
    r.live = live;
    uint32_t code = BN_INVALID;
    float nx = 0.f, ny = 0.f, nz = 0.f;
    if (is_multiscale(M) && live) {
        const uint32_t y = row_of(i, f.inv_gpr);
        const uint32_t x = i - y * f.gpr;
        const uint32_t reach = (uint32_t)(f.scales * f.alpha);
        const bool inside = (x + reach < (uint32_t)f.W) & (y + reach < (uint32_t)f.H);
        const float *p = f.depth + (int64_t)y * f.stride + x;
        const PixelOut o = eval_pixel_multiscale(inside, p, (float)x - f.cx, (float)y - f.cy, f);
        nx = o.nx;
        ny = o.ny;
        nz = o.nz;
        code = o.code;
    } else if (!is_multiscale(M) && live) {
        const uint32_t y = row_of(i, f.inv_gpr);
        const uint32_t x = i - y * f.gpr;
        const bool inside = (x >= (uint32_t)A) & (x + A < (uint32_t)f.W) &
                            (y >= (uint32_t)A) & (y + A < (uint32_t)f.H);
        const float *p = f.depth + (int64_t)y * f.stride + x;
        float d1 = *p, d2 = 0.f, d3 = 0.f, d4 = 0.f, d5 = 0.f;
        if (inside) {
            d2 = p[A];
            d4 = p[-A];
            d3 = p[(int64_t)A * f.stride];
            d5 = p[-(int64_t)A * f.stride];
        }
        const float xc = (float)x - f.cx;
        const float yc = (float)y - f.cy;
        const PixelOut o = eval_method<M>(inside, d1, d2, d3, d4, d5, xc, yc, f);
        nx = o.nx;
        ny = o.ny;
        nz = o.nz;
        code = o.code;
    }
    r.nx = nx;
    r.ny = ny;
    r.nz = nz;
    r.code = code;
}

__device__ __forceinline__ void scalar_write(const FrameArgs &f, uint32_t tile, TileLds &lds,
                                             const ScalarOut &r) {
    float *s = reinterpret_cast<float *>(lds.v);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w = wave_id();
    const uint32_t p0 = tile * kBlock + 64 * w;  // first pixel of this wavefront
    // unconditional stores, as in vec4_write (size 0 past the frame's end)
    const uint32_t np = p0 < f.nitems ? min(64u, f.nitems - p0) : 0u;
    out_store_byte((uint8_t)r.code, out_buf(f.mask + p0, np), lane);
    const float nx = r.nx, ny = r.ny, nz = r.nz;
    // wavefront-local transpose through this wavefront's LDS slice
    float *slice = s + 192 * w;
    wave_lds_sync();
    slice[3 * lane + 0] = nx;
    slice[3 * lane + 1] = ny;
    slice[3 * lane + 2] = nz;
    wave_lds_sync();
    const OutBuf nb = out_buf(f.normals + 3 * (int64_t)p0, 12 * np);
#pragma unroll
    for (int k = 0; k < 3; ++k) out_store(slice[64 * k + lane], nb, 4 * lane + 256 * k);
}

__device__ __forceinline__ void scalar_count(const ScalarOut &r, uint32_t &cv, uint32_t &cb) {
    cv += wave_count(r.live & (r.code == BN_VALID));
    cb += wave_count(r.live & (r.code == BN_BOUNDARY));
}

// One whole tile of either kind, method M.  No workgroup barrier:
// consecutive tiles of a workgroup may overlap freely.  The multi-scale
// method takes vector tiles only when alpha * scales <= kMsVecReach (the host's
// choice).
template <int A, int M>
__device__ __forceinline__ void run_tile(const FrameArgs &f, bool vec, uint32_t tile, TileLds &lds,
                                         uint32_t &cv, uint32_t &cb) {
    if (vec) {
        Vec4Out o;
        vec4_eval_method<A, M>(f, tile, o, lds);
        vec4_write<M>(f, tile, lds, o);
        if (f.stats) vec4_count(o, cv, cb);
    } else {
        ScalarOut r;
        scalar_eval<A, M>(f, tile, r);
        scalar_write(f, tile, lds, r);
        if (f.stats) scalar_count(r, cv, cb);
    }
}

// One vector tile with its counts, as part `part` of `nparts` of the frame.
// The counts are known before the stores, so the count atomic goes out first
// and its round trip overlaps the stores.
template <int A, int M, int TB = kBlock>
__device__ __forceinline__ void vec4_tile_counted(const FrameArgs &f, uint32_t tile,
                                                  uint32_t part, uint32_t nparts,
                                                  TileLdsT<TB> &lds) {
    Vec4Out o;
    if constexpr (TB == kBlock) {
        vec4_eval_method<A, M>(f, tile, o, lds);
    } else {
        vec4_eval<A, M, TB>(f, tile, o, lds);  // the five-tap methods only
    }
    CountTicket tk;
    bool have = false;
    uint32_t cv = 0, cb = 0;
    vec4_count(o, cv, cb);
    if (f.stats) {
        uint32_t v, b;
        block_sum<TB>(cv, cb, v, b);
        if (threadIdx.x == 0) {
            tk = count_issue(f.work, f.stats, part, nparts, v, b, f.npix, f.overwrite);
            have = true;
        }
    }
    vec4_write<M, TB>(f, tile, lds, o);
    if (have) count_finish(tk);
}

// One scalar tile with its counts, as part `part` of `nparts` of the frame:
// as in vec4_tile_counted, the count atomic goes out before the stores.
template <int A, int M>
__device__ __forceinline__ void scalar_tile_counted(const FrameArgs &f, uint32_t tile,
                                                    uint32_t part, uint32_t nparts,
                                                    TileLds &lds) {
    ScalarOut r;
    scalar_eval<A, M>(f, tile, r);
    CountTicket tk;
    bool have = false;
    if (f.stats) {
        uint32_t cv = 0, cb = 0, v, b;
        scalar_count(r, cv, cb);
        block_sum(cv, cb, v, b);
        if (threadIdx.x == 0) {
            tk = count_issue(f.work, f.stats, part, nparts, v, b, f.npix, f.overwrite);
            have = true;
        }
    }
    scalar_write(f, tile, lds, r);
    if (have) count_finish(tk);
}

// Two vector tiles of one workgroup, software-pipelined: the second tile's
// loads are issued before the first tile's arithmetic, so they are in flight
// while it computes and stores.  (On gfx9 one counter tracks loads and
// stores in issue order: the wait for the second tile's loads, issued before
// the first tile's stores, does not wait for those stores.)  The counts of
// both tiles go out as one part; tile t1 may lie past the frame's end (its
// lanes are then not live).
template <int A, int M>
__device__ __forceinline__ void vec4_tile_pair_counted(const FrameArgs &f, uint32_t t0,
                                                       uint32_t t1, uint32_t part,
                                                       uint32_t nparts, TileLds &lds) {
    Vec4In<A> a, b;
    vec4_load<A>(f, t0, a);
    vec4_load<A>(f, t1, b);
    uint32_t cv = 0, cb = 0;
    {
        Vec4Out o;
        vec4_compute<A, M>(f, a, o, lds);
        vec4_count(o, cv, cb);
        // the second tile's loads have been in flight during this
        // arithmetic: wait for them now, while no store is outstanding (the
        // counter cannot tell loads from stores, so a wait after the stores
        // would wait for those too)
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
        vec4_write<M>(f, t0, lds, o);
    }
    Vec4Out o;
    vec4_compute<A, M>(f, b, o, lds);
    vec4_count(o, cv, cb);
    CountTicket tk;
    bool have = false;
    if (f.stats) {
        uint32_t v, bb;
        block_sum(cv, cb, v, bb);
        if (threadIdx.x == 0) {
            tk = count_issue(f.work, f.stats, part, nparts, v, bb, f.npix, f.overwrite);
            have = true;
        }
    }
    vec4_write<M>(f, t1, lds, o);
    if (have) count_finish(tk);
}

}  // namespace bn
