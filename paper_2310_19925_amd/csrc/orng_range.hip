// Integer samples in [lo, hi) (section 3: the generators are meant to feed
// standard-library distributions; the paper defines no integer conversion).
//
// Sample p of stream (seed, ctr) takes the 64-bit integer x made of the words
// at positions 2p and 2p+1, (w1 << 32) | w0, and returns lo + floor(x r / 2^64)
// with r = hi - lo < 2^32.  With x = w1 2^32 + w0:
//   floor(x r / 2^64) = floor((w1 r + floor(w0 r / 2^32)) / 2^32),
// two 32x32->64 multiply-adds, and the sum stays below 2^64.  Each value has
// floor(2^64 / r) or ceil(2^64 / r) preimages, so its probability is within
// 2^-64 of 1/r; no remainder is taken and no sample is rejected, so every
// sample keeps its fixed pair of stream positions.  (range_sample, in the
// device header, is shared with the batched and served kernels.)
//
// Work decomposition.  A wave handles one group per loop trip.  Counter
// generators: a group is 256 samples; lane l makes blocks 2m and 2m+1,
// m = 64 g + l (words 8m..8m+7 = samples 4m..4m+3) and writes them with one
// 16-byte store, so a store instruction of the wave covers 1 KiB.  Tyche: a
// group is one 16384-word tile (8192 samples); lane l steps substream
// t*64 + l through blocks k*64 + l (the Tyche stream layout) and writes the two
// samples of each block with one 8-byte store (512 contiguous bytes per
// instruction).  Groups are numbered in absolute sample space, so a fill that
// starts mid-group masks the samples in front of its first one; samples at the
// range ends, and outputs not aligned with the store width, are written one
// word at a time.  Many streams of a few samples each (under 64 units per
// stream) take one lane per (stream, unit) instead, so a wave is not spent on
// one stream's handful of samples.
#include "../../include/orng.h"
#include "orng_device.hpp"
#include "orng_internal.hpp"
#include "orng_span.hpp"

namespace orng {

constexpr uint64_t RANGE_GROUP = 256;                       // samples, counter generators
constexpr uint64_t RANGE_TILE = TYCHE_TILE_WORDS / 2;       // samples per Tyche tile

struct RangeArgs {
    KeySched ks;
    int32_t *out;               // sample s0 of stream 0
    uint64_t s0, n;             // first sample, samples per stream
    uint64_t first_span;        // first span of every stream
    uint64_t spans_per_stream;
    uint64_t total_spans;       // n_streams * spans_per_stream
    uint32_t ctr0;              // counter of stream 0
    uint32_t lo, r;             // lo as its two's-complement bits, r = hi - lo
    uint32_t mis;               // (stream 0 output address in words - s0) mod 4
    uint32_t unroll;            // groups per span (counter generators)
};

// Group g of a counter generator's stream: lane l makes blocks 2m and 2m + 1,
// m = 64 g + l, i.e. samples 4m .. 4m + 3, and writes them with one 16-byte
// store.
template <int G>
__device__ __forceinline__ void range_group(const RangeArgs &a, uint64_t g, uint32_t ctr,
                                            int32_t *base, uint64_t send, bool aligned,
                                            uint32_t lane) {
    const uint64_t m = g * 64u + lane;
    if (4 * m >= send || 4 * m + 4 <= a.s0) return;
    uint32_t w[4], x[4];
    counter_block<G>((uint32_t)(2 * m), ctr, a.ks, w);
    counter_block<G>((uint32_t)(2 * m + 1), ctr, a.ks, x);
    const uint32_t v[4] = {range_sample(w[0], w[1], a.r, a.lo),
                           range_sample(w[2], w[3], a.r, a.lo),
                           range_sample(x[0], x[1], a.r, a.lo),
                           range_sample(x[2], x[3], a.r, a.lo)};
    store_samples<4, false>(base, 4 * m, a.s0, send, aligned, v);
}

// One span per wave and loop trip, like the fill kernels: counter generators
// take `unroll` consecutive groups of 256 samples (the launch table's span
// length), Tyche one tile.  The grid normally covers every span with one wave
// (short-lived waves keep the most stores in flight); a grid cap makes the
// waves loop.
template <int G>
__global__ __launch_bounds__(512) void k_range(RangeArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wpg = blockDim.x >> 6;
    const uint64_t wave0 =
        __builtin_amdgcn_readfirstlane(blockIdx.x * wpg + (threadIdx.x >> 6));
    const uint64_t nwaves = (uint64_t)gridDim.x * wpg;
    const uint64_t send = a.s0 + a.n;
    for (uint64_t t = wave0; t < a.total_spans; t += nwaves) {
        uint64_t si = 0, sl = t;
        if (a.spans_per_stream != a.total_spans) {
            si = t / a.spans_per_stream;
            sl = t - si * a.spans_per_stream;
        }
        const uint64_t span = a.first_span + sl;
        const uint32_t ctr = a.ctr0 + (uint32_t)si;
        int32_t *base = a.out + si * a.n;
        const uint32_t mis = (a.mis + (uint32_t)(si * a.n)) & 3u;
        if constexpr (tyche_like(G)) {
            TycheT<G == G_TYCHE_I> st;
            st.seed(a.ks, (uint32_t)span * 64u + lane, ctr);
            const uint64_t b0 = span * TYCHE_TILE_BLOCKS;
            for (uint32_t k = 0; k < 64; ++k) {
                const uint64_t bw = b0 + 64u * k;  // first block of this step
                if (2 * bw >= send) break;
                uint32_t w[4];
                st.next4(w);
                if (2 * (bw + 64) <= a.s0) continue;
                const uint32_t v[2] = {range_sample(w[0], w[1], a.r, a.lo),
                                       range_sample(w[2], w[3], a.r, a.lo)};
                store_samples<2, false>(base, 2 * (bw + lane), a.s0, send, (mis & 1u) == 0, v);
            }
        } else {
            const uint64_t g0 = span * a.unroll;
            const uint64_t q0 = g0 * RANGE_GROUP, q1 = q0 + a.unroll * RANGE_GROUP;
            if (mis == 0 && q0 >= a.s0 && q1 <= send) {
                // A span inside the range with 16-byte aligned output: no
                // per-sample checks, the store address steps by 1 KiB.  The
                // store of a group is issued after the next group is made,
                // and stores are non-temporal: on MI355X both let the
                // generation overlap the writes better (the span's 1-4 MiB
                // are not read back soon).
                typedef uint32_t u4 __attribute__((ext_vector_type(4)));
                u4 *o = reinterpret_cast<u4 *>(base + (q0 - a.s0)) + lane;
                uint32_t blk = (uint32_t)(2 * (g0 * 64u + lane));
                auto make = [&](uint32_t b) {
                    uint32_t w[4], x[4];
                    counter_block<G>(b, ctr, a.ks, w);
                    counter_block<G>(b + 1u, ctr, a.ks, x);
                    return u4{range_sample(w[0], w[1], a.r, a.lo),
                              range_sample(w[2], w[3], a.r, a.lo),
                              range_sample(x[0], x[1], a.r, a.lo),
                              range_sample(x[2], x[3], a.r, a.lo)};
                };
                u4 prev = make(blk);
                for (uint32_t u = 1; u < a.unroll; ++u) {
                    blk += 128u;
                    const u4 v = make(blk);
                    __builtin_nontemporal_store(prev, o);
                    o += 64;
                    prev = v;
                }
                __builtin_nontemporal_store(prev, o);
                continue;
            }
            // groups wholly before the range's first sample are skipped,
            // and the span ends at the range's last one
            uint32_t u = a.s0 / RANGE_GROUP > g0 ? (uint32_t)(a.s0 / RANGE_GROUP - g0) : 0u;
            for (; u < a.unroll; ++u) {
                const uint64_t g = g0 + u;
                if (g * RANGE_GROUP >= send) break;
                range_group<G>(a, g, ctr, base, send, mis == 0, lane);
            }
        }
    }
}

// Many short streams: one lane per (stream, unit).  Counter generators: unit
// u is blocks 2u and 2u+1 (samples 4u..4u+3); Tyche: unit u is block u
// (samples 2u, 2u+1), reached by seeding its substream and stepping it to
// the block.  Samples outside [s0, s0 + n) are not written.
struct RangeUnitArgs {
    KeySched ks;
    int32_t *out;
    uint64_t s0, n;
    uint32_t first_unit, units_per_stream, total_units;
    uint32_t ctr0, lo, r;
};

template <int G>
__global__ __launch_bounds__(256) void k_range_units(RangeUnitArgs a) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.total_units) return;
    const uint32_t i = g / a.units_per_stream;
    const uint32_t u = a.first_unit + (g - i * a.units_per_stream);
    const uint32_t ctr = a.ctr0 + i;
    int32_t *base = a.out + (uint64_t)i * a.n;
    const uint64_t send = a.s0 + a.n;
    if constexpr (tyche_like(G)) {
        const uint32_t t = u / TYCHE_TILE_BLOCKS, l = u & 63u;
        const uint32_t k = (u % TYCHE_TILE_BLOCKS) >> 6;
        TycheT<G == G_TYCHE_I> st;
        st.seed(a.ks, t * 64u + l, ctr);
        for (uint32_t j = 0; j < 4 * k; ++j) st.mix();
        uint32_t w[4];
        st.next4(w);
        const uint32_t v[2] = {range_sample(w[0], w[1], a.r, a.lo),
                               range_sample(w[2], w[3], a.r, a.lo)};
        store_samples<2, false>(base, 2 * (uint64_t)u, a.s0, send, false, v);
    } else {
        uint32_t w[4], x[4];
        counter_block<G>(2 * u, ctr, a.ks, w);
        counter_block<G>(2 * u + 1, ctr, a.ks, x);
        const uint32_t v[4] = {range_sample(w[0], w[1], a.r, a.lo),
                               range_sample(w[2], w[3], a.r, a.lo),
                               range_sample(x[0], x[1], a.r, a.lo),
                               range_sample(x[2], x[3], a.r, a.lo)};
        store_samples<4, false>(base, 4 * (uint64_t)u, a.s0, send, false, v);
    }
}

static void *range_units_kernel(int gen) {
    switch (gen) {
    case G_PHILOX: return reinterpret_cast<void *>(&k_range_units<G_PHILOX>);
    case G_TF4X32: return reinterpret_cast<void *>(&k_range_units<G_TF4X32>);
    case G_TF2X64: return reinterpret_cast<void *>(&k_range_units<G_TF2X64>);
    case G_SQUARES: return reinterpret_cast<void *>(&k_range_units<G_SQUARES>);
    case G_TF4X32_13: return reinterpret_cast<void *>(&k_range_units<G_TF4X32_13>);
    case G_TF2X64_13: return reinterpret_cast<void *>(&k_range_units<G_TF2X64_13>);
    case G_TYCHE_I: return reinterpret_cast<void *>(&k_range_units<G_TYCHE_I>);
    case G_SQUARES64: return reinterpret_cast<void *>(&k_range_units<G_SQUARES64>);
    case G_PHILOX2X32: return reinterpret_cast<void *>(&k_range_units<G_PHILOX2X32>);
    default: return reinterpret_cast<void *>(&k_range_units<G_TYCHE>);
    }
}

static void *range_kernel(int gen) {
    switch (gen) {
    case G_PHILOX: return reinterpret_cast<void *>(&k_range<G_PHILOX>);
    case G_TF4X32: return reinterpret_cast<void *>(&k_range<G_TF4X32>);
    case G_TF2X64: return reinterpret_cast<void *>(&k_range<G_TF2X64>);
    case G_SQUARES: return reinterpret_cast<void *>(&k_range<G_SQUARES>);
    case G_TF4X32_13: return reinterpret_cast<void *>(&k_range<G_TF4X32_13>);
    case G_TF2X64_13: return reinterpret_cast<void *>(&k_range<G_TF2X64_13>);
    case G_TYCHE_I: return reinterpret_cast<void *>(&k_range<G_TYCHE_I>);
    case G_SQUARES64: return reinterpret_cast<void *>(&k_range<G_SQUARES64>);
    case G_PHILOX2X32: return reinterpret_cast<void *>(&k_range<G_PHILOX2X32>);
    default: return reinterpret_cast<void *>(&k_range<G_TYCHE>);
    }
}

}  // namespace orng

using namespace orng;

extern "C" int orng_fill_range(int gen, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                               uint64_t offset, uint64_t per_stream, int32_t lo, int32_t hi,
                               int32_t *d_out, void *stream) {
    if (gen < 0 || gen >= NGEN || lo >= hi || !seed_ok(gen, seed)) return ORNG_EINVAL;
    const uint64_t lim = PERIOD / 2;
    if (offset > lim || per_stream > lim - offset) return ORNG_ERANGE;
    if (n_streams && (uint64_t)ctr0 + n_streams - 1 > 0xFFFFFFFFull) return ORNG_ERANGE;
    if (n_streams == 0 || per_stream == 0) return ORNG_OK;
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & 3u)) return ORNG_EINVAL;
    // many streams of a few samples each: one lane per unit (see k_range_units)
    const uint64_t spu = tyche_like(gen) ? 2 : 4;  // samples per unit
    const uint64_t fu = offset / spu, lu = (offset + per_stream - 1) / spu;
    if (n_streams > 1 && lu - fu + 1 < 64 && (uint64_t)n_streams * (lu - fu + 1) < (1ull << 31)) {
        RangeUnitArgs u;
        u.ks = make_keysched(seed);
        u.out = d_out;
        u.s0 = offset;
        u.n = per_stream;
        u.first_unit = (uint32_t)fu;
        u.units_per_stream = (uint32_t)(lu - fu + 1);
        u.total_units = (uint32_t)(n_streams * (lu - fu + 1));
        u.ctr0 = ctr0;
        u.lo = (uint32_t)lo;
        u.r = (uint32_t)((int64_t)hi - (int64_t)lo);
        void *uargs[] = {&u};
        const hipError_t e = hipLaunchKernel(range_units_kernel(gen),
                                             dim3((u.total_units + 255) / 256), dim3(256), uargs,
                                             0, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) {
            set_hip_error(e);
            return ORNG_EHIP;
        }
        return ORNG_OK;
    }
    RangeArgs a;
    a.ks = make_keysched(seed);
    a.out = d_out;
    a.s0 = offset;
    a.n = per_stream;
    a.ctr0 = ctr0;
    a.lo = (uint32_t)lo;
    a.r = (uint32_t)((int64_t)hi - (int64_t)lo);
    a.mis = (uint32_t)((reinterpret_cast<uintptr_t>(d_out) / 4 - offset) & 3u);
    const LaunchCfg cfg = launch_cfg();
    const Tuned tu = tuned_range(gen);
    a.unroll = tyche_like(gen) ? 1 : (cfg.unroll ? cfg.unroll : tu.unroll);
    const uint64_t span_samples = tyche_like(gen) ? RANGE_TILE : RANGE_GROUP * a.unroll;
    a.first_span = offset / span_samples;
    a.spans_per_stream = (offset + per_stream - 1) / span_samples - a.first_span + 1;
    a.total_spans = a.spans_per_stream * n_streams;
    const uint32_t wg = cfg.wg_size ? cfg.wg_size : tu.wg_size, wpg = wg / 64;
    uint64_t grid = (a.total_spans + wpg - 1) / wpg;
    const uint64_t cap = cfg.max_wgs ? cfg.max_wgs : (tu.max_wgs ? tu.max_wgs : (1ull << 30));
    if (grid > cap) grid = cap;
    if (grid > max_wgs_1d(wg)) grid = max_wgs_1d(wg);  // spans are grid-strided
    void *args[] = {&a};
    const hipError_t e = hipLaunchKernel(range_kernel(gen), dim3((uint32_t)grid), dim3(wg), args,
                                         0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        set_hip_error(e);
        return ORNG_EHIP;
    }
    return ORNG_OK;
}
