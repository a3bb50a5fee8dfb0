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
// sample keeps its fixed pair of stream positions.
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

namespace orng {

constexpr uint64_t RANGE_GROUP = 256;                       // samples, counter generators
constexpr uint64_t RANGE_TILE = TYCHE_TILE_WORDS / 2;       // samples per Tyche tile

__device__ __forceinline__ uint32_t range_scale(uint32_t w0, uint32_t w1, uint32_t r) {
    const uint64_t t = (uint64_t)w0 * r;
    const uint64_t s = (uint64_t)w1 * r + (t >> 32);
    return (uint32_t)(s >> 32);
}

struct RangeArgs {
    KeySched ks;
    int32_t *out;               // sample s0 of stream 0
    uint64_t s0, n;             // first sample, samples per stream
    uint64_t first_group;       // first group of every stream
    uint64_t groups_per_stream;
    uint64_t total_groups;      // n_streams * groups_per_stream
    uint32_t ctr0;              // counter of stream 0
    uint32_t lo, r;             // lo as its two's-complement bits, r = hi - lo
    uint32_t mis;               // (stream 0 output address in words - s0) mod 4
};

template <int N>
__device__ __forceinline__ void range_store(int32_t *base, uint64_t q, uint64_t s0, uint64_t send,
                                            bool aligned, const uint32_t v[N]) {
    if (aligned && q >= s0 && q + N <= send) {
        if constexpr (N == 4) {
            typedef uint32_t u4 __attribute__((ext_vector_type(4)));
            *reinterpret_cast<u4 *>(base + (q - s0)) = u4{v[0], v[1], v[2], v[3]};
        } else {
            typedef uint32_t u2 __attribute__((ext_vector_type(2)));
            *reinterpret_cast<u2 *>(base + (q - s0)) = u2{v[0], v[1]};
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (q + i >= s0 && q + i < send) base[q + i - s0] = (int32_t)v[i];
}

template <int G>
__global__ __launch_bounds__(256) void k_range(RangeArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wpg = blockDim.x >> 6;
    const uint64_t wave0 =
        __builtin_amdgcn_readfirstlane(blockIdx.x * wpg + (threadIdx.x >> 6));
    const uint64_t nwaves = (uint64_t)gridDim.x * wpg;
    const uint64_t send = a.s0 + a.n;
    for (uint64_t t = wave0; t < a.total_groups; t += nwaves) {
        uint64_t si = 0, gl = t;
        if (a.groups_per_stream != a.total_groups) {
            si = t / a.groups_per_stream;
            gl = t - si * a.groups_per_stream;
        }
        const uint64_t g = a.first_group + gl;
        const uint32_t ctr = a.ctr0 + (uint32_t)si;
        int32_t *base = a.out + si * a.n;
        const uint32_t mis = (a.mis + (uint32_t)(si * a.n)) & 3u;
        if constexpr (tyche_like(G)) {
            TycheT<G == G_TYCHE_I> st;
            st.seed(a.ks, (uint32_t)g * 64u + lane, ctr);
            const uint64_t b0 = g * TYCHE_TILE_BLOCKS;
            for (uint32_t k = 0; k < 64; ++k) {
                const uint64_t bw = b0 + 64u * k;  // first block of this step
                if (2 * bw >= send) break;
                uint32_t w[4];
                st.next4(w);
                if (2 * (bw + 64) <= a.s0) continue;
                const uint32_t v[2] = {a.lo + range_scale(w[0], w[1], a.r),
                                       a.lo + range_scale(w[2], w[3], a.r)};
                range_store<2>(base, 2 * (bw + lane), a.s0, send, (mis & 1u) == 0, v);
            }
        } else {
            const uint64_t m = g * 64u + lane;
            if (4 * m < send && 4 * m + 4 > a.s0) {
                uint32_t w[4], x[4];
                counter_block<G>((uint32_t)(2 * m), ctr, a.ks, w);
                counter_block<G>((uint32_t)(2 * m + 1), ctr, a.ks, x);
                const uint32_t v[4] = {a.lo + range_scale(w[0], w[1], a.r),
                                       a.lo + range_scale(w[2], w[3], a.r),
                                       a.lo + range_scale(x[0], x[1], a.r),
                                       a.lo + range_scale(x[2], x[3], a.r)};
                range_store<4>(base, 4 * m, a.s0, send, mis == 0, v);
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
        const uint32_t v[2] = {a.lo + range_scale(w[0], w[1], a.r),
                               a.lo + range_scale(w[2], w[3], a.r)};
        range_store<2>(base, 2 * (uint64_t)u, a.s0, send, false, v);
    } else {
        uint32_t w[4], x[4];
        counter_block<G>(2 * u, ctr, a.ks, w);
        counter_block<G>(2 * u + 1, ctr, a.ks, x);
        const uint32_t v[4] = {a.lo + range_scale(w[0], w[1], a.r),
                               a.lo + range_scale(w[2], w[3], a.r),
                               a.lo + range_scale(x[0], x[1], a.r),
                               a.lo + range_scale(x[2], x[3], a.r)};
        range_store<4>(base, 4 * (uint64_t)u, a.s0, send, false, v);
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
    const uint64_t gs = tyche_like(gen) ? RANGE_TILE : RANGE_GROUP;
    a.first_group = offset / gs;
    a.groups_per_stream = (offset + per_stream - 1) / gs - a.first_group + 1;
    a.total_groups = a.groups_per_stream * n_streams;
    const uint32_t wg = 256, wpg = wg / 64;
    uint64_t grid = (a.total_groups + wpg - 1) / wpg;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (grid > cap) grid = cap;
    void *args[] = {&a};
    const hipError_t e = hipLaunchKernel(range_kernel(gen), dim3((uint32_t)grid), dim3(wg), args,
                                         0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        set_hip_error(e);
        return ORNG_EHIP;
    }
    return ORNG_OK;
}
