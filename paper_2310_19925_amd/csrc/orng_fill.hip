// Fill kernels: counter-partitioned bulk generation of one or many streams.
//
// Output sample j of stream (seed, ctr) is sample offset + j of that stream
// (paper section 3.1: the (seed, counter) pair names the stream; any position
// can be computed directly, so a fill is embarrassingly parallel and the
// result cannot depend on the launch geometry).
//
// Work decomposition.  Positions are grouped in blocks of four words (one
// Philox/Threefry output block, two Box-Muller pairs, four Squares words).
// A span is 64*U consecutive blocks handled by one wave: in iteration u,
// lane l produces block span*64U + u*64 + l, so each 16-byte store
// instruction of the wave covers 1 KiB of contiguous output.  For Tyche a
// span is one 16384-word tile: lane l steps its own substream through blocks
// k*64 + l, k = 0..63, which is the same store pattern.  Spans are numbered
// in absolute block space, so a fill that starts mid-span simply masks the
// blocks in front of its first position.  Blocks that straddle the start or
// end of the range are written one dword at a time; an output whose address
// is not 16-byte aligned with the block grid is realigned across lanes.
#include "orng_internal.hpp"
#include "orng_span.hpp"

namespace orng {

struct SpanArgs {
    KeySched ks;
    char *out;                 // output of stream 0
    uint64_t p0;               // first position of every stream
    uint64_t n;                // samples per stream
    uint64_t first_span;       // absolute index of the first span
    uint64_t spans_per_stream;
    uint64_t total_spans;      // n_streams * spans_per_stream
    uint32_t ctr0;             // counter of stream 0
    uint32_t unroll;           // U (counter generators)
    uint32_t delta;            // (stream 0 output address in words - p0) mod 4
};

// Fill kernels that take the check-free loop for interior spans (see
// process_span): 1 with two blocks per iteration, 2 with one, 0 the general
// loop only.  Measured on MI355X (2^30-sample fills, 2^29 for float64, builds
// interleaved on one box): two blocks per iteration made Squares32 u32 /
// uniform 1-9% faster, Threefry2x64 3-10% (float64 normals 10%), Squares64
// 2-7%, Tyche and Tyche-i u32 / uniform / float64 uniform 2-4%, the 13-round
// Threefry2x64 normals and float64 fills 3-10%; one block per iteration made
// Philox and Philox2x32 float64 normals 10-11% faster, their float64 uniforms
// and normals and Philox2x32 uniforms 1-9%.  Left out where neither helped:
// Threefry4x32 (8-10% slower with two blocks, as the compiler then held both
// blocks' state, 38 -> 62 VGPRs; 15-20% slower with one), Philox and
// Philox2x32 u32, Tyche normals, 13-round Threefry2x64 u32 / uniform.
template <int G, int D>
constexpr int fast_span() {
    if constexpr (G == G_TF2X64 || G == G_SQUARES || G == G_SQUARES64)
        return 1;
    else if constexpr (G == G_TF2X64_13)
        return D != D_U32 && D != D_UNIFORM ? 1 : 0;
    else if constexpr (tyche_like(G))
        return D != D_NORMAL && D != D_F64N ? 1 : 0;
    else if constexpr (G == G_PHILOX)
        return D == D_NORMAL || D == D_F64U || D == D_F64N ? 2 : 0;
    else if constexpr (G == G_PHILOX2X32)
        return D != D_U32 && D != D_F64U ? 2 : 0;
    else
        return 0;
}

template <int G, int D, bool NT>
__global__ __launch_bounds__(512) void k_span(SpanArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wpg = blockDim.x >> 6;
    const uint64_t wave0 = wave_uniform(blockIdx.x * wpg + (threadIdx.x >> 6));
    const uint64_t nwaves = (uint64_t)gridDim.x * wpg;
    const uint64_t pend = a.p0 + a.n;
    for (uint64_t t = wave0; t < a.total_spans; t += nwaves) {
        uint64_t si = 0, sl = t;
        if (a.spans_per_stream != a.total_spans) {
            si = t / a.spans_per_stream;
            sl = t - si * a.spans_per_stream;
        }
        const uint64_t span = a.first_span + sl;
        const uint32_t ctr = a.ctr0 + (uint32_t)si;
        char *base = a.out + si * a.n * 4;
        const uint32_t delta = (a.delta + (uint32_t)(si * a.n)) & 3u;
        process_span<G, D, NT, fast_span<G, D>()>(a.ks, ctr, base, a.p0, pend, span, a.unroll,
                                                  delta, lane);
    }
}

// Many short streams: one lane per (stream, block) pair.
struct UnitArgs {
    KeySched ks;
    char *out;
    uint64_t p0, n;
    uint32_t first_block, bps;  // blocks per stream
    uint32_t total_units;
    uint32_t ctr0;
    uint32_t aligned;
};

template <int G, int D, bool NT>
__global__ __launch_bounds__(256) void k_units(UnitArgs a) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.total_units) return;
    const uint32_t i = g / a.bps;
    const uint32_t blk = a.first_block + (g - i * a.bps);
    const uint32_t ctr = a.ctr0 + i;
    uint32_t w[4];
    if constexpr (tyche_like(G)) {
        const uint32_t t = blk / TYCHE_TILE_BLOCKS, l = blk & 63u;
        const uint32_t k = (blk % TYCHE_TILE_BLOCKS) >> 6;
        TycheT<G == G_TYCHE_I> st;
        st.seed(a.ks, t * 64u + l, ctr);
        for (uint32_t s = 0; s < 4 * k; ++s) st.mix();
        st.next4(w);
    } else {
        counter_block<G>(blk, ctr, a.ks, w);
    }
    convert4<D>(w);
    store_block<NT>(a.out + (uint64_t)i * a.n * 4, (uint64_t)blk * 4, a.p0, a.p0 + a.n,
                    a.aligned, w);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <int G, int D, bool NT>
struct Kern {
    static void *span() { return reinterpret_cast<void *>(&k_span<G, D, NT>); }
    static void *units() { return reinterpret_cast<void *>(&k_units<G, D, NT>); }
};

template <int G, int D>
static void *pick(bool units, bool nt) {
    if (units) return nt ? Kern<G, D, true>::units() : Kern<G, D, false>::units();
    return nt ? Kern<G, D, true>::span() : Kern<G, D, false>::span();
}

template <int G>
static void *pick_d(int dist, bool units, bool nt) {
    switch (dist) {
    case D_U32: return pick<G, D_U32>(units, nt);
    case D_UNIFORM: return pick<G, D_UNIFORM>(units, nt);
    case D_NORMAL: return pick<G, D_NORMAL>(units, nt);
    case D_F64U: return pick<G, D_F64U>(units, nt);
    default: return pick<G, D_F64N>(units, nt);
    }
}

static void *pick_kernel(int gen, int dist, bool units, bool nt) {
    switch (gen) {
    case G_PHILOX: return pick_d<G_PHILOX>(dist, units, nt);
    case G_TF4X32: return pick_d<G_TF4X32>(dist, units, nt);
    case G_TF2X64: return pick_d<G_TF2X64>(dist, units, nt);
    case G_SQUARES: return pick_d<G_SQUARES>(dist, units, nt);
    case G_TF4X32_13: return pick_d<G_TF4X32_13>(dist, units, nt);
    case G_TF2X64_13: return pick_d<G_TF2X64_13>(dist, units, nt);
    case G_TYCHE_I: return pick_d<G_TYCHE_I>(dist, units, nt);
    case G_SQUARES64: return pick_d<G_SQUARES64>(dist, units, nt);
    case G_PHILOX2X32: return pick_d<G_PHILOX2X32>(dist, units, nt);
    default: return pick_d<G_TYCHE>(dist, units, nt);
    }
}

hipError_t launch_fill(int gen, int dist, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                       uint64_t offset, uint64_t per_stream, void *out, hipStream_t s) {
    if (n_streams == 0 || per_stream == 0) return hipSuccess;
    const LaunchCfg cfg = launch_cfg();
    const bool nt = cfg.nontemporal ? cfg.nontemporal == 1 : tuned_fill(gen, dist).nontemporal == 1;
    const uint64_t addr_words = reinterpret_cast<uintptr_t>(out) / 4;
    const bool aligned = ((addr_words - offset) & 3u) == 0 && (n_streams == 1 || per_stream % 4 == 0);
    const uint32_t delta = (uint32_t)((addr_words - offset) & 3u);
    const uint64_t first_block = offset / 4;
    const uint64_t last_block = (offset + per_stream - 1) / 4;
    const uint64_t bps = last_block - first_block + 1;
    const KeySched ks = make_keysched(seed);

    if (n_streams > 1 && bps < 64 && (uint64_t)n_streams * bps < (1ull << 31)) {
        UnitArgs a;
        a.ks = ks;
        a.out = static_cast<char *>(out);
        a.p0 = offset;
        a.n = per_stream;
        a.first_block = (uint32_t)first_block;
        a.bps = (uint32_t)bps;
        a.total_units = (uint32_t)(n_streams * bps);
        a.ctr0 = ctr0;
        a.aligned = aligned;
        const uint32_t wg = 256;
        const uint32_t grid = (a.total_units + wg - 1) / wg;
        void *args[] = {&a};
        return hipLaunchKernel(pick_kernel(gen, dist, true, nt), dim3(grid), dim3(wg), args, 0, s);
    }

    SpanArgs a;
    a.ks = ks;
    a.out = static_cast<char *>(out);
    a.p0 = offset;
    a.n = per_stream;
    a.ctr0 = ctr0;
    a.delta = delta;
    const Tuned tu = tuned_fill(gen, dist);
    a.unroll = tyche_like(gen) ? 64 : (cfg.unroll ? cfg.unroll : tu.unroll);
    const uint64_t sb = span_blocks(gen, a.unroll);
    a.first_span = first_block / sb;
    a.spans_per_stream = last_block / sb - a.first_span + 1;
    a.total_spans = a.spans_per_stream * n_streams;
    const uint32_t wg = cfg.wg_size ? cfg.wg_size : tu.wg_size;
    const uint64_t wpg = wg / 64;
    uint64_t grid = (a.total_spans + wpg - 1) / wpg;
    const uint64_t cap = cfg.max_wgs ? cfg.max_wgs : (tu.max_wgs ? tu.max_wgs : (1ull << 30));
    if (grid > cap) grid = cap;
    if (grid > max_wgs_1d(wg)) grid = max_wgs_1d(wg);  // spans are grid-strided
    void *args[] = {&a};
    return hipLaunchKernel(pick_kernel(gen, dist, false, nt), dim3((uint32_t)grid), dim3(wg), args,
                           0, s);
}

}  // namespace orng
