// Span processing shared by the fill, batched and served kernels.
//
// A span is the unit of work of one wave.  Counter-based generators: 64*U
// consecutive blocks of four words, block span*64U + u*64 + lane in iteration
// u, so every 16-byte store instruction of the wave covers 1 KiB of
// contiguous output.  Tyche: one 16384-word tile, lane l stepping its own
// substream through blocks k*64 + l, k = 0..63 (the Tyche stream layout).
// Spans are numbered in absolute block space of the stream; blocks outside
// [p0, pend) are masked.  Blocks straddling the range ends, and outputs whose
// address is not 16-byte aligned with the block grid, are stored per dword.
#pragma once

#include "orng_device.hpp"

namespace orng {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ void store16(char *p, const uint32_t w[4]) {
    u32x4 v = {w[0], w[1], w[2], w[3]};
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
    else
        *reinterpret_cast<u32x4 *>(p) = v;
}

// Store the block whose first position is p into base[q - p0], q in [p0, pend).
template <bool NT>
__device__ __forceinline__ void store_block(char *base, uint64_t p, uint64_t p0, uint64_t pend,
                                            bool aligned, const uint32_t w[4]) {
    if (aligned && p >= p0 && p + 4 <= pend) {
        store16<NT>(base + 4 * (p - p0), w);
        return;
    }
    uint32_t *o = reinterpret_cast<uint32_t *>(base);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t q = p + (uint64_t)i;
        if (q >= p0 && q < pend) o[q - p0] = w[i];
    }
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}

template <int G, int D, bool NT>
__device__ __forceinline__ void process_span(const KeySched &ks, uint32_t ctr, char *base,
                                             uint64_t p0, uint64_t pend, uint64_t span,
                                             uint32_t unroll, bool aligned, uint32_t lane) {
    if constexpr (G == G_TYCHE) {
        Tyche st;
        st.seed(ks, (uint32_t)span * 64u + lane, ctr);
        const uint64_t tile_block = span * TYCHE_TILE_BLOCKS;
        for (uint32_t k = 0; k < 64; ++k) {
            const uint64_t bw = tile_block + 64u * k;
            if (bw * 4 >= pend) break;
            uint32_t w[4];
            st.next4(w);
            const uint64_t p = (bw + lane) * 4;
            if (p + 4 <= p0) continue;
            convert4<D>(w);
            store_block<NT>(base, p, p0, pend, aligned, w);
        }
    } else {
        const uint64_t b0 = span * 64u * unroll;
        for (uint32_t u = 0; u < unroll; ++u) {
            const uint64_t bw = b0 + 64u * u;
            if (bw * 4 >= pend) break;
            if ((bw + 64) * 4 <= p0) continue;
            const uint64_t b = bw + lane;
            uint32_t w[4];
            counter_block<G>((uint32_t)b, ctr, ks, w);
            convert4<D>(w);
            store_block<NT>(base, b * 4, p0, pend, aligned, w);
        }
    }
}

// Runtime (gen, dist) dispatch for kernels whose requests mix generators.
template <bool NT>
__device__ __forceinline__ void process_span_any(int gen, int dist, const KeySched &ks,
                                                 uint32_t ctr, char *base, uint64_t p0,
                                                 uint64_t pend, uint64_t span, uint32_t unroll,
                                                 bool aligned, uint32_t lane) {
#define ORNG_CASE(G, D)                                                                    \
    case G * 3 + D:                                                                        \
        process_span<G, D, NT>(ks, ctr, base, p0, pend, span, unroll, aligned, lane);      \
        break;
    switch (gen * 3 + dist) {
        ORNG_CASE(0, 0) ORNG_CASE(0, 1) ORNG_CASE(0, 2)
        ORNG_CASE(1, 0) ORNG_CASE(1, 1) ORNG_CASE(1, 2)
        ORNG_CASE(2, 0) ORNG_CASE(2, 1) ORNG_CASE(2, 2)
        ORNG_CASE(3, 0) ORNG_CASE(3, 1) ORNG_CASE(3, 2)
        ORNG_CASE(4, 0) ORNG_CASE(4, 1) ORNG_CASE(4, 2)
        default: break;
    }
#undef ORNG_CASE
}

// Blocks per span for a generator.
__host__ __device__ inline uint64_t span_blocks(int gen, uint32_t unroll) {
    return gen == G_TYCHE ? (uint64_t)TYCHE_TILE_BLOCKS : 64ull * unroll;
}

}  // namespace orng
