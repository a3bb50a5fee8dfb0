// Span processing shared by the fill, batched and served kernels.
//
// A span is the unit of work of one wave.  Counter-based generators: 64*U
// consecutive blocks of four words, block span*64U + u*64 + lane in iteration
// u, so every 16-byte store instruction of the wave covers 1 KiB of
// contiguous output.  Tyche: one 16384-word tile, lane l stepping its own
// substream through blocks k*64 + l, k = 0..63 (the Tyche stream layout).
// Spans are numbered in absolute block space of the stream; blocks outside
// [p0, pend) are masked.  Blocks straddling the range ends, and outputs whose
// address is not 16-byte aligned with the block grid, go through SpanOut.
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

// Output writer of one span.  delta = (output address in words - p0) mod 4.
// delta == 0: block b maps onto one 16-byte chunk.  delta != 0: the chunk
// that holds the head of block b also holds the last delta words of block
// b - 1; lane l takes them from lane l - 1 and lane 0 from lane 63 of the
// previous iteration (carried in uniform registers), so every interior chunk
// is still one 16-byte store.  The shift is a DPP whole-wave shift right by
// one lane (a VALU move; lane 0, which has no source lane, keeps the `old`
// operand, the carry): on MI355X the LDS permute it replaces put a wait for
// the LDS unit between every block and its store.  Lane 63 writes its block's tail
// itself when no further iteration of the span follows; lane 0 of the first
// iteration writes only its own words.  Positions outside [p0, pend) are never
// written.
struct SpanOut {
    char *base;
    uint64_t p0, pend;
    uint32_t delta;
    bool have_carry;
    uint32_t carry[4];
};

template <bool NT>
__device__ __forceinline__ void put_word(const SpanOut &o, int64_t q, uint32_t v) {
    if (q >= (int64_t)o.p0 && q < (int64_t)o.pend)
        reinterpret_cast<uint32_t *>(o.base)[q - (int64_t)o.p0] = v;
}

template <bool NT>
__device__ __forceinline__ void emit_block(SpanOut &o, uint64_t b, const uint32_t w[4],
                                           uint32_t lane, bool last_iter) {
    if (o.delta == 0) {
        store_block<NT>(o.base, b * 4, o.p0, o.pend, true, w);
        return;
    }
    const int d = (int)o.delta;
    uint32_t prev[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)  // wave_shr:1, all rows and banks, no bound_ctrl
        prev[j] = (uint32_t)__builtin_amdgcn_update_dpp((int)o.carry[j], (int)w[j], 0x138, 0xF,
                                                        0xF, false);
    const bool prev_ok = lane > 0 || o.have_carry;
    const int64_t q0 = (int64_t)(b * 4) - d;  // first position of the chunk
    // chunk word j (position q0 + j) comes from the previous block if j < d.
    // The words are taken into scalars first and chosen by the uniform d:
    // selecting array elements by a run-time index instead let the compiler
    // keep the block in scratch memory when it holds split float64 values.
    const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
    const uint32_t p1 = prev[1], p2 = prev[2], p3 = prev[3];
    uint32_t v[4];
    if (d == 1) {
        v[0] = p3; v[1] = w0; v[2] = w1; v[3] = w2;
    } else if (d == 2) {
        v[0] = p2; v[1] = p3; v[2] = w0; v[3] = w1;
    } else {
        v[0] = p1; v[1] = p2; v[2] = p3; v[3] = w0;
    }
    if (prev_ok && q0 >= (int64_t)o.p0 && q0 + 4 <= (int64_t)o.pend) {
        store16<NT>(o.base + 4 * (q0 - (int64_t)o.p0), v);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j >= d || prev_ok) put_word<NT>(o, q0 + j, v[j]);
    }
    if (last_iter && lane == 63) {
        // tail of this block: words 4 - d .. 3 at positions 4b + 4 - d .. 4b + 3
#pragma unroll
        for (int j = 1; j <= 3; ++j)
            if (j <= d) put_word<NT>(o, (int64_t)(b * 4) + 4 - j, w[4 - j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) o.carry[j] = __builtin_amdgcn_readlane(w[j], 63);
    o.have_carry = true;
}

// FAST: compile in the check-free loop for spans wholly inside the range on
// the block grid (the plain fill kernel; 1: two blocks per iteration, 2: one);
// the batched and served kernels, whose outputs are mostly off the grid, leave
// it out (0) to keep their register counts (34 instead of 58-59 VGPRs).
template <int G, int D, bool NT, int FAST = 0>
__device__ __forceinline__ void process_span(const KeySched &ks, uint32_t ctr, char *base,
                                             uint64_t p0, uint64_t pend, uint64_t span,
                                             uint32_t unroll, uint32_t delta, uint32_t lane) {
    SpanOut o;
    o.base = base;
    o.p0 = p0;
    o.pend = pend;
    o.delta = delta;
    o.have_carry = false;
    o.carry[0] = o.carry[1] = o.carry[2] = o.carry[3] = 0;
    // Counter generators: where the next iteration's block is also in range,
    // two blocks are made and converted before either is emitted; their work
    // is independent, which gives the scheduler twice the instruction-level
    // parallelism (four Box-Muller pairs instead of two; the Threefry4x32
    // normal fill gains ~5% on MI355X).  Emission stays in block order.  Tyche's
    // words come from one sequential state, so it keeps one block per step.
    // A span wholly inside [p0, pend) whose output lies on the block grid
    // (delta == 0) -- every span of an aligned fill but its first and last --
    // takes a loop with no per-block range checks or carries: the store
    // address steps by 1 KiB per iteration.  On MI355X the checks and 64-bit
    // address arithmetic of the general path cost ~3.5 instructions per word,
    // a quarter of a Squares32 word's arithmetic.
    if constexpr (tyche_like(G)) {
        TycheT<G == G_TYCHE_I> st;
        st.seed(ks, (uint32_t)span * 64u + lane, ctr);
        const uint64_t tile_block = span * TYCHE_TILE_BLOCKS;
        if (FAST != 0 && delta == 0 && tile_block * 4 >= p0 &&
            (tile_block + TYCHE_TILE_BLOCKS) * 4 <= pend) {
            char *q = base + 4 * ((tile_block + lane) * 4 - p0);
            for (uint32_t k = 0; k < 64; ++k) {
                uint32_t w[4];
                st.next4(w);
                convert4<D>(w);
                store16<NT>(q, w);
                q += 1024;
            }
            return;
        }
        for (uint32_t k = 0; k < 64; ++k) {
            const uint64_t bw = tile_block + 64u * k;
            if (bw * 4 >= pend) break;
            uint32_t w[4];
            st.next4(w);
            if ((bw + 64) * 4 <= p0) {  // whole iteration before p0
                o.have_carry = false;
                continue;
            }
            convert4<D>(w);
            const bool last = k == 63 || (bw + 64) * 4 >= pend;
            emit_block<NT>(o, bw + lane, w, lane, last);
        }
    } else {
        const uint64_t b0 = span * 64u * unroll;
        if (FAST != 0 && delta == 0 && b0 * 4 >= p0 && (b0 + 64u * unroll) * 4 <= pend) {
            char *q = base + 4 * ((b0 + lane) * 4 - p0);
            uint32_t b = (uint32_t)(b0 + lane);
            uint32_t u = 0;
            if constexpr (FAST == 2) {
                for (; u < unroll; ++u) {
                    uint32_t w[4];
                    counter_block<G>(b, ctr, ks, w);
                    convert4<D>(w);
                    store16<NT>(q, w);
                    q += 1024;
                    b += 64u;
                }
                return;
            }
            for (; u + 1 < unroll; u += 2) {
                uint32_t w[4], w2[4];
                counter_block<G>(b, ctr, ks, w);
                counter_block<G>(b + 64u, ctr, ks, w2);
                convert4<D>(w);
                convert4<D>(w2);
                store16<NT>(q, w);
                store16<NT>(q + 1024, w2);
                q += 2048;
                b += 128u;
            }
            if (u < unroll) {
                uint32_t w[4];
                counter_block<G>(b, ctr, ks, w);
                convert4<D>(w);
                store16<NT>(q, w);
            }
            return;
        }
        for (uint32_t u = 0; u < unroll;) {
            const uint64_t bw = b0 + 64u * u;
            if (bw * 4 >= pend) break;
            if ((bw + 64) * 4 <= p0) {
                o.have_carry = false;
                ++u;
                continue;
            }
            const uint64_t b = bw + lane;
            uint32_t w[4];
            if (u + 1 < unroll && (bw + 64) * 4 < pend) {
                uint32_t w2[4];
                counter_block<G>((uint32_t)b, ctr, ks, w);
                counter_block<G>((uint32_t)(b + 64), ctr, ks, w2);
                convert4<D>(w);
                convert4<D>(w2);
                emit_block<NT>(o, b, w, lane, false);
                const bool last = u + 2 == unroll || (bw + 128) * 4 >= pend;
                emit_block<NT>(o, b + 64, w2, lane, last);
                u += 2;
                continue;
            }
            counter_block<G>((uint32_t)b, ctr, ks, w);
            convert4<D>(w);
            const bool last = u + 1 == unroll || (bw + 64) * 4 >= pend;
            emit_block<NT>(o, b, w, lane, last);
            ++u;
        }
    }
}

// Store the N (2 or 4) int32 samples whose first sample number is q into
// base[q - s0], q in [s0, send): one 8- or 16-byte store when the whole group
// is in range and `aligned` (the address of sample q is a multiple of 4 N
// bytes), else one masked word at a time.
template <int N, bool NT>
__device__ __forceinline__ void store_samples(int32_t *base, uint64_t q, uint64_t s0,
                                              uint64_t send, bool aligned, const uint32_t v[N]) {
    static_assert(N == 2 || N == 4, "sample group");
    if (aligned && q >= s0 && q + N <= send) {
        if constexpr (N == 4) {
            store16<NT>(reinterpret_cast<char *>(base + (q - s0)), v);
        } else {
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            u32x2 x = {v[0], v[1]};
            u32x2 *p = reinterpret_cast<u32x2 *>(base + (q - s0));
            if constexpr (NT)
                __builtin_nontemporal_store(x, p);
            else
                *p = x;
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (q + i >= s0 && q + i < send) base[q + i - s0] = (int32_t)v[i];
}

// A span of integer samples in [lo, hi) (D_I32R), in the span numbering of
// process_span: block b of the stream gives samples 2b and 2b + 1 (its word
// pairs), so p0 and pend, in words, are twice the first and end sample.
// Counter generators: where two iterations of the span remain, lane l makes
// the adjacent blocks bw + 2l and bw + 2l + 1 of the 128-block window, so its
// four samples are one 16-byte store and the wave writes 1 KiB per store
// instruction; a last single iteration makes block bw + l (one 8-byte store).
// Tyche: block k*64 + l of the tile from lane l's substream, one 8-byte store.
// mis = (output address in words - first sample) mod 4 decides which
// stores are aligned; samples outside the range are never written.
template <int G, bool NT>
__device__ __forceinline__ void process_span_range(const KeySched &ks, uint32_t ctr,
                                                   int32_t *base, uint64_t p0, uint64_t pend,
                                                   uint64_t span, uint32_t unroll,
                                                   uint32_t mis, uint32_t lane, uint32_t lo,
                                                   uint32_t r) {
    const uint64_t s0 = p0 / 2, send = pend / 2;
    const bool al2 = (mis & 1u) == 0, al4 = mis == 0;
    if constexpr (tyche_like(G)) {
        TycheT<G == G_TYCHE_I> st;
        st.seed(ks, (uint32_t)span * 64u + lane, ctr);
        const uint64_t tile_block = span * TYCHE_TILE_BLOCKS;
        for (uint32_t k = 0; k < 64; ++k) {
            const uint64_t bw = tile_block + 64u * k;
            if (2 * bw >= send) break;
            uint32_t w[4];
            st.next4(w);
            if (2 * (bw + 64) <= s0) continue;
            const uint32_t v[2] = {range_sample(w[0], w[1], r, lo), range_sample(w[2], w[3], r, lo)};
            store_samples<2, NT>(base, 2 * (bw + lane), s0, send, al2, v);
        }
    } else {
        const uint64_t b0 = span * 64u * unroll;
        for (uint32_t u = 0; u < unroll;) {
            const uint64_t bw = b0 + 64u * u;
            if (2 * bw >= send) break;
            if (u + 1 < unroll) {
                if (2 * (bw + 128) > s0) {
                    const uint64_t b = bw + 2u * lane;
                    uint32_t w[4], x[4];
                    counter_block<G>((uint32_t)b, ctr, ks, w);
                    counter_block<G>((uint32_t)(b + 1), ctr, ks, x);
                    const uint32_t v[4] = {range_sample(w[0], w[1], r, lo),
                                           range_sample(w[2], w[3], r, lo),
                                           range_sample(x[0], x[1], r, lo),
                                           range_sample(x[2], x[3], r, lo)};
                    store_samples<4, NT>(base, 2 * b, s0, send, al4, v);
                }
                u += 2;
                continue;
            }
            if (2 * (bw + 64) > s0) {
                const uint64_t b = bw + lane;
                uint32_t w[4];
                counter_block<G>((uint32_t)b, ctr, ks, w);
                const uint32_t v[2] = {range_sample(w[0], w[1], r, lo),
                                       range_sample(w[2], w[3], r, lo)};
                store_samples<2, NT>(base, 2 * b, s0, send, al2, v);
            }
            ++u;
        }
    }
}

// Workgroups are dealt to the 8 XCDs of the device round-robin (workgroup b
// runs on XCD b mod 8); the batched and served launchers round their grids to
// a multiple of this.
constexpr uint32_t XCDS = 8;

// Runtime (gen, dist) dispatch for kernels whose requests mix generators.
// F64N and RNG select whether the float64 normal and the integer-range cases
// are compiled in: the float64 normal code needs more than twice the vector
// registers of every other case, the range cases raise the persistent batched
// kernel's count too, and a kernel's register count (so its occupancy) is that
// of its largest case, so the launchers use a variant without them unless a
// request needs them.  lo and r (= hi - lo) are read by the range cases only.
template <bool NT, bool F64N, bool RNG>
__device__ __forceinline__ void process_span_any(int gen, int dist, const KeySched &ks,
                                                 uint32_t ctr, char *base, uint64_t p0,
                                                 uint64_t pend, uint64_t span, uint32_t unroll,
                                                 uint32_t delta, uint32_t lane, uint32_t lo,
                                                 uint32_t r) {
#define ORNG_CASE(G, D)                                                                    \
    case G * 8 + D:                                                                        \
        process_span<G, D, NT>(ks, ctr, base, p0, pend, span, unroll, delta, lane);        \
        break;
#define ORNG_RCASE(G)                                                                      \
    case G * 8 + D_I32R:                                                                   \
        process_span_range<G, NT>(ks, ctr, reinterpret_cast<int32_t *>(base), p0, pend,    \
                                  span, unroll, delta, lane, lo, r);                       \
        break;
    switch (gen * 8 + dist) {
        ORNG_CASE(0, 0) ORNG_CASE(0, 1) ORNG_CASE(0, 2) ORNG_CASE(0, 3)
        ORNG_CASE(1, 0) ORNG_CASE(1, 1) ORNG_CASE(1, 2) ORNG_CASE(1, 3)
        ORNG_CASE(2, 0) ORNG_CASE(2, 1) ORNG_CASE(2, 2) ORNG_CASE(2, 3)
        ORNG_CASE(3, 0) ORNG_CASE(3, 1) ORNG_CASE(3, 2) ORNG_CASE(3, 3)
        ORNG_CASE(4, 0) ORNG_CASE(4, 1) ORNG_CASE(4, 2) ORNG_CASE(4, 3)
        ORNG_CASE(5, 0) ORNG_CASE(5, 1) ORNG_CASE(5, 2) ORNG_CASE(5, 3)
        ORNG_CASE(6, 0) ORNG_CASE(6, 1) ORNG_CASE(6, 2) ORNG_CASE(6, 3)
        ORNG_CASE(7, 0) ORNG_CASE(7, 1) ORNG_CASE(7, 2) ORNG_CASE(7, 3)
        ORNG_CASE(8, 0) ORNG_CASE(8, 1) ORNG_CASE(8, 2) ORNG_CASE(8, 3)
        ORNG_CASE(9, 0) ORNG_CASE(9, 1) ORNG_CASE(9, 2) ORNG_CASE(9, 3)
        default:
            if constexpr (F64N) {
                switch (gen * 8 + dist) {
                    ORNG_CASE(0, 4) ORNG_CASE(1, 4) ORNG_CASE(2, 4) ORNG_CASE(3, 4)
                    ORNG_CASE(4, 4) ORNG_CASE(5, 4) ORNG_CASE(6, 4) ORNG_CASE(7, 4)
                    ORNG_CASE(8, 4) ORNG_CASE(9, 4)
                    default: break;
                }
            }
            if constexpr (RNG) {
                switch (gen * 8 + dist) {
                    ORNG_RCASE(0) ORNG_RCASE(1) ORNG_RCASE(2) ORNG_RCASE(3) ORNG_RCASE(4)
                    ORNG_RCASE(5) ORNG_RCASE(6) ORNG_RCASE(7) ORNG_RCASE(8) ORNG_RCASE(9)
                    default: break;
                }
            }
            break;
    }
#undef ORNG_CASE
#undef ORNG_RCASE
}


}  // namespace orng
