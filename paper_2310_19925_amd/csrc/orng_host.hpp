// Host-side definitions shared by the library's translation units and by its
// host-only tests: generator and distribution ids, the stream's word
// arithmetic, span sizes, and request validation.  Plain C++ with no HIP
// dependency (the device headers include it; constexpr functions here are
// usable in device code as well).
#pragma once

#include <stdint.h>

#include "../../include/orng.h"

namespace orng {

enum GenId : int { G_PHILOX = 0, G_TF4X32 = 1, G_TF2X64 = 2, G_SQUARES = 3, G_TYCHE = 4,
                   G_TF4X32_13 = 5, G_TF2X64_13 = 6, G_TYCHE_I = 7, G_SQUARES64 = 8,
                   G_PHILOX2X32 = 9 };
enum DistId : int { D_U32 = 0, D_UNIFORM = 1, D_NORMAL = 2, D_F64U = 3, D_F64N = 4,
                    D_I32R = 5 };
// NDIST: distributions of the fill kernels and launch tables; request records
// (batched and served) also take D_I32R, integers in [lo, hi), whose bounds
// they carry.
constexpr int NGEN = 10, NDIST = 5, NREQDIST = 6;

// Tyche and Tyche-i share the tile layout (no random access within a
// substream); every other generator is counter-based with 4-word blocks.
constexpr bool tyche_like(int g) { return g == G_TYCHE || g == G_TYCHE_I; }

constexpr uint32_t TYCHE_TILE_WORDS = 16384;
constexpr uint32_t TYCHE_TILE_BLOCKS = 4096;

constexpr uint64_t PERIOD = 1ull << 32;

// Stream words per sample: a float64 sample is made from the word pair
// (2p, 2p+1) (a float64 normal pair from the block 4m..4m+3), and so is an
// integer in [lo, hi); every other distribution from one word.  The public
// calls take offsets and counts in samples and convert them to words
// (positions) once; below that, every launcher and kernel works in words.
inline uint64_t words_per_sample(int dist) { return dist >= D_F64U ? 2 : 1; }
inline uint64_t sample_limit(int dist) { return PERIOD / words_per_sample(dist); }
// Output bytes per sample: 8 for the float64 distributions, 4 otherwise.
inline uint64_t bytes_per_sample(int dist) { return dist == D_F64U || dist == D_F64N ? 8 : 4; }
// The launch-table row a request's distribution takes in the batched and
// served paths: integers in [lo, hi) read the same two words per sample as
// float64 uniforms and use that row.
inline int shape_dist(int dist) { return dist == D_I32R ? D_F64U : dist; }

// Philox2x32-10 keys with one 32-bit word: its seeds must be below 2^32.
inline bool seed_ok(int gen, uint64_t seed) { return gen != G_PHILOX2X32 || seed <= 0xFFFFFFFFull; }

// Blocks (of four words) per span for a generator: 64 per unit of `unroll`,
// or one Tyche tile.
constexpr uint64_t span_blocks(int gen, uint32_t unroll) {
    return tyche_like(gen) ? (uint64_t)TYCHE_TILE_BLOCKS : 64ull * unroll;
}

// A request record as orng_fill / orng_fill_range would take it: ORNG_OK or
// the error those calls return.
inline int validate_request(const orng_req_t &r) {
    if (r.gen > ORNG_PHILOX2X32 || r.dist > ORNG_I32_RANGE || r.flags != 0) return ORNG_EINVAL;
    if (!seed_ok((int)r.gen, r.seed)) return ORNG_EINVAL;
    if (r.dist == ORNG_I32_RANGE && r.lo >= r.hi) return ORNG_EINVAL;
    const uint64_t lim = sample_limit((int)r.dist);
    if (r.offset > lim || r.n > lim - r.offset) return ORNG_ERANGE;
    if (r.n == 0) return ORNG_OK;
    if (!r.out || (reinterpret_cast<uintptr_t>(r.out) & (bytes_per_sample((int)r.dist) - 1)))
        return ORNG_EINVAL;
    return ORNG_OK;
}

// Kernel-side bounds of an integer-range request: lo's bits and r = hi - lo.
inline void range_bounds(const orng_req_t &r, uint32_t *lo, uint32_t *rr) {
    const bool on = r.dist == ORNG_I32_RANGE;
    *lo = on ? (uint32_t)r.lo : 0u;
    *rr = on ? (uint32_t)((int64_t)r.hi - (int64_t)r.lo) : 0u;
}

// (address of out in words - first position) mod 4: the alignment class of a
// request's output against its block grid, in words; for integer ranges,
// whose output samples are one word each, against its sample grid.
inline uint32_t output_delta(const orng_req_t &r, const void *out) {
    const uint64_t addr_words = reinterpret_cast<uintptr_t>(out) / 4;
    const uint64_t first =
        r.dist == ORNG_I32_RANGE ? r.offset : r.offset * words_per_sample((int)r.dist);
    return (uint32_t)((addr_words - first) & 3u);
}

}  // namespace orng
