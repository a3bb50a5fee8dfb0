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

// Workgroups of `wg` threads that cover n items, rounded up in 64 bits so that
// counts up to 2^32 - 1 do not wrap.
constexpr uint32_t blocks_for(uint32_t n, uint32_t wg) {
    return (uint32_t)(((uint64_t)n + wg - 1) / wg);
}
static_assert(blocks_for(0xFFFFFFFFu, 256) == 1u << 24 && blocks_for(257, 256) == 2 &&
                  blocks_for(0, 64) == 0,
              "workgroup counts round up without wrapping");

// A dispatch holds its grid size per dimension in work-items, as a 32-bit
// count: one dimension takes at most max_wgs_1d(wg) workgroups of wg threads.
constexpr uint32_t max_wgs_1d(uint32_t wg) { return (uint32_t)(0xFFFFFFFFull / wg); }

// `blocks` workgroups as a 2-D grid (x fastest, so the linear workgroup id
// y * x_dim + x counts them in dispatch order; it stays below 2^32 for
// blocks < 2^32 - 2^16): one row up to 2^16 workgroups, then rows of at most
// 2^16.  x * y >= blocks, with fewer than y workgroups beyond `blocks`; the
// kernels return from those.
struct Grid2 {
    uint32_t x, y;
};
constexpr Grid2 grid_2d(uint64_t blocks) {
    const uint64_t row = 65536;
    const uint64_t rows = (blocks + row - 1) / row;       // at least 1 for blocks > 0
    if (rows <= 1) return Grid2{(uint32_t)blocks, 1u};
    const uint64_t per_row = (blocks + rows - 1) / rows;  // <= row
    return Grid2{(uint32_t)per_row, (uint32_t)rows};
}
static_assert(grid_2d(100).x == 100 && grid_2d(100).y == 1, "one row");
static_assert((uint64_t)grid_2d((1ull << 32) - 1).x * grid_2d((1ull << 32) - 1).y >=
                      (1ull << 32) - 1 &&
                  grid_2d((1ull << 32) - 1).x <= 65536,
              "rows cover every workgroup");

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
