/*
 * orng oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of everything the
 * counter-based generation path computes: the four generator families, the
 * stream-to-block mapping, the float32 conversions, the Box-Muller normal,
 * the fused Brownian walk, the float64 uniform and the paper's own 2-D
 * Brownian dynamics example.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  The product library never
 * links, includes or calls anything here, and nothing here includes the
 * product's headers: the two are independent transcriptions of the same
 * definitions, so that one can check the other.
 *
 * Stream model (paper, section 3.1 "API Design"): a 64-bit seed and a 32-bit
 * counter together name one stream of period 2^32.  A stream is a sequence of
 * 32-bit words indexed by a position p in [0, 2^32).  Every output is a pure
 * function of (generator, distribution, seed, counter, position): no state is
 * kept anywhere (paper, section 3.1, second paragraph; section 2 on the 96-bit
 * state), so results cannot depend on thread count or launch order
 * (paper, section 4).
 *
 * Parity status of each function (how it is pinned to something other than
 * itself) is stated in the header comment of the definition in
 * orng_oracle.cc.  Squares32 and the Tyche sequencing (init rounds, output
 * word) are "parity unpinned" with respect to external values: no
 * implementation of either exists on this machine.
 *
 * Build: g++ -std=c++17 -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (contraction off so that every float operation written here is one IEEE
 * operation; fmaf is written explicitly where a fused multiply-add is meant).
 */
#ifndef ORNG_ORACLE_H
#define ORNG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* generator and distribution codes (same numbering as the public API; the
   numbers are part of the interface, not shared code) */
enum { OR_PHILOX = 0, OR_THREEFRY4X32 = 1, OR_THREEFRY2X64 = 2, OR_SQUARES = 3, OR_TYCHE = 4,
       OR_THREEFRY4X32_13 = 5, OR_THREEFRY2X64_13 = 6, OR_TYCHE_I = 7, OR_SQUARES64 = 8,
       OR_PHILOX2X32 = 9 };
enum { OR_U32 = 0, OR_F32_UNIFORM = 1, OR_F32_NORMAL = 2, OR_F64_UNIFORM = 3, OR_F64_NORMAL = 4 };

/* --- raw generator cores ------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_philox2x32_10(const uint32_t ctr[2], uint32_t key, uint32_t out[2]);
void oracle_threefry4x32_20(const uint32_t ctr[4], const uint32_t key[4], uint32_t out[4]);
void oracle_threefry2x64_20(const uint64_t ctr[2], const uint64_t key[2], uint64_t out[2]);
void oracle_threefry4x32_13(const uint32_t ctr[4], const uint32_t key[4], uint32_t out[4]);
void oracle_threefry2x64_13(const uint64_t ctr[2], const uint64_t key[2], uint64_t out[2]);
uint32_t oracle_squares32(uint64_t ctr, uint64_t key);
uint64_t oracle_squares_key(uint64_t seed);
void oracle_tyche_mix(uint32_t st[4]);             /* st = {a, b, c, d}, in place */
void oracle_tyche_init(uint64_t seed, uint32_t c_xor, uint32_t d_xor, uint32_t st[4]);
uint32_t oracle_tyche_next(uint32_t st[4]);        /* one MIX, returns b */
void oracle_tyche_mix_i(uint32_t st[4]);           /* the inverse of MIX, in place */
void oracle_tyche_i_init(uint64_t seed, uint32_t c_xor, uint32_t d_xor, uint32_t st[4]);
uint32_t oracle_tyche_i_next(uint32_t st[4]);      /* one inverse MIX, returns b */
uint64_t oracle_squares64(uint64_t ctr, uint64_t key);  /* five rounds, 64-bit output */

/* --- stream model -------------------------------------------------------- */
/* word at position p of stream (seed, ctr) of generator gen (Philox2x32-10
   keys with the low 32 bits of seed; the entry points below reject its seeds
   of 2^32 and above) */
uint32_t oracle_word(int gen, uint64_t seed, uint32_t ctr, uint64_t p);
/* sample at position p of the given distribution; writes 4 bytes to *out
   (8 for OR_F64_UNIFORM and OR_F64_NORMAL, whose sample p is made from words
   2p and 2p+1, so their positions end at 2^31) */
void oracle_sample(int gen, int dist, uint64_t seed, uint32_t ctr, uint64_t p, void *out);

/* --- float32 conversions --------------------------------------------------- */
float oracle_u01(uint32_t x);                      /* (x >> 8) * 2^-24 */
float oracle_ln_u1(uint32_t k);                    /* ln(k * 2^-24), k in [1, 2^24] */
void oracle_sincos2pi(uint32_t k, float *c, float *s);  /* cos, sin of 2*pi*k/2^24 */
void oracle_normal_pair(uint32_t x0, uint32_t x1, float out[2]);
/* element-wise over arrays, for exhaustive tests */
void oracle_u01_n(const uint32_t *x, uint64_t n, float *out);
void oracle_ln_u1_n(const uint32_t *k, uint64_t n, float *out);
void oracle_sincos2pi_n(const uint32_t *k, uint64_t n, float *c, float *s);
void oracle_normal_pair_n(const uint32_t *x0, const uint32_t *x1, uint64_t n, float *z0, float *z1);

/* --- bulk operations (multi-threaded over disjoint output ranges only) --- */
/* out[j] = sample(offset + j) for j < n.  4 bytes per sample. */
int oracle_fill(int gen, int dist, uint64_t seed, uint32_t ctr, uint64_t offset, uint64_t n,
                void *out, int nthreads);
/* out[i*per_stream + j] = sample(offset + j) of stream (seed, ctr0 + i) */
int oracle_fill_multi(int gen, int dist, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                      uint64_t offset, uint64_t per_stream, void *out, int nthreads);
/* sampled check: out[k] = sample(pos[k]) of stream (seed, ctrs[k]) */
void oracle_samples_at(int gen, int dist, uint64_t seed, const uint32_t *ctrs,
                       const uint64_t *pos, uint64_t count, void *out, int nthreads);

/* Brownian walk, see orng_oracle.cc.  pos is SoA [dim][n_particles] (in/out).
   ids (nullable) selects particle ids; then pos is [dim][count] for those ids.
   msd (nullable) receives, for every msd_every-th step, the sum over the
   selected particles of |x|^2 (float64). */
float oracle_walk_sigma(float dt, float D);
int oracle_brownian(uint64_t seed, uint32_t ctr0, const uint32_t *ids, uint32_t count,
                    uint32_t dim, uint64_t step0, uint32_t n_steps, float dt, float D,
                    float *pos, double *msd, uint32_t msd_every, int nthreads);

/* --- the paper's 2-D Brownian dynamics (section 4, Fig. 1) ---------------- */
/* float64 uniform in [0, 1) from two consecutive words of a stream (w0 at the
   even position): the top 53 bits of (w1 << 32 | w0) times 2^-53 */
double oracle_u01_f64(uint32_t w0, uint32_t w1);
/* n_steps steps of the paper's example for particles pid0 + (ids ? ids[k] : k),
   k < count; state arrays x, y, vx, vy (count entries each, float64) are
   updated in place.  c = gamma / mass.  Returns 0, or -2 if a counter
   step0 + s would pass 2^32 - 1. */
int oracle_bd2(uint64_t pid0, const uint32_t *ids, uint32_t count, uint32_t step0,
               uint32_t n_steps, double dt, double c, double *x, double *y, double *vx,
               double *vy, int nthreads);

/* --- parallel micro-streams (section 5.2) ---------------------------------- */
/* out[((t * n_particles) + p) * draws + k] = word k of stream
   (seed0 + p, ctr0 + t) of generator gen, for t < n_iters, p < n_particles,
   k < draws.  Returns 0, -1 (gen, draws not in 1..16) or -2 (counter or
   seed range overflows). */
int oracle_particle_streams(int gen, uint64_t seed0, uint32_t n_particles, uint32_t draws,
                            uint32_t ctr0, uint32_t n_iters, uint32_t *out, int nthreads);

/* --- float64 Box-Muller normals (see orng_oracle.cc) --------------------- */
double oracle_ln_u1_f64(uint64_t K);               /* ln(K 2^-53), K in [1, 2^53] */
void oracle_sincos_turn_f64(uint64_t k, double *c, double *s); /* of 2 pi k 2^-53, k < 2^53 */
void oracle_normal_pair_f64(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, double out[2]);
void oracle_ln_u1_f64_n(const uint64_t *K, uint64_t n, double *out);
void oracle_sincos_turn_f64_n(const uint64_t *k, uint64_t n, double *c, double *s);

/* --- integers in [lo, hi) (section 3: standard-distribution use) --------- */
/* sample from two consecutive words of a stream (w0 at the even position):
   lo + floor(x * (hi - lo) / 2^64) with x = (w1 << 32) | w0.  lo < hi. */
int32_t oracle_range_i32(uint32_t w0, uint32_t w1, int32_t lo, int32_t hi);
/* out[i*per_stream + j] = integer sample (offset + j) of stream (seed, ctr0 + i);
   sample p is made from words 2p and 2p+1, so positions end at 2^31.
   Returns 0, -1 (gen, or lo >= hi) or -2 (position or counter range). */
int oracle_fill_range(int gen, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                      uint64_t offset, uint64_t per_stream, int32_t lo, int32_t hi,
                      int32_t *out, int nthreads);

#ifdef __cplusplus
}
#endif

#endif /* ORNG_ORACLE_H */
