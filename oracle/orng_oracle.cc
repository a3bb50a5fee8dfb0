/*
 * orng oracle -- TEST INFRASTRUCTURE ONLY (see orng_oracle.h).
 *
 * Every function is written as the plain definition, one word or one sample
 * at a time, in the order the defining source states it.  The only
 * parallelism is a split of the output range over std::thread, which cannot
 * change any value because each output is a pure function of its position.
 *
 * Sources.  The paper (OpenRAND, arXiv 2310.19925) names the generators
 * (section 3.1) and the stream model but defines none of them; the round
 * functions come from the primary publications the paper cites:
 *   Philox, Threefry : Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers:
 *                      As Easy as 1, 2, 3", SC'11 (sections 3.2-3.3).
 *   Squares          : Widynski, "Squares: A Fast Counter-Based RNG",
 *                      arXiv:2004.06278 (the 32-bit output, four-round form).
 *   Tyche            : Neves, Araujo, "Fast and Small Nonlinear Pseudorandom
 *                      Number Generators for Computer Simulation", PPAM 2011.
 * Stream layouts, the float conversions and the walk are readings of the
 * paper where it is silent; each is stated where it is defined.
 */
#include "orng_oracle.h"

#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace {

inline uint32_t rotl32(uint32_t x, unsigned r) { return (x << r) | (x >> (32u - r)); }
inline uint64_t rotl64(uint64_t x, unsigned r) { return (x << r) | (x >> (64u - r)); }

/* ---------------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11, section 3.3).
 * One round multiplies the even lanes by two odd constants, and builds the new
 * block from the high halves XOR the odd lanes XOR the round key, and the low
 * halves.  The key is bumped by two Weyl constants between rounds.
 * Pinned: rocRAND's Philox engine (built host-only in the test-suite) on
 * random keys and counters, and the big-integer transcription.
 * ------------------------------------------------------------------------- */
const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void philox_round(uint32_t x[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * x[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ k[0];
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x[3] ^ k[1];
    uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

/* ---------------------------------------------------------------------------
 * Philox2x32-10 (same source): the two-word member of the Philox family.  One
 * round multiplies the first word by one odd constant; the new first word is
 * the product's high half XOR the second word XOR the 32-bit round key, the
 * new second word is its low half.  The key is bumped by the first Weyl
 * constant between rounds.  Its key is a single 32-bit word, so this library
 * offers it for seeds below 2^32 (the paper's Squares is likewise limited to
 * 32-bit seeds, section 3.1).  Parity unpinned (no implementation of it is at
 * hand); pinned by round inversion, distinct outputs over enumerated
 * counters and statistics.
 * ------------------------------------------------------------------------- */
const uint32_t PHILOX2_M = 0xD256D193u;

/* ---------------------------------------------------------------------------
 * Threefry4x32-20 (Salmon et al., SC'11, section 3.2; Threefish-style ARX).
 * Key schedule: four key words plus their XOR with the Skein parity constant.
 * The key is injected before round 0 and after every fourth round, with the
 * injection number added to the last word.  Rotation pairs repeat with
 * period 8; even rounds mix (0,1),(2,3), odd rounds mix (0,3),(2,1) (the
 * Threefish word permutation after every round).
 * Pinned in two steps: rocRAND's Threefry4x32-20 switches mixing pairs every
 * second round, so a big-integer transcription run with rocRAND's schedule
 * is checked against rocRAND (rotations, key schedule, parity constant,
 * injections), and the same transcription with the schedule above is checked
 * against this function.
 * ------------------------------------------------------------------------- */
const unsigned TF4_ROT[8][2] = {{10, 26}, {11, 21}, {13, 27}, {23, 5},
                                {6, 20},  {17, 11}, {25, 10}, {18, 20}};
const uint32_t SKEIN_PARITY32 = 0x1BD11BDAu;

/* ---------------------------------------------------------------------------
 * Threefry2x64-20 (same source): two 64-bit words, one mix per round,
 * rotations 16 42 12 31 16 32 24 21, 64-bit Skein parity constant.
 * Pinned: rocRAND's Threefry2x64-20 rounds on random keys/counters.
 * ------------------------------------------------------------------------- */
const unsigned TF2_ROT[8] = {16, 42, 12, 31, 16, 32, 24, 21};
const uint64_t SKEIN_PARITY64 = 0x1BD11BDAA9FC1A22ull;

/* ---------------------------------------------------------------------------
 * Tyche (Neves and Araujo, PPAM 2011).  The state is four 32-bit words; the
 * MIX function is the ChaCha quarter round (add, xor, rotate by 16, 12, 8, 7).
 * Seeding puts the seed's high and low halves in a and b, the constants
 * floor(2^32/phi) and floor(2^32/pi) in c and d (d XOR a 32-bit index), then
 * applies MIX twenty times.  Each output applies MIX once and returns b.
 * Pinned: MIX against OpenSSL's ChaCha20 keystream (a ChaCha20 block built
 * from this MIX in the test-suite); the two constants against their closed
 * forms.  The init count and the output word are parity unpinned.
 * ------------------------------------------------------------------------- */
const uint32_t TYCHE_C0 = 2654435769u; /* floor(2^32 / golden ratio) */
const uint32_t TYCHE_D0 = 1367130551u; /* floor(2^32 / pi) */

/* ---------------------------------------------------------------------------
 * Tyche stream layout (reading; the paper gives a 32-bit counter per stream
 * but Tyche has no random access).  A stream is cut into tiles of
 * T = 16384 words.  Within tile t, word offset r = p mod T belongs to lane
 * l = (r / 4) mod 64, block k = r / 256, word w = r mod 4, and equals output
 * number 4k + w of the Tyche instance seeded with (seed, index = ctr) whose c
 * word is additionally XORed with the substream number t*64 + l.
 * Substream 0 is exactly textbook Tyche(seed, ctr).
 * ------------------------------------------------------------------------- */
const uint64_t TYCHE_TILE = 16384, TYCHE_LANES = 64, TYCHE_BLOCKS = 64;

/* ---------------------------------------------------------------------------
 * Squares key derivation (reading; the paper notes Squares takes a 32-bit
 * seed, without saying how it becomes a key).  Here the 64-bit seed is mapped
 * through one SplitMix64 output step (Steele, Lea, Flood, OOPSLA 2014: add the
 * 64-bit golden-ratio increment, then the two xor-shift-multiply rounds and a
 * final xor-shift) and the low bit is forced to 1.  The finalizer (its
 * constants and shifts) is pinned to pybind11's own implementation of it
 * (test_squares_key_vs_pybind11_splitmix64); the increment and the low bit
 * are the reading.
 * ------------------------------------------------------------------------- */

/* ---------------------------------------------------------------------------
 * Counter-based block for position p (reading of the stream model, section
 * 3.1: 64-bit seed + 32-bit counter, period 2^32 words):
 *   Philox4x32-10   : counter (p/4, ctr, 0, 0), key (lo seed, hi seed)
 *   Threefry4x32-20 : counter (p/4, ctr, 0, 0), key (lo seed, hi seed, 0, 0)
 *   Threefry2x64-20 : counter (p/4, ctr) as 64-bit words, key (seed, 0);
 *                     the four 32-bit words are lo X0, hi X0, lo X1, hi X1
 *   the 13-round Threefry variants: as their 20-round forms
 *   Philox2x32-10   : word p is word p mod 2 of Philox2x32(counter (p/2, ctr),
 *                     key lo seed); the block of four words p/4 holds the
 *                     two-word blocks 2(p/4) and 2(p/4) + 1
 * word(p) is word p mod 4 of that block.
 * ------------------------------------------------------------------------- */
void counter_block(int gen, uint64_t seed, uint32_t ctr, uint64_t b, uint32_t out[4]) {
    uint32_t lo = (uint32_t)seed, hi = (uint32_t)(seed >> 32);
    if (gen == OR_PHILOX2X32) {
        for (uint64_t h = 0; h < 2; ++h) {
            const uint32_t c[2] = {(uint32_t)(2 * b + h), ctr};
            oracle_philox2x32_10(c, lo, out + 2 * h);
        }
    } else if (gen == OR_PHILOX) {
        uint32_t c[4] = {(uint32_t)b, ctr, 0u, 0u};
        uint32_t k[2] = {lo, hi};
        oracle_philox4x32_10(c, k, out);
    } else if (gen == OR_THREEFRY4X32 || gen == OR_THREEFRY4X32_13) {
        uint32_t c[4] = {(uint32_t)b, ctr, 0u, 0u};
        uint32_t k[4] = {lo, hi, 0u, 0u};
        if (gen == OR_THREEFRY4X32) oracle_threefry4x32_20(c, k, out);
        else oracle_threefry4x32_13(c, k, out);
    } else { /* OR_THREEFRY2X64, OR_THREEFRY2X64_13 */
        uint64_t c[2] = {b, (uint64_t)ctr};
        uint64_t k[2] = {seed, 0ull};
        uint64_t r[2];
        if (gen == OR_THREEFRY2X64) oracle_threefry2x64_20(c, k, r);
        else oracle_threefry2x64_13(c, k, r);
        out[0] = (uint32_t)r[0];
        out[1] = (uint32_t)(r[0] >> 32);
        out[2] = (uint32_t)r[1];
        out[3] = (uint32_t)(r[1] >> 32);
    }
}

/* raw words of positions [p0, p0 + count) into dst */
void words_range(int gen, uint64_t seed, uint32_t ctr, uint64_t p0, uint64_t count, uint32_t *dst) {
    if (count == 0) return;
    const uint64_t p1 = p0 + count;
    if (gen == OR_SQUARES) {
        const uint64_t key = oracle_squares_key(seed);
        for (uint64_t p = p0; p < p1; ++p)
            dst[p - p0] = oracle_squares32(((uint64_t)ctr << 32) | p, key);
    } else if (gen == OR_SQUARES64) {
        /* word p is the low (p even) or high half of call p/2 */
        const uint64_t key = oracle_squares_key(seed);
        for (uint64_t p = p0; p < p1; ++p) {
            const uint64_t v = oracle_squares64(((uint64_t)ctr << 32) | (p / 2), key);
            dst[p - p0] = (uint32_t)(p & 1 ? v >> 32 : v);
        }
    } else if (gen == OR_TYCHE || gen == OR_TYCHE_I) {
        const bool inv = gen == OR_TYCHE_I;
        /* walk every substream (tile, lane) that owns a position in range */
        for (uint64_t t = p0 / TYCHE_TILE; t * TYCHE_TILE < p1; ++t) {
            for (uint64_t l = 0; l < TYCHE_LANES; ++l) {
                uint32_t st[4];
                if (inv) oracle_tyche_i_init(seed, (uint32_t)(t * TYCHE_LANES + l), ctr, st);
                else oracle_tyche_init(seed, (uint32_t)(t * TYCHE_LANES + l), ctr, st);
                for (uint64_t k = 0; k < TYCHE_BLOCKS; ++k) {
                    for (uint64_t w = 0; w < 4; ++w) {
                        uint32_t v = inv ? oracle_tyche_i_next(st) : oracle_tyche_next(st);
                        uint64_t p = t * TYCHE_TILE + (k * TYCHE_LANES + l) * 4 + w;
                        if (p >= p0 && p < p1) dst[p - p0] = v;
                    }
                }
            }
        }
    } else {
        for (uint64_t b = p0 / 4; b * 4 < p1; ++b) {
            uint32_t blk[4];
            counter_block(gen, seed, ctr, b, blk);
            for (uint64_t w = 0; w < 4; ++w) {
                uint64_t p = b * 4 + w;
                if (p >= p0 && p < p1) dst[p - p0] = blk[w];
            }
        }
    }
}

/* samples of positions [p0, p0 + count) into dst (4 bytes each) */
void samples_range(int gen, int dist, uint64_t seed, uint32_t ctr, uint64_t p0, uint64_t count,
                   void *dst) {
    if (count == 0) return;
    if (dist == OR_U32) {
        words_range(gen, seed, ctr, p0, count, (uint32_t *)dst);
        return;
    }
    if (dist == OR_F32_UNIFORM) {
        std::vector<uint32_t> w(count);
        words_range(gen, seed, ctr, p0, count, w.data());
        float *o = (float *)dst;
        for (uint64_t j = 0; j < count; ++j) o[j] = oracle_u01(w[j]);
        return;
    }
    if (dist == OR_F64_UNIFORM) {
        /* sample p is made from words 2p and 2p+1 */
        std::vector<uint32_t> w(2 * count);
        words_range(gen, seed, ctr, 2 * p0, 2 * count, w.data());
        double *o = (double *)dst;
        for (uint64_t j = 0; j < count; ++j) o[j] = oracle_u01_f64(w[2 * j], w[2 * j + 1]);
        return;
    }
    if (dist == OR_F64_NORMAL) {
        /* sample p is member (p mod 2) of pair p/2, which is built from the
           four words 4*(p/2) .. 4*(p/2)+3 */
        const uint64_t m0 = p0 / 2, m1 = (p0 + count - 1) / 2;
        std::vector<uint32_t> w(4 * (m1 - m0 + 1));
        words_range(gen, seed, ctr, 4 * m0, w.size(), w.data());
        double *o = (double *)dst;
        for (uint64_t j = 0; j < count; ++j) {
            const uint64_t p = p0 + j, m = p / 2;
            const uint32_t *q = &w[4 * (m - m0)];
            double pair[2];
            oracle_normal_pair_f64(q[0], q[1], q[2], q[3], pair);
            o[j] = pair[p & 1];
        }
        return;
    }
    /* normal: sample p is member (p mod 2) of pair p/2, which is built from
       words 2*(p/2) and 2*(p/2)+1 */
    const uint64_t m0 = p0 / 2, m1 = (p0 + count - 1) / 2;
    std::vector<uint32_t> w(2 * (m1 - m0 + 1));
    words_range(gen, seed, ctr, 2 * m0, w.size(), w.data());
    float *o = (float *)dst;
    for (uint64_t j = 0; j < count; ++j) {
        uint64_t p = p0 + j, m = p / 2;
        float pair[2];
        oracle_normal_pair(w[2 * (m - m0)], w[2 * (m - m0) + 1], pair);
        o[j] = pair[p & 1];
    }
}

bool valid_gen(int g) { return g >= OR_PHILOX && g <= OR_PHILOX2X32; }
/* Philox2x32-10 has a 32-bit key: its seeds must be below 2^32 */
bool valid_seed(int g, uint64_t seed) { return g != OR_PHILOX2X32 || seed <= 0xFFFFFFFFull; }
bool valid_dist(int d) { return d >= OR_U32 && d <= OR_F64_NORMAL; }
/* bytes per sample, and stream positions (words) per sample */
bool is_f64(int dist) { return dist == OR_F64_UNIFORM || dist == OR_F64_NORMAL; }
uint64_t sample_bytes(int dist) { return is_f64(dist) ? 8 : 4; }
uint64_t sample_limit(int dist) { return is_f64(dist) ? (1ull << 31) : (1ull << 32); }

template <class F>
void parallel_ranges(uint64_t n, int nthreads, F body) {
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > n) nthreads = (int)(n ? n : 1);
    if (nthreads == 1) { body(0, n, 0); return; }
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t a = n * t / nthreads, b = n * (t + 1) / nthreads;
        th.emplace_back([=] { body(a, b, t); });
    }
    for (auto &x : th) x.join();
}

const uint64_t PERIOD = 1ull << 32;
const uint64_t PIECE = 1ull << 16;

} // namespace

extern "C" {

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    philox_round(x, k);
    for (int r = 1; r < 10; ++r) {
        k[0] += PHILOX_W0;
        k[1] += PHILOX_W1;
        philox_round(x, k);
    }
    std::memcpy(out, x, sizeof x);
}

void oracle_philox2x32_10(const uint32_t ctr[2], uint32_t key, uint32_t out[2]) {
    uint32_t a = ctr[0], b = ctr[1], k = key;
    for (int r = 0; r < 10; ++r) {
        if (r > 0) k += PHILOX_W0;
        const uint64_t prod = (uint64_t)PHILOX2_M * a;
        const uint32_t hi = (uint32_t)(prod >> 32), lo = (uint32_t)prod;
        a = hi ^ b ^ k;
        b = lo;
    }
    out[0] = a;
    out[1] = b;
}

/* R rounds of Threefry4x32: the key is injected before round 0 and after
   every fourth round (after round 4, 8, ...), so a round count that is not
   a multiple of four ends on a plain round. */
static void threefry4x32_r(const uint32_t ctr[4], const uint32_t key[4], int R, uint32_t out[4]) {
    uint32_t ks[5];
    ks[4] = SKEIN_PARITY32;
    for (int i = 0; i < 4; ++i) { ks[i] = key[i]; ks[4] ^= key[i]; }
    uint32_t x[4];
    for (int i = 0; i < 4; ++i) x[i] = ctr[i] + ks[i];
    for (int r = 0; r < R; ++r) {
        const unsigned ra = TF4_ROT[r % 8][0], rb = TF4_ROT[r % 8][1];
        if (r % 2 == 0) {
            x[0] += x[1]; x[1] = rotl32(x[1], ra) ^ x[0];
            x[2] += x[3]; x[3] = rotl32(x[3], rb) ^ x[2];
        } else {
            x[0] += x[3]; x[3] = rotl32(x[3], ra) ^ x[0];
            x[2] += x[1]; x[1] = rotl32(x[1], rb) ^ x[2];
        }
        if (r % 4 == 3) {
            const uint32_t s = (uint32_t)(r + 1) / 4;
            for (int i = 0; i < 4; ++i) x[i] += ks[(s + i) % 5];
            x[3] += s;
        }
    }
    std::memcpy(out, x, sizeof x);
}

void oracle_threefry4x32_20(const uint32_t ctr[4], const uint32_t key[4], uint32_t out[4]) {
    threefry4x32_r(ctr, key, 20, out);
}

/* The 13-round variants: the same rounds, rotations and key schedule,
   stopped after round 13 (after the injection that follows round 12).
   Pinned like their 20-round forms: Threefry2x64-13 against rocRAND's engine
   instantiated with 13 rounds; Threefry4x32-13 through the big-integer
   transcription run with 13 rounds under both mixing schedules. */
void oracle_threefry4x32_13(const uint32_t ctr[4], const uint32_t key[4], uint32_t out[4]) {
    threefry4x32_r(ctr, key, 13, out);
}

static void threefry2x64_r(const uint64_t ctr[2], const uint64_t key[2], int R, uint64_t out[2]) {
    const uint64_t ks[3] = {key[0], key[1], SKEIN_PARITY64 ^ key[0] ^ key[1]};
    uint64_t x0 = ctr[0] + ks[0], x1 = ctr[1] + ks[1];
    for (int r = 0; r < R; ++r) {
        x0 += x1;
        x1 = rotl64(x1, TF2_ROT[r % 8]) ^ x0;
        if (r % 4 == 3) {
            const uint64_t s = (uint64_t)(r + 1) / 4;
            x0 += ks[s % 3];
            x1 += ks[(s + 1) % 3] + s;
        }
    }
    out[0] = x0;
    out[1] = x1;
}

void oracle_threefry2x64_20(const uint64_t ctr[2], const uint64_t key[2], uint64_t out[2]) {
    threefry2x64_r(ctr, key, 20, out);
}

void oracle_threefry2x64_13(const uint64_t ctr[2], const uint64_t key[2], uint64_t out[2]) {
    threefry2x64_r(ctr, key, 13, out);
}

uint32_t oracle_squares32(uint64_t ctr, uint64_t key) {
    uint64_t y = ctr * key;
    uint64_t z = y + key;
    uint64_t x = y;
    x = x * x + y; x = (x >> 32) | (x << 32); /* round 1 */
    x = x * x + z; x = (x >> 32) | (x << 32); /* round 2 */
    x = x * x + y; x = (x >> 32) | (x << 32); /* round 3 */
    return (uint32_t)((x * x + z) >> 32);     /* round 4 */
}

uint64_t oracle_squares_key(uint64_t seed) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return z | 1ull;
}

void oracle_tyche_mix(uint32_t st[4]) {
    uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
    a += b; d = rotl32(d ^ a, 16);
    c += d; b = rotl32(b ^ c, 12);
    a += b; d = rotl32(d ^ a, 8);
    c += d; b = rotl32(b ^ c, 7);
    st[0] = a; st[1] = b; st[2] = c; st[3] = d;
}

void oracle_tyche_init(uint64_t seed, uint32_t c_xor, uint32_t d_xor, uint32_t st[4]) {
    st[0] = (uint32_t)(seed >> 32);
    st[1] = (uint32_t)seed;
    st[2] = TYCHE_C0 ^ c_xor;
    st[3] = TYCHE_D0 ^ d_xor;
    for (int i = 0; i < 20; ++i) oracle_tyche_mix(st);
}

uint32_t oracle_tyche_next(uint32_t st[4]) {
    oracle_tyche_mix(st);
    return st[1];
}

/* ---------------------------------------------------------------------------
 * Tyche-i (Neves, Araujo, PPAM 2011: the variant of Tyche built on the
 * inverse of MIX).  Reading: MIX-i undoes MIX's four steps in reverse order
 * (so b = rotr(b, 7) ^ c; c -= d; d = rotr(d, 8) ^ a; a -= b; then the same
 * with 12 and 16); seeding and output are Tyche's with MIX-i in place of MIX
 * (twenty rounds, then one round per output word, returning b), and the
 * stream layout is Tyche's.  A Tyche-i stream is therefore a Tyche state
 * orbit walked backwards.  Pinned in the test-suite: MIX-i inverts the pinned
 * MIX on random states, and twenty pinned MIX rounds take a Tyche-i seeded
 * state back to the raw seeding words.  Which word is output is parity
 * unpinned (no implementation in the container).
 * ------------------------------------------------------------------------- */
void oracle_tyche_mix_i(uint32_t st[4]) {
    uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
    b = rotl32(b, 25) ^ c; c -= d;
    d = rotl32(d, 24) ^ a; a -= b;
    b = rotl32(b, 20) ^ c; c -= d;
    d = rotl32(d, 16) ^ a; a -= b;
    st[0] = a; st[1] = b; st[2] = c; st[3] = d;
}

void oracle_tyche_i_init(uint64_t seed, uint32_t c_xor, uint32_t d_xor, uint32_t st[4]) {
    st[0] = (uint32_t)(seed >> 32);
    st[1] = (uint32_t)seed;
    st[2] = TYCHE_C0 ^ c_xor;
    st[3] = TYCHE_D0 ^ d_xor;
    for (int i = 0; i < 20; ++i) oracle_tyche_mix_i(st);
}

uint32_t oracle_tyche_i_next(uint32_t st[4]) {
    oracle_tyche_mix_i(st);
    return st[1];
}

/* ---------------------------------------------------------------------------
 * Squares64 (Widynski, arXiv:2004.06278, the five-round 64-bit output form):
 * rounds 1-4 as Squares32, keeping the full 64-bit value t of round 4; round
 * 5 squares the swapped t, adds y, and XORs its high half into t's low half.
 * Stream layout (reading, as for Squares32 with two words per call): word p is
 * the low (p even) or high (p odd) half of squares64((ctr << 32) | p/2, K),
 * K the Squares key of the seed.  Pinned in the test-suite: the high half of
 * every output is the (separately transcribed) Squares32 output of the same
 * counter and key.  Otherwise parity unpinned.
 * ------------------------------------------------------------------------- */
uint64_t oracle_squares64(uint64_t ctr, uint64_t key) {
    uint64_t y = ctr * key;
    uint64_t z = y + key;
    uint64_t x = y;
    x = x * x + y; x = (x >> 32) | (x << 32); /* round 1 */
    x = x * x + z; x = (x >> 32) | (x << 32); /* round 2 */
    x = x * x + y; x = (x >> 32) | (x << 32); /* round 3 */
    const uint64_t t = x * x + z;             /* round 4 */
    x = (t >> 32) | (t << 32);
    return t ^ ((x * x + y) >> 32);           /* round 5 */
}

uint32_t oracle_word(int gen, uint64_t seed, uint32_t ctr, uint64_t p) {
    uint32_t w = 0;
    if (gen == OR_TYCHE || gen == OR_TYCHE_I) {
        /* direct evaluation of the layout: fresh instance, step to the word */
        const bool inv = gen == OR_TYCHE_I;
        const uint64_t t = p / TYCHE_TILE, r = p % TYCHE_TILE;
        const uint64_t l = (r / 4) % TYCHE_LANES, k = r / 256, wi = r % 4;
        uint32_t st[4];
        if (inv) oracle_tyche_i_init(seed, (uint32_t)(t * TYCHE_LANES + l), ctr, st);
        else oracle_tyche_init(seed, (uint32_t)(t * TYCHE_LANES + l), ctr, st);
        for (uint64_t i = 0; i <= 4 * k + wi; ++i)
            w = inv ? oracle_tyche_i_next(st) : oracle_tyche_next(st);
        return w;
    }
    words_range(gen, seed, ctr, p, 1, &w);
    return w;
}

void oracle_sample(int gen, int dist, uint64_t seed, uint32_t ctr, uint64_t p, void *out) {
    if (gen == OR_TYCHE) {
        /* use the direct per-word form so a single sample costs O(256) MIX */
        if (dist == OR_U32) { uint32_t w = oracle_word(gen, seed, ctr, p); std::memcpy(out, &w, 4); return; }
        if (dist == OR_F32_UNIFORM) { float f = oracle_u01(oracle_word(gen, seed, ctr, p)); std::memcpy(out, &f, 4); return; }
        if (dist == OR_F64_UNIFORM) {
            const double d = oracle_u01_f64(oracle_word(gen, seed, ctr, 2 * p),
                                            oracle_word(gen, seed, ctr, 2 * p + 1));
            std::memcpy(out, &d, 8);
            return;
        }
        if (dist == OR_F64_NORMAL) {
            const uint64_t m = p / 2;
            double pair[2];
            oracle_normal_pair_f64(oracle_word(gen, seed, ctr, 4 * m), oracle_word(gen, seed, ctr, 4 * m + 1),
                                   oracle_word(gen, seed, ctr, 4 * m + 2), oracle_word(gen, seed, ctr, 4 * m + 3),
                                   pair);
            std::memcpy(out, &pair[p & 1], 8);
            return;
        }
        uint64_t m = p / 2;
        float pair[2];
        oracle_normal_pair(oracle_word(gen, seed, ctr, 2 * m), oracle_word(gen, seed, ctr, 2 * m + 1), pair);
        std::memcpy(out, &pair[p & 1], 4);
        return;
    }
    samples_range(gen, dist, seed, ctr, p, 1, out);
}

/* ---------------------------------------------------------------------------
 * float32 uniform in [0, 1) (reading; the paper does not define its float
 * conversion): the top 24 bits of the word times 2^-24.  Exact: a 24-bit
 * integer times a power of two.  Pinned: exhaustive over all 2^24 top parts
 * against float64 arithmetic in the test-suite.
 * ------------------------------------------------------------------------- */
float oracle_u01(uint32_t x) {
    return (float)(x >> 8) * 0x1p-24f;
}

/* ---------------------------------------------------------------------------
 * ln(k * 2^-24) for k in [1, 2^24], in float32 (reading, used for u1 of the
 * Box-Muller transform).  Definition, every step one IEEE float operation:
 *   k = m * 2^e exactly, m in [sqrt(1/2), sqrt(2))   (frexp, then one
 *     doubling when the fraction is below the float nearest sqrt(1/2))
 *   s = (m - 1) / (m + 1)
 *   ln m = 2 atanh(s) = 2s + s*z*(2/3 + z*(2/5 + z*(2/7 + z*2/9))),  z = s*s
 *   ln(k 2^-24) = (e - 24) * LN2_HI + ((e - 24) * LN2_LO + ln m)
 * The atanh series is truncated after s^9 (the next term is below 1e-9
 * relative); LN2_HI has 15 significant bits so (e-24)*LN2_HI is exact
 * (Cody-Waite split).  Pinned: exhaustive over all 2^24 arguments against
 * float64 log in the test-suite, within 2 ulp.
 * ------------------------------------------------------------------------- */
float oracle_ln_u1(uint32_t k) {
    const float LN2_HI = 0x1.62e4p-1f;     /* 0.693145751953125 */
    const float LN2_LO = 0x1.7f7d1cp-20f;  /* float(ln 2 - LN2_HI) */
    const float RSQRT2 = 0x1.6a09e6p-1f;   /* float nearest sqrt(1/2) */
    const float A3 = (float)(2.0 / 3.0), A5 = (float)(2.0 / 5.0);
    const float A7 = (float)(2.0 / 7.0), A9 = (float)(2.0 / 9.0);
    int e;
    float m = std::frexp((float)k, &e); /* (float)k exact; m in [0.5, 1) */
    if (m < RSQRT2) { m = m * 2.0f; e = e - 1; }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float q = std::fmaf(z, A9, A7);
    q = std::fmaf(z, q, A5);
    q = std::fmaf(z, q, A3);
    q = z * q;
    const float lnm = std::fmaf(s, q, s + s);
    const float t = (float)(e - 24);
    return std::fmaf(t, LN2_HI, std::fmaf(t, LN2_LO, lnm));
}

/* ---------------------------------------------------------------------------
 * cos and sin of 2*pi*k/2^24 for k in [0, 2^24), in float32 (reading, used
 * for u2 of the Box-Muller transform).  Definition:
 *   j = nearest quarter turn = ((k + 2^21) >> 22) mod 4, exact in integers
 *   d = k - 2^22 * round((k)/2^22) in [-2^21, 2^21), exact signed integer
 *   theta = d * (float(2 pi) * 2^-24)            one rounding
 *   sin theta ~ theta + theta^3*(-1/3! + z*(1/5! + z*(-1/7! + z/9!)))
 *   cos theta ~ 1 + z*(-1/2! + z*(1/4! + z*(-1/6! + z*(1/8! - z/10!))))
 *   with z = theta^2 and |theta| <= pi/4 (Taylor series; truncation below
 *   3e-9 relative), then rotate (cos, sin) by j quarter turns.
 * Pinned: exhaustive over all 2^24 arguments against float64 cos/sin in the
 * test-suite, within 2^-23 absolute.
 * ------------------------------------------------------------------------- */
void oracle_sincos2pi(uint32_t k, float *c, float *s) {
    const float STEP = 0x1.921fb6p+2f * 0x1p-24f; /* float(2 pi) * 2^-24, exact scaling */
    const float S3 = (float)(-1.0 / 6.0), S5 = (float)(1.0 / 120.0);
    const float S7 = (float)(-1.0 / 5040.0), S9 = (float)(1.0 / 362880.0);
    const float C2 = -0.5f, C4 = (float)(1.0 / 24.0), C6 = (float)(-1.0 / 720.0);
    const float C8 = (float)(1.0 / 40320.0), C10 = (float)(-1.0 / 3628800.0);
    const uint32_t q = (k + (1u << 21)) >> 22;  /* 0..4 */
    const uint32_t j = q & 3u;
    const int32_t d = (int32_t)k - (int32_t)(q << 22);
    const float th = (float)d * STEP;
    const float z = th * th;
    float ps = std::fmaf(z, S9, S7);
    ps = std::fmaf(z, ps, S5);
    ps = std::fmaf(z, ps, S3);
    const float sn = std::fmaf(th * z, ps, th);
    float pc = std::fmaf(z, C10, C8);
    pc = std::fmaf(z, pc, C6);
    pc = std::fmaf(z, pc, C4);
    pc = std::fmaf(z, pc, C2);
    const float cs = std::fmaf(z, pc, 1.0f);
    switch (j) {
    case 0: *c = cs; *s = sn; break;
    case 1: *c = -sn; *s = cs; break;
    case 2: *c = -cs; *s = -sn; break;
    default: *c = sn; *s = -cs; break;
    }
}

/* ---------------------------------------------------------------------------
 * Box-Muller pair (reading; the paper has no normal sampler, the method is
 * Box and Muller 1958).  From the even word x0 and odd word x1 of a pair:
 *   u1 = ((x0 >> 8) + 1) * 2^-24 in (0, 1]      (never 0, so ln is finite)
 *   u2 = (x1 >> 8) * 2^-24 in [0, 1)
 *   R  = sqrt(-2 ln u1)                          (correctly rounded sqrt)
 *   out = (R cos 2 pi u2, R sin 2 pi u2)
 * Pinned: against the same formula in float64 within a bound derived from the
 * ulp bounds above, and by moments / Kolmogorov-Smirnov on many samples.
 * ------------------------------------------------------------------------- */
void oracle_normal_pair(uint32_t x0, uint32_t x1, float out[2]) {
    const float l = oracle_ln_u1((x0 >> 8) + 1u);
    const float r = std::sqrt(-2.0f * l);
    float c, s;
    oracle_sincos2pi(x1 >> 8, &c, &s);
    out[0] = r * c;
    out[1] = r * s;
}

void oracle_u01_n(const uint32_t *x, uint64_t n, float *out) {
    for (uint64_t i = 0; i < n; ++i) out[i] = oracle_u01(x[i]);
}

void oracle_ln_u1_n(const uint32_t *k, uint64_t n, float *out) {
    for (uint64_t i = 0; i < n; ++i) out[i] = oracle_ln_u1(k[i]);
}

void oracle_sincos2pi_n(const uint32_t *k, uint64_t n, float *c, float *s) {
    for (uint64_t i = 0; i < n; ++i) oracle_sincos2pi(k[i], &c[i], &s[i]);
}

void oracle_normal_pair_n(const uint32_t *x0, const uint32_t *x1, uint64_t n, float *z0, float *z1) {
    for (uint64_t i = 0; i < n; ++i) {
        float p[2];
        oracle_normal_pair(x0[i], x1[i], p);
        z0[i] = p[0];
        z1[i] = p[1];
    }
}

int oracle_fill(int gen, int dist, uint64_t seed, uint32_t ctr, uint64_t offset, uint64_t n,
                void *out, int nthreads) {
    if (!valid_gen(gen) || !valid_dist(dist) || !valid_seed(gen, seed)) return -1;
    const uint64_t lim = sample_limit(dist), sb = sample_bytes(dist);
    if (offset > lim || n > lim - offset) return -2;
    char *o = (char *)out;
    parallel_ranges(n, nthreads, [&](uint64_t a, uint64_t b, int) {
        for (uint64_t j = a; j < b; j += PIECE) {
            uint64_t c = (b - j < PIECE) ? b - j : PIECE;
            samples_range(gen, dist, seed, ctr, offset + j, c, o + sb * j);
        }
    });
    return 0;
}

int oracle_fill_multi(int gen, int dist, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                      uint64_t offset, uint64_t per_stream, void *out, int nthreads) {
    if (!valid_gen(gen) || !valid_dist(dist) || !valid_seed(gen, seed)) return -1;
    const uint64_t lim = sample_limit(dist), sb = sample_bytes(dist);
    if (offset > lim || per_stream > lim - offset) return -2;
    if (n_streams && (uint64_t)ctr0 + n_streams - 1 > 0xFFFFFFFFull) return -2;
    char *o = (char *)out;
    parallel_ranges(n_streams, nthreads, [&](uint64_t a, uint64_t b, int) {
        for (uint64_t i = a; i < b; ++i)
            samples_range(gen, dist, seed, ctr0 + (uint32_t)i, offset, per_stream,
                          o + sb * i * per_stream);
    });
    return 0;
}

void oracle_samples_at(int gen, int dist, uint64_t seed, const uint32_t *ctrs,
                       const uint64_t *pos, uint64_t count, void *out, int nthreads) {
    char *o = (char *)out;
    parallel_ranges(count, nthreads, [&](uint64_t a, uint64_t b, int) {
        for (uint64_t k = a; k < b; ++k)
            oracle_sample(gen, dist, seed, ctrs[k], pos[k], o + sample_bytes(dist) * k);
    });
}

/* ---------------------------------------------------------------------------
 * Brownian walk (paper, section 4, Fig. 1 and section 5.1: particles diffuse
 * by a random walk; each particle's randoms come from its own stream).
 * Reading for the overdamped, float32, Gaussian form used here: particle i
 * owns the Philox stream (seed, ctr0 + i); step number g (global, g = step0 +
 * s) uses normal samples dim*g .. dim*g + dim-1 of that stream, and each
 * coordinate is updated as x_d = fmaf(sigma, normal, x_d) with
 * sigma = float(sqrt(2 D dt)) evaluated in float64.  msd[q] accumulates, in
 * float64, the sum over particles of |x|^2 after local step (q+1)*msd_every.
 * Pinned: D = 0 leaves positions unchanged; the mean squared displacement
 * from the origin follows 2 * dim * D * t (test-suite, statistical bound);
 * running 2k steps equals k steps then k more from step0 = k.
 * ------------------------------------------------------------------------- */
float oracle_walk_sigma(float dt, float D) {
    return (float)std::sqrt(2.0 * (double)D * (double)dt);
}

int oracle_brownian(uint64_t seed, uint32_t ctr0, const uint32_t *ids, uint32_t count,
                    uint32_t dim, uint64_t step0, uint32_t n_steps, float dt, float D,
                    float *pos, double *msd, uint32_t msd_every, int nthreads) {
    if (dim < 1 || dim > 3) return -1;
    if ((step0 + n_steps) * (uint64_t)dim > PERIOD) return -2;
    const float sigma = oracle_walk_sigma(dt, D);
    const uint32_t nsnap = (msd && msd_every) ? n_steps / msd_every : 0;
    if (nthreads < 1) nthreads = 1;
    std::vector<std::vector<double>> part(nthreads, std::vector<double>(nsnap, 0.0));
    parallel_ranges(count, nthreads, [&](uint64_t a, uint64_t b, int tid) {
        std::vector<float> g((size_t)n_steps * dim);
        for (uint64_t k = a; k < b; ++k) {
            const uint32_t pid = ids ? ids[k] : (uint32_t)k;
            samples_range(OR_PHILOX, OR_F32_NORMAL, seed, ctr0 + pid, step0 * dim,
                          (uint64_t)n_steps * dim, g.data());
            float x[3];
            for (uint32_t d = 0; d < dim; ++d) x[d] = pos[(uint64_t)d * count + k];
            for (uint32_t s = 0; s < n_steps; ++s) {
                for (uint32_t d = 0; d < dim; ++d)
                    x[d] = std::fmaf(sigma, g[(size_t)s * dim + d], x[d]);
                if (nsnap && (s + 1) % msd_every == 0) {
                    double r2 = 0.0;
                    for (uint32_t d = 0; d < dim; ++d) r2 += (double)x[d] * (double)x[d];
                    part[tid][(s + 1) / msd_every - 1] += r2;
                }
            }
            for (uint32_t d = 0; d < dim; ++d) pos[(uint64_t)d * count + k] = x[d];
        }
    });
    for (uint32_t q = 0; q < nsnap; ++q) {
        double acc = 0.0;
        for (int t = 0; t < nthreads; ++t) acc += part[t][q];
        msd[q] = acc;
    }
    return 0;
}


/* ---------------------------------------------------------------------------
 * float64 uniform in [0, 1) (reading; the paper draws two doubles per call in
 * its example, section 4 Fig. 1, without defining the conversion): the two
 * words at positions 2j and 2j+1 form the 64-bit integer (w1 << 32) | w0, and
 * its top 53 bits times 2^-53 are the double.  Exact: a 53-bit integer times a
 * power of two.  Pinned: against exact rational arithmetic in the test-suite.
 * ------------------------------------------------------------------------- */
double oracle_u01_f64(uint32_t w0, uint32_t w1) {
    const uint64_t x = ((uint64_t)w1 << 32) | w0;
    return (double)(x >> 11) * 0x1p-53;
}

/* ---------------------------------------------------------------------------
 * float64 Box-Muller normals (reading: the paper's generators feed standard
 * distributions, section 3, and it names no conversion).  Pair m (samples 2m
 * and 2m+1) is made from the four words 4m..4m+3: x = (w1 << 32) | w0 and
 * y = (w3 << 32) | w2 give u1 = ((x >> 11) + 1) 2^-53 in (0, 1] and
 * u2 = (y >> 11) 2^-53 in [0, 1); R = sqrt(-2 ln u1), z0 = R cos 2 pi u2,
 * z1 = R sin 2 pi u2 (Box and Muller, Ann. Math. Stat. 1958).  ln, cos and
 * sin are this library's own float64 functions below, so a result is a fixed
 * sequence of IEEE float64 operations, each rounded once (every Horner step
 * is one fused multiply-add; division and square root correctly rounded).
 *
 * ln u1, u1 = K 2^-53: K = m 2^e with m in [sqrt(1/2), sqrt(2)) split off in
 * integers (bit length of K; m is exact); ln m = 2 atanh(s), s = (m-1)/(m+1),
 * by its series through s^21 (|s| <= 0.1716, first omitted term below
 * 2^-60 relative); ln u1 = (e - 53) ln2_hi + ((e - 53) ln2_lo + ln m), ln2_hi
 * holding ln 2's leading 40 bits, so the first product is exact.
 * cos and sin of 2 pi k 2^-53: the nearest quarter turn j is taken off k in
 * integers, leaving a fraction f of at most 1/8 turn, exact; x = f * 2pi
 * (one rounding), |x| <= pi/4; Taylor series of sin through x^19 and of cos
 * through x^18 (first omitted terms below 2^-65), then the quarter-turn
 * rotation, which is exact.
 * Pinned in the test-suite: against 40-digit decimal arithmetic (its own
 * series for ln, pi, sin, cos) within stated ulp bounds on edge and random
 * arguments over every binade; exact values at quarter turns and at u1 = 1;
 * moments and Kolmogorov-Smirnov of many samples.
 * ------------------------------------------------------------------------- */
static const double LN2_HI = 0x1.62e42fefa2p-1;         /* ln 2 truncated to 40 bits */
static const double LN2_LO = 0x1.9ef35793c7673p-41;     /* ln 2 - LN2_HI, rounded */
static const double SQRT2 = 0x1.6a09e667f3bcdp+0;       /* sqrt 2, rounded */
static const double TWO_PI = 0x1.921fb54442d18p+2;      /* 2 pi, rounded */

double oracle_ln_u1_f64(uint64_t K) {
    int e = 63 - __builtin_clzll(K);                     /* 2^e <= K < 2^(e+1) */
    double m = std::ldexp((double)K, -e);                /* [1, 2), exact */
    if (m >= SQRT2) {
        m = m * 0.5;
        e = e + 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double P = 1.0 / 21.0;                               /* sum of z^k / (2k+1), k >= 1, over z */
    P = std::fma(P, z, 1.0 / 19.0);
    P = std::fma(P, z, 1.0 / 17.0);
    P = std::fma(P, z, 1.0 / 15.0);
    P = std::fma(P, z, 1.0 / 13.0);
    P = std::fma(P, z, 1.0 / 11.0);
    P = std::fma(P, z, 1.0 / 9.0);
    P = std::fma(P, z, 1.0 / 7.0);
    P = std::fma(P, z, 1.0 / 5.0);
    P = std::fma(P, z, 1.0 / 3.0);
    const double t = 2.0 * s;
    const double ln_m = std::fma(t, z * P, t);           /* 2s (1 + z P) */
    const double E = (double)(e - 53);
    return std::fma(E, LN2_HI, std::fma(E, LN2_LO, ln_m));
}

void oracle_sincos_turn_f64(uint64_t k, double *c, double *s) {
    const uint64_t j = (k + (1ull << 50)) >> 51;         /* nearest quarter turn, 0..4 */
    const int64_t r = (int64_t)k - (int64_t)(j << 51);   /* [-2^50, 2^50] */
    const double f = (double)r * 0x1p-53;                /* turns, exact */
    const double x = f * TWO_PI;
    const double z = x * x;
    double S = -1.0 / 121645100408832000.0;              /* -1/19! */
    S = std::fma(S, z, 1.0 / 355687428096000.0);         /*  1/17! */
    S = std::fma(S, z, -1.0 / 1307674368000.0);          /* -1/15! */
    S = std::fma(S, z, 1.0 / 6227020800.0);              /*  1/13! */
    S = std::fma(S, z, -1.0 / 39916800.0);               /* -1/11! */
    S = std::fma(S, z, 1.0 / 362880.0);                  /*  1/9!  */
    S = std::fma(S, z, -1.0 / 5040.0);                   /* -1/7!  */
    S = std::fma(S, z, 1.0 / 120.0);                     /*  1/5!  */
    S = std::fma(S, z, -1.0 / 6.0);                      /* -1/3!  */
    const double sn = std::fma(x * z, S, x);
    double Cp = 1.0 / 6402373705728000.0;                /*  1/18! */
    Cp = std::fma(Cp, z, -1.0 / 20922789888000.0);       /* -1/16! */
    Cp = std::fma(Cp, z, 1.0 / 87178291200.0);           /*  1/14! */
    Cp = std::fma(Cp, z, -1.0 / 479001600.0);            /* -1/12! */
    Cp = std::fma(Cp, z, 1.0 / 3628800.0);               /*  1/10! */
    Cp = std::fma(Cp, z, -1.0 / 40320.0);                /* -1/8!  */
    Cp = std::fma(Cp, z, 1.0 / 720.0);                   /*  1/6!  */
    Cp = std::fma(Cp, z, -1.0 / 24.0);                   /* -1/4!  */
    Cp = std::fma(Cp, z, 1.0 / 2.0);                     /*  1/2!, sign below */
    const double cs = std::fma(-z, Cp, 1.0);
    switch (j & 3) {
    case 0: *c = cs; *s = sn; break;
    case 1: *c = -sn; *s = cs; break;
    case 2: *c = -cs; *s = -sn; break;
    default: *c = sn; *s = -cs; break;
    }
}

void oracle_normal_pair_f64(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, double out[2]) {
    const uint64_t x = ((uint64_t)w1 << 32) | w0;
    const uint64_t y = ((uint64_t)w3 << 32) | w2;
    const double ln = oracle_ln_u1_f64((x >> 11) + 1);
    const double R = std::sqrt(std::fma(-2.0, ln, 0.0)); /* -2 ln exactly; u1 = 1 gives +0 */
    double c, s;
    oracle_sincos_turn_f64(y >> 11, &c, &s);
    out[0] = R * c;
    out[1] = R * s;
}

void oracle_ln_u1_f64_n(const uint64_t *K, uint64_t n, double *out) {
    for (uint64_t i = 0; i < n; ++i) out[i] = oracle_ln_u1_f64(K[i]);
}

void oracle_sincos_turn_f64_n(const uint64_t *k, uint64_t n, double *c, double *s) {
    for (uint64_t i = 0; i < n; ++i) oracle_sincos_turn_f64(k[i], &c[i], &s[i]);
}

/* ---------------------------------------------------------------------------
 * The paper's Brownian dynamics example (section 4, Fig. 1; the benchmark of
 * section 5.1 runs it in 2-D).  Particle id pid is the seed and the step's
 * counter is step0 + s (the example keys its generator by the particle id and
 * the loop iteration).  One draw of two doubles takes words 0..3 of Philox
 * stream (pid, counter): r.x from words 0, 1 and r.y from words 2, 3.
 * Model: a velocity component relaxes at rate c = gamma/mass and receives a
 * uniform kick on [-sqrt(dt), sqrt(dt)); the position integrates the
 * velocity.  Reading (the example elides the rest of a step and the float
 * evaluation order): with the step constants a = 1 - c*dt and w = 2*sqrt(dt),
 * each component takes v = a*v + (r - 0.5)*w, then x = x + v*dt.  Every
 * operation is one IEEE float64 operation (no contraction); r - 0.5 is exact.
 * Pinned in the test-suite: (a) with c = 2^10 and dt = 2^-10, a = 0 exactly,
 * so after every step v is the kick alone, (2u - 1) / 32 from the pinned
 * Philox words and conversion, and one step from rest moves x by exactly
 * v dt; (b) for general parameters the sample mean and variance of v and x
 * over many particles match the closed forms of the AR(1) velocity process
 * and its running sum.
 * ------------------------------------------------------------------------- */
int oracle_bd2(uint64_t pid0, const uint32_t *ids, uint32_t count, uint32_t step0,
               uint32_t n_steps, double dt, double c, double *x, double *y, double *vx,
               double *vy, int nthreads) {
    if (n_steps && (uint64_t)step0 + n_steps - 1 > 0xFFFFFFFFull) return -2;
    const double decay = 1.0 - c * dt;
    const double width = 2.0 * std::sqrt(dt);
    parallel_ranges(count, nthreads, [&](uint64_t lo, uint64_t hi, int) {
        for (uint64_t k = lo; k < hi; ++k) {
            const uint64_t pid = pid0 + (ids ? ids[k] : k);
            const uint32_t key[2] = {(uint32_t)pid, (uint32_t)(pid >> 32)};
            double *pos[2] = {&x[k], &y[k]};
            double *vel[2] = {&vx[k], &vy[k]};
            for (uint32_t s = 0; s < n_steps; ++s) {
                const uint32_t ctr[4] = {0u, step0 + s, 0u, 0u};
                uint32_t w[4];
                oracle_philox4x32_10(ctr, key, w);
                const double r[2] = {oracle_u01_f64(w[0], w[1]), oracle_u01_f64(w[2], w[3])};
                for (int d = 0; d < 2; ++d) {
                    const double v = decay * *vel[d] + (r[d] - 0.5) * width;
                    *vel[d] = v;
                    *pos[d] = *pos[d] + v * dt;
                }
            }
        }
    });
    return 0;
}


/* ---------------------------------------------------------------------------
 * Parallel micro-streams for statistical testing (section 5.2, after the
 * parallel-stream procedure it cites): each of n_particles particles draws a
 * micro-stream of `draws` words per iteration from its own stream, keyed as in
 * the paper's example (seed = particle id, counter = iteration); an
 * iteration's micro-streams are concatenated in particle order, and the
 * iterations follow one another.  Built from oracle_word, whose stream layout
 * is pinned in the test-suite; the concatenation is checked against
 * per-stream fills there.
 * ------------------------------------------------------------------------- */
int oracle_particle_streams(int gen, uint64_t seed0, uint32_t n_particles, uint32_t draws,
                            uint32_t ctr0, uint32_t n_iters, uint32_t *out, int nthreads) {
    if (!valid_gen(gen) || draws < 1 || draws > 16) return -1;
    if (n_iters && (uint64_t)ctr0 + n_iters - 1 > 0xFFFFFFFFull) return -2;
    if (n_particles && seed0 + (n_particles - 1) < seed0) return -2;
    if (n_particles && !valid_seed(gen, seed0 + (n_particles - 1))) return -2;
    const uint64_t units = (uint64_t)n_iters * n_particles;
    parallel_ranges(units, nthreads, [&](uint64_t a, uint64_t b, int) {
        for (uint64_t u = a; u < b; ++u) {
            const uint64_t t = u / n_particles, p = u % n_particles;
            for (uint32_t k = 0; k < draws; ++k)
                out[u * draws + k] = oracle_word(gen, seed0 + p, ctr0 + (uint32_t)t, k);
        }
    });
    return 0;
}

/* ---------------------------------------------------------------------------
 * Integers in [lo, hi) (reading of section 3, whose generators are meant to
 * feed standard-library distributions; the paper defines no integer
 * conversion).  Sample p takes the 64-bit integer x made of the words at
 * positions 2p and 2p+1 (as the float64 uniform does) and scales it to the
 * range by a full-width multiplication: lo + floor(x * r / 2^64), r = hi - lo.
 * No remainder is taken: each of the r values has floor(2^64 / r) or
 * ceil(2^64 / r) preimages among the 2^64 inputs, so its probability is within
 * 2^-64 of 1/r (relative bias below r / 2^64 < 2^-32), where the remainder
 * x mod r of one 32-bit word would favour low values by up to 2:1.  No
 * rejection step either: it would consume a variable number of words and
 * break the fixed sample-to-position map of the stream.  Pinned in the
 * test-suite: power-of-two ranges against the top bits of the high word; the
 * preimage thresholds ceil(v 2^64 / r) for random r and v in exact integer
 * arithmetic; frequencies of a range where the remainder method would be
 * off by 2:1.
 * ------------------------------------------------------------------------- */
int32_t oracle_range_i32(uint32_t w0, uint32_t w1, int32_t lo, int32_t hi) {
    const uint64_t x = ((uint64_t)w1 << 32) | w0;
    const uint64_t r = (uint64_t)((int64_t)hi - (int64_t)lo);
    const unsigned __int128 prod = (unsigned __int128)x * r;
    const uint64_t v = (uint64_t)(prod >> 64);
    return (int32_t)((int64_t)lo + (int64_t)v);
}

int oracle_fill_range(int gen, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                      uint64_t offset, uint64_t per_stream, int32_t lo, int32_t hi,
                      int32_t *out, int nthreads) {
    if (!valid_gen(gen) || lo >= hi || !valid_seed(gen, seed)) return -1;
    const uint64_t lim = 1ull << 31;
    if (offset > lim || per_stream > lim - offset) return -2;
    if (n_streams && (uint64_t)ctr0 + n_streams - 1 > 0xFFFFFFFFull) return -2;
    const uint64_t total = (uint64_t)n_streams * per_stream;
    parallel_ranges(total, nthreads, [&](uint64_t a, uint64_t b, int) {
        std::vector<uint32_t> w;
        for (uint64_t j = a; j < b;) {
            const uint64_t i = j / per_stream, q = j % per_stream;
            uint64_t c = per_stream - q;
            if (c > b - j) c = b - j;
            if (c > PIECE) c = PIECE;
            w.resize(2 * c);
            words_range(gen, seed, ctr0 + (uint32_t)i, 2 * (offset + q), 2 * c, w.data());
            for (uint64_t k = 0; k < c; ++k) out[j + k] = oracle_range_i32(w[2 * k], w[2 * k + 1], lo, hi);
            j += c;
        }
    });
    return 0;
}

} // extern "C"
