// Device-side generator cores, float conversions and the Box-Muller normal
// for gfx950.  Everything here is a __device__ function kept in VGPRs; key
// material that is the same for every lane of a launch is precomputed once per
// launch on the host (KeySched) and arrives in SGPRs through the kernarg
// segment, so the per-block work is only the data-dependent part.
//
// Definitions (the paper names the generators in section 3.1 but defines none
// of them; the round functions follow the primary sources it cites):
//   Philox4x32-10, Threefry4x32-20, Threefry2x64-20 : Salmon et al., SC'11.
//   Squares32 (four rounds)                         : Widynski 2020.
//   Tyche                                           : Neves and Araujo 2012.
// The stream-to-counter mappings, the float32 uniform, the float32 logarithm
// and quarter-turn sine/cosine and the Box-Muller pairing are readings of the
// paper's stream model (section 3.1: 64-bit seed, 32-bit counter, period 2^32
// words) stated next to each function.  Every float expression below is one
// IEEE operation (the library is built with -ffp-contract=off); fused
// multiply-adds are written as fmaf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "orng_host.hpp"

namespace orng {

// Linear workgroup id of a grid launched as grid_2d(blocks) (x fastest).
__device__ __forceinline__ uint32_t flat_block() {
    return blockIdx.y * gridDim.x + blockIdx.x;
}

// Per-launch key material, uniform across the grid.
struct KeySched {
    uint32_t k[10][2];   // Philox round keys (key bumped by the Weyl pair)
    uint32_t ks4[5];     // Threefry4x32 key schedule: key words + parity word
    uint64_t ks2[3];     // Threefry2x64 key schedule
    uint64_t sqkey;      // Squares key derived from the seed
    uint32_t seed_lo, seed_hi;
};

// a ^ b ^ c in one gfx950 v_bitop3_b32 (truth table 0x96: the output bit is
// the parity of the three input bits).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// ---------------------------------------------------------------------------
// Philox4x32-10.  Counter (c0, c1, 0, 0): c0 is the block number inside the
// stream, c1 the stream counter.  The two zero words make the first round's
// second product vanish; the compiler folds that.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox_block(uint32_t c0, uint32_t c1, const KeySched &ks,
                                             uint32_t o[4]) {
    uint32_t x0 = c0, x1 = c1, x2 = 0u, x3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)x0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)x2 * 0xCD9E8D57u;
        const uint32_t n0 = xor3((uint32_t)(b >> 32), x1, ks.k[r][0]);
        const uint32_t n2 = xor3((uint32_t)(a >> 32), x3, ks.k[r][1]);
        x1 = (uint32_t)b;
        x3 = (uint32_t)a;
        x0 = n0;
        x2 = n2;
    }
    o[0] = x0; o[1] = x1; o[2] = x2; o[3] = x3;
}

// ---------------------------------------------------------------------------
// Philox2x32-10 (the two-word Philox).  Its key is one 32-bit word, the low
// word of a seed below 2^32, so its round keys are the first column of the
// Philox4x32 schedule.  Positions 4 blk .. 4 blk + 3 are the two-word blocks
// (2 blk, c1) and (2 blk + 1, c1), computed side by side: one 32x32->64
// product and one xor3 per round and block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox2_block(uint32_t blk, uint32_t c1, const KeySched &ks,
                                              uint32_t o[4]) {
    uint32_t a0 = 2u * blk, a1 = 2u * blk + 1u, b0 = c1, b1 = c1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)a0 * 0xD256D193u;
        const uint64_t p1 = (uint64_t)a1 * 0xD256D193u;
        const uint32_t n0 = xor3((uint32_t)(p0 >> 32), b0, ks.k[r][0]);
        const uint32_t n1 = xor3((uint32_t)(p1 >> 32), b1, ks.k[r][0]);
        b0 = (uint32_t)p0;
        b1 = (uint32_t)p1;
        a0 = n0;
        a1 = n1;
    }
    o[0] = a0; o[1] = b0; o[2] = a1; o[3] = b1;
}

// Block 0 of Philox stream (seed, c1) with the key in VGPRs, for kernels in
// which every lane has its own seed (one stream per particle): round r uses
// (lo + r W0, hi + r W1), bumped as the rounds go.
__device__ __forceinline__ void philox_block0_lanekey(uint32_t c1, uint32_t klo, uint32_t khi,
                                                      uint32_t o[4]) {
    uint32_t x0 = 0u, x1 = c1, x2 = 0u, x3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)x0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)x2 * 0xCD9E8D57u;
        const uint32_t n0 = xor3((uint32_t)(b >> 32), x1, klo);
        const uint32_t n2 = xor3((uint32_t)(a >> 32), x3, khi);
        x1 = (uint32_t)b;
        x3 = (uint32_t)a;
        x0 = n0;
        x2 = n2;
        klo += 0x9E3779B9u;
        khi += 0xBB67AE85u;
    }
    o[0] = x0; o[1] = x1; o[2] = x2; o[3] = x3;
}

// ---------------------------------------------------------------------------
// Threefry4x32-20.  Counter (c0, c1, 0, 0), key (lo seed, hi seed, 0, 0).
// Mixing pairs follow the Threefish permutation: (0,1)(2,3) on even rounds,
// (0,3)(2,1) on odd rounds; key injection after every fourth round.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) {
    return (x << r) | (x >> (32 - r));
}

template <int R>
__device__ __forceinline__ void tf4_round(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3) {
    constexpr int RA[8] = {10, 11, 13, 23, 6, 17, 25, 18};
    constexpr int RB[8] = {26, 21, 27, 5, 20, 11, 10, 20};
    if constexpr ((R & 1) == 0) {
        x0 += x1; x1 = rotl32(x1, RA[R & 7]) ^ x0;
        x2 += x3; x3 = rotl32(x3, RB[R & 7]) ^ x2;
    } else {
        x0 += x3; x3 = rotl32(x3, RA[R & 7]) ^ x0;
        x2 += x1; x1 = rotl32(x1, RB[R & 7]) ^ x2;
    }
}

template <int S>
__device__ __forceinline__ void tf4_inject(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                           const KeySched &ks) {
    x0 += ks.ks4[(S + 0) % 5];
    x1 += ks.ks4[(S + 1) % 5];
    x2 += ks.ks4[(S + 2) % 5];
    x3 += ks.ks4[(S + 3) % 5] + (uint32_t)S;
}

template <int S>
__device__ __forceinline__ void tf4_quad(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                         const KeySched &ks) {
    tf4_round<4 * S - 4>(x0, x1, x2, x3);
    tf4_round<4 * S - 3>(x0, x1, x2, x3);
    tf4_round<4 * S - 2>(x0, x1, x2, x3);
    tf4_round<4 * S - 1>(x0, x1, x2, x3);
    tf4_inject<S>(x0, x1, x2, x3, ks);
}

// NR = 20 (five quads) or 13 (three quads, then round 12 with no injection
// after it).
template <int NR>
__device__ __forceinline__ void tf4_block(uint32_t c0, uint32_t c1, const KeySched &ks,
                                          uint32_t o[4]) {
    static_assert(NR == 20 || NR == 13, "Threefry4x32 round count");
    uint32_t x0 = c0 + ks.ks4[0], x1 = c1 + ks.ks4[1], x2 = ks.ks4[2], x3 = ks.ks4[3];
    tf4_quad<1>(x0, x1, x2, x3, ks);
    tf4_quad<2>(x0, x1, x2, x3, ks);
    tf4_quad<3>(x0, x1, x2, x3, ks);
    if constexpr (NR == 20) {
        tf4_quad<4>(x0, x1, x2, x3, ks);
        tf4_quad<5>(x0, x1, x2, x3, ks);
    } else {
        tf4_round<12>(x0, x1, x2, x3);
    }
    o[0] = x0; o[1] = x1; o[2] = x2; o[3] = x3;
}

// ---------------------------------------------------------------------------
// Threefry2x64-20.  Counter (block, stream counter) as 64-bit words, key
// (seed, 0); the block's four 32-bit words are lo X0, hi X0, lo X1, hi X1.
// ---------------------------------------------------------------------------
// 64-bit rotate as two funnel shifts of the 32-bit halves (v_alignbit_b32):
// for 0 < r < 32, hi' = (hi:lo) >> (32 - r) and lo' = (lo:hi) >> (32 - r);
// r > 32 rotates the swapped halves by r - 32; r == 32 is the swap itself.
template <int R>
__device__ __forceinline__ uint64_t rotl64(uint64_t x) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    if constexpr (R == 32) {
        return ((uint64_t)lo << 32) | hi;
    } else if constexpr (R < 32) {
        const uint32_t nh = __builtin_amdgcn_alignbit(hi, lo, 32 - R);
        const uint32_t nl = __builtin_amdgcn_alignbit(lo, hi, 32 - R);
        return ((uint64_t)nh << 32) | nl;
    } else {
        const uint32_t nh = __builtin_amdgcn_alignbit(lo, hi, 64 - R);
        const uint32_t nl = __builtin_amdgcn_alignbit(hi, lo, 64 - R);
        return ((uint64_t)nh << 32) | nl;
    }
}

template <int R>
__device__ __forceinline__ void tf2_round(uint64_t &x0, uint64_t &x1) {
    x0 += x1;
    x1 = rotl64<R>(x1) ^ x0;
}

template <int S>
__device__ __forceinline__ void tf2_quad(uint64_t &x0, uint64_t &x1, const KeySched &ks) {
    constexpr int ROT[8] = {16, 42, 12, 31, 16, 32, 24, 21};
    tf2_round<ROT[(4 * S - 4) & 7]>(x0, x1);
    tf2_round<ROT[(4 * S - 3) & 7]>(x0, x1);
    tf2_round<ROT[(4 * S - 2) & 7]>(x0, x1);
    tf2_round<ROT[(4 * S - 1) & 7]>(x0, x1);
    x0 += ks.ks2[S % 3];
    x1 += ks.ks2[(S + 1) % 3] + (uint64_t)S;
}

// NR = 20 (five quads) or 13 (three quads, then round 12 with no injection
// after it; rotation constants repeat with period 8).
template <int NR>
__device__ __forceinline__ void tf2_block(uint32_t c0, uint32_t c1, const KeySched &ks,
                                          uint32_t o[4]) {
    static_assert(NR == 20 || NR == 13, "Threefry2x64 round count");
    uint64_t x0 = (uint64_t)c0 + ks.ks2[0];
    uint64_t x1 = (uint64_t)c1 + ks.ks2[1];
    tf2_quad<1>(x0, x1, ks);
    tf2_quad<2>(x0, x1, ks);
    tf2_quad<3>(x0, x1, ks);
    if constexpr (NR == 20) {
        tf2_quad<4>(x0, x1, ks);
        tf2_quad<5>(x0, x1, ks);
    } else {
        tf2_round<16>(x0, x1);  // round 12: rotation constant index 12 mod 8 = 4
    }
    o[0] = (uint32_t)x0; o[1] = (uint32_t)(x0 >> 32);
    o[2] = (uint32_t)x1; o[3] = (uint32_t)(x1 >> 32);
}

// ---------------------------------------------------------------------------
// Squares32: counter ((stream counter << 32) | position), key from the seed.
// x*x + a mod 2^64 = (xl*xl + a) + 2*xl*xh*2^32: one v_mad_u64_u32 for the
// first sum, and the cross term only touches the high word (its low word is
// zero), so it is a 32-bit multiply and a shift-add.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sq_add(uint32_t xl, uint32_t xh, uint64_t a,
                                       uint32_t &rl, uint32_t &rh) {
    const uint64_t t = (uint64_t)xl * xl + a;
    rl = (uint32_t)t;
    rh = (uint32_t)(t >> 32) + 2u * (xl * xh);
}

// Four rounds on y = ((ctr << 32) | pos) * key and z = y + key (mod 2^64);
// each round squares, adds, and swaps the 32-bit halves (the swap is a
// renaming of the result words).
__device__ __forceinline__ uint32_t squares_rounds(uint64_t y, uint64_t z) {
    uint32_t l, h;
    sq_add((uint32_t)y, (uint32_t)(y >> 32), y, l, h);  // round 1: x = y
    sq_add(h, l, z, l, h);                              // round 2
    sq_add(h, l, y, l, h);                              // round 3
    sq_add(h, l, z, l, h);                              // round 4: output the high word
    return h;
}

// Words of positions 4*blk .. 4*blk+3.  y is affine in the position, so
// y(p+1) = y(p) + key = z(p): after one full product per block, every further
// y and z is one 64-bit add.
__device__ __forceinline__ void squares_block(uint32_t blk, uint32_t ctr, uint64_t key,
                                              uint32_t w[4]) {
    const uint32_t p = blk << 2;
    const uint32_t kl = (uint32_t)key, kh = (uint32_t)(key >> 32);
    uint64_t y = (uint64_t)p * kl + ((uint64_t)(p * kh + ctr * kl) << 32);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t z = y + key;
        w[i] = squares_rounds(y, z);
        y = z;
    }
}

// Squares64: rounds 1-4 as Squares32 but keeping round 4's full value t;
// round 5 squares t with its halves swapped and adds y, and its high half is
// XORed into t's low half.  Counter ((stream counter << 32) | call), two words
// per call (low half first), so block blk is calls 2 blk and 2 blk + 1.
__device__ __forceinline__ void squares64_rounds(uint64_t y, uint64_t z, uint32_t &lo,
                                                 uint32_t &hi) {
    uint32_t l, h, l5, h5;
    sq_add((uint32_t)y, (uint32_t)(y >> 32), y, l, h);  // round 1: x = y
    sq_add(h, l, z, l, h);                              // round 2
    sq_add(h, l, y, l, h);                              // round 3
    sq_add(h, l, z, l, h);                              // round 4: t = (h, l)
    sq_add(h, l, y, l5, h5);                            // round 5
    lo = l ^ h5;
    hi = h;
}

__device__ __forceinline__ void squares64_block(uint32_t blk, uint32_t ctr, uint64_t key,
                                                uint32_t w[4]) {
    const uint32_t q = blk << 1;
    const uint32_t kl = (uint32_t)key, kh = (uint32_t)(key >> 32);
    const uint64_t y = (uint64_t)q * kl + ((uint64_t)(q * kh + ctr * kl) << 32);
    const uint64_t z = y + key;
    squares64_rounds(y, z, w[0], w[1]);
    squares64_rounds(z, z + key, w[2], w[3]);
}

// ---------------------------------------------------------------------------
// Tyche.  MIX is the ChaCha quarter round; seeding puts (hi seed, lo seed,
// floor(2^32/phi) ^ substream, floor(2^32/pi) ^ counter) in (a, b, c, d) and
// mixes twenty times; each output mixes once and returns b.  Stream layout:
// tiles of 16384 words; in tile t, lane l (0..63) owns blocks k*64 + l,
// k = 0..63, and produces them from substream t*64 + l in order.
// Tyche-i (INV): the same with MIX-i, the inverse of MIX (its four steps
// undone in reverse order), so its stream walks Tyche's state orbit backwards.
// ---------------------------------------------------------------------------
template <bool INV>
struct TycheT {
    uint32_t a, b, c, d;
    __device__ __forceinline__ void mix() {
        if constexpr (!INV) {
            a += b; d = rotl32(d ^ a, 16);
            c += d; b = rotl32(b ^ c, 12);
            a += b; d = rotl32(d ^ a, 8);
            c += d; b = rotl32(b ^ c, 7);
        } else {
            b = rotl32(b, 25) ^ c; c -= d;
            d = rotl32(d, 24) ^ a; a -= b;
            b = rotl32(b, 20) ^ c; c -= d;
            d = rotl32(d, 16) ^ a; a -= b;
        }
    }
    __device__ __forceinline__ void seed(const KeySched &ks, uint32_t substream, uint32_t ctr) {
        a = ks.seed_hi;
        b = ks.seed_lo;
        c = 2654435769u ^ substream;
        d = 1367130551u ^ ctr;
#pragma unroll 4
        for (int i = 0; i < 20; ++i) mix();
    }
    __device__ __forceinline__ uint32_t next() {
        mix();
        return b;
    }
    __device__ __forceinline__ void next4(uint32_t o[4]) {
        o[0] = next(); o[1] = next(); o[2] = next(); o[3] = next();
    }
};
using Tyche = TycheT<false>;

// Key material for a seed.  Host and device: the batched and served kernels
// build it per request with scalar instructions.
__host__ __device__ inline KeySched make_keysched(uint64_t seed) {
    KeySched k{};
    k.seed_lo = (uint32_t)seed;
    k.seed_hi = (uint32_t)(seed >> 32);
    uint32_t k0 = k.seed_lo, k1 = k.seed_hi;
    for (int r = 0; r < 10; ++r) {
        k.k[r][0] = k0;
        k.k[r][1] = k1;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    k.ks4[0] = k.seed_lo;
    k.ks4[1] = k.seed_hi;
    k.ks4[2] = 0u;
    k.ks4[3] = 0u;
    k.ks4[4] = 0x1BD11BDAu ^ k.seed_lo ^ k.seed_hi;
    k.ks2[0] = seed;
    k.ks2[1] = 0ull;
    k.ks2[2] = 0x1BD11BDAA9FC1A22ull ^ seed;
    // Squares key: one SplitMix64 output step of the seed, low bit forced on
    uint64_t z = seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    k.sqkey = (z ^ (z >> 31)) | 1ull;
    return k;
}


// ---------------------------------------------------------------------------
// float32 conversions.
//   uniform  : (x >> 8) * 2^-24, exact, in [0, 1 - 2^-24].
//   ln_u1(k) : ln(k * 2^-24) for k in [1, 2^24]: k = m 2^e with m in
//              [sqrt(1/2), sqrt(2)) split off with integer arithmetic on the float's bits, ln m =
//              2 atanh(s), s = (m-1)/(m+1), series to s^9, then the exponent
//              part with a two-piece ln 2 (high piece exact times e-24).
//   sincos   : cos, sin of 2 pi k/2^24 for k in [0, 2^24): nearest quarter
//              turn j and signed remainder d in integers, theta = d * (float(2
//              pi) 2^-24), Taylor polynomials to theta^9 / theta^10, rotate by j.
//   normal   : (R cos 2 pi u2, R sin 2 pi u2), R = sqrt(-2 ln u1) with
//              u1 = ((x0>>8)+1) 2^-24 from the even word and u2 = (x1>>8) 2^-24
//              from the odd word of each pair (Box and Muller 1958).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float to_uniform(uint32_t x) {
    return __uint2float_rn(x >> 8) * 0x1p-24f;
}

// n / d rounded to nearest for the operands ln_u1 produces (d = m + 1 in
// [1.70, 2.42], n = m - 1 in [-0.30, 0.42]): hardware reciprocal estimate,
// then one residual correction of the quotient (Markstein).  On this operand
// set the result is the IEEE quotient for every one of the 2^24 arguments of
// ln_u1 (checked exhaustively on the GPU against the CPU oracle).
__device__ __forceinline__ float div_ln(float n, float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    const float q = n * r;
    return fmaf(fmaf(-d, q, n), r, q);
}

// sqrt(y) rounded to nearest for y in [0, 34] (the range of -2 ln u1):
// s = y * rsq(y), then one Markstein correction s + (y - s^2) * rsq(y) / 2;
// y = 0 (u1 = 1) is passed through.  Equal to the IEEE square root on every
// one of the 2^24 arguments (checked exhaustively on the GPU).
__device__ __forceinline__ float sqrt_r(float y) {
    const float r = __builtin_amdgcn_rsqf(y);
    const float s = y * r;
    const float o = fmaf(fmaf(-s, s, y), 0.5f * r, s);
    return y == 0.0f ? y : o;
}

__device__ __forceinline__ float ln_u1(uint32_t k) {
    const float f = __uint2float_rn(k);  // exact, k <= 2^24
    const uint32_t bits = __float_as_uint(f);
    // f = m 2^e with m in [sqrt(1/2), sqrt(2)): subtracting the bits of the
    // float nearest sqrt(1/2) (0x3F3504F3) borrows from the exponent exactly
    // when the fraction is below that of sqrt(2), so the shifted difference is
    // e, and removing e from the exponent field leaves m
    const int e = (int)(bits - 0x3F3504F3u) >> 23;
    const float m = __uint_as_float(bits - ((uint32_t)e << 23));
    const float s = div_ln(m - 1.0f, m + 1.0f);
    const float z = s * s;
    float q = fmaf(z, (float)(2.0 / 9.0), (float)(2.0 / 7.0));
    q = fmaf(z, q, (float)(2.0 / 5.0));
    q = fmaf(z, q, (float)(2.0 / 3.0));
    q = z * q;
    const float lnm = fmaf(s, q, s + s);
    const float t = (float)(e - 24);
    return fmaf(t, 0x1.62e4p-1f, fmaf(t, 0x1.7f7d1cp-20f, lnm));
}

__device__ __forceinline__ void sincos_turn(uint32_t k, float &c, float &s) {
    const uint32_t q = (k + 0x200000u) >> 22;
    const int d = (int)k - (int)(q << 22);
    const float th = (float)d * (0x1.921fb6p+2f * 0x1p-24f);
    const float z = th * th;
    float ps = fmaf(z, (float)(1.0 / 362880.0), (float)(-1.0 / 5040.0));
    ps = fmaf(z, ps, (float)(1.0 / 120.0));
    ps = fmaf(z, ps, (float)(-1.0 / 6.0));
    const float sn = fmaf(th * z, ps, th);
    float pc = fmaf(z, (float)(-1.0 / 3628800.0), (float)(1.0 / 40320.0));
    pc = fmaf(z, pc, (float)(-1.0 / 720.0));
    pc = fmaf(z, pc, (float)(1.0 / 24.0));
    pc = fmaf(z, pc, -0.5f);
    const float cs = fmaf(z, pc, 1.0f);
    // rotate (cs, sn) by j = q mod 4 quarter turns: swap for odd j, then flip
    // the sign bit of cos for j = 1, 2 and of sin for j = 2, 3
    const uint32_t v = k + 0x200000u;  // bits 22, 23 of v are the two bits of j
    const bool odd = (v & 0x400000u) != 0;
    const float cr = odd ? sn : cs;
    const float sr = odd ? cs : sn;
    c = __uint_as_float(__float_as_uint(cr) ^ (((v + 0x400000u) & 0x800000u) << 8));
    s = __uint_as_float(__float_as_uint(sr) ^ ((v & 0x800000u) << 8));
}

__device__ __forceinline__ void normal_pair(uint32_t x0, uint32_t x1, float &z0, float &z1) {
    const float l = ln_u1((x0 >> 8) + 1u);
    const float r = sqrt_r(-2.0f * l);
    float c, s;
    sincos_turn(x1 >> 8, c, s);
    z0 = r * c;
    z1 = r * s;
}

// float64 in [0, 1) from the words at positions 2j (w0) and 2j+1 (w1): the top
// 53 bits of (w1 << 32 | w0) times 2^-53.  w1 * 2^21 + (w0 >> 11) is an integer
// below 2^53, so the fma is exact, and so is the power-of-two scaling.
__device__ __forceinline__ double u01_f64(uint32_t w0, uint32_t w1) {
    return fma((double)w1, 0x1p21, (double)(w0 >> 11)) * 0x1p-53;
}

// ---------------------------------------------------------------------------
// float64 Box-Muller pair from the four words of a block: x = (w1 << 32) | w0,
// y = (w3 << 32) | w2, u1 = ((x >> 11) + 1) 2^-53 in (0, 1], u2 = (y >> 11)
// 2^-53; z0 = R cos 2 pi u2, z1 = R sin 2 pi u2, R = sqrt(-2 ln u1).  ln, cos
// and sin are float64 functions of this library: a fixed sequence of IEEE
// operations, each rounded once (Horner steps are fused multiply-adds), so the
// result does not depend on the math library.
//   ln u1, u1 = K 2^-53: K = m 2^e, m in [sqrt(1/2), sqrt(2)) (exact split);
//     ln m = 2 atanh(s), s = (m-1)/(m+1), series through s^21;
//     ln u1 = (e-53) ln2_hi + ((e-53) ln2_lo + ln m), ln2_hi = ln 2 cut to 40
//     bits, so its product is exact.
//   cos, sin of 2 pi k 2^-53: the nearest quarter turn j comes off k in
//     integers, leaving r = k - j 2^51 (|r| <= 2^50); x = r (2 pi 2^-53), one
//     rounding, |x| <= pi/4; Taylor series of sin through x^19 and of cos
//     through x^18; rotate by j quarter turns (swaps and sign flips, exact).
// ---------------------------------------------------------------------------
constexpr double F64_LN2_HI = 0x1.62e42fefa2p-1;
constexpr double F64_LN2_LO = 0x1.9ef35793c7673p-41;
constexpr double F64_SQRT2 = 0x1.6a09e667f3bcdp+0;
constexpr double F64_TWO_PI_2M53 = 0x1.921fb54442d18p-51;  // float64(2 pi) * 2^-53

// One float64 fused multiply-add as one VOP3 instruction (a*b + c, rounded
// once, as fma()), with the addend (a series coefficient) in a scalar register
// pair.  Written out because with fma() the compiler keeps every coefficient
// in vector registers and, per Horner step, copies it into the destination of
// the two-address form (v_fmac_f64): 80-90 VGPRs and a move per step.  With
// scalar addends the float64 normal fills need 47-59 VGPRs and run 5-11%
// faster on MI355X (the compiler rematerialises or spills the constants to
// vector lanes; results are the same bits).
__device__ __forceinline__ double fma3(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

__device__ __forceinline__ double ln_u1_f64(uint64_t K) {
    // K <= 2^53, so its float64 value is exact; frexp splits it exactly
    const double Kd = fma((double)(uint32_t)(K >> 32), 0x1p32, (double)(uint32_t)K);
    int e = __builtin_amdgcn_frexp_exp(Kd) - 1;                // 2^e <= K < 2^(e+1)
    double m = 2.0 * __builtin_amdgcn_frexp_mant(Kd);          // [1, 2)
    if (m >= F64_SQRT2) {
        m = m * 0.5;
        e = e + 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double P = 1.0 / 21.0;
    P = fma3(P, z, 1.0 / 19.0);
    P = fma3(P, z, 1.0 / 17.0);
    P = fma3(P, z, 1.0 / 15.0);
    P = fma3(P, z, 1.0 / 13.0);
    P = fma3(P, z, 1.0 / 11.0);
    P = fma3(P, z, 1.0 / 9.0);
    P = fma3(P, z, 1.0 / 7.0);
    P = fma3(P, z, 1.0 / 5.0);
    P = fma3(P, z, 1.0 / 3.0);
    const double t = 2.0 * s;
    const double ln_m = fma(t, z * P, t);
    const double E = (double)(e - 53);
    return fma(E, F64_LN2_HI, fma(E, F64_LN2_LO, ln_m));
}

__device__ __forceinline__ void sincos_turn_f64(uint64_t k, double &c, double &s) {
    const uint64_t j = (k + (1ull << 50)) >> 51;                // 0..4
    const int64_t r = (int64_t)k - (int64_t)(j << 51);           // [-2^50, 2^50]
    const double x = (double)r * F64_TWO_PI_2M53;
    const double z = x * x;
    double S = -1.0 / 121645100408832000.0;
    S = fma3(S, z, 1.0 / 355687428096000.0);
    S = fma3(S, z, -1.0 / 1307674368000.0);
    S = fma3(S, z, 1.0 / 6227020800.0);
    S = fma3(S, z, -1.0 / 39916800.0);
    S = fma3(S, z, 1.0 / 362880.0);
    S = fma3(S, z, -1.0 / 5040.0);
    S = fma3(S, z, 1.0 / 120.0);
    S = fma3(S, z, -1.0 / 6.0);
    const double sn = fma(x * z, S, x);
    double C = 1.0 / 6402373705728000.0;
    C = fma3(C, z, -1.0 / 20922789888000.0);
    C = fma3(C, z, 1.0 / 87178291200.0);
    C = fma3(C, z, -1.0 / 479001600.0);
    C = fma3(C, z, 1.0 / 3628800.0);
    C = fma3(C, z, -1.0 / 40320.0);
    C = fma3(C, z, 1.0 / 720.0);
    C = fma3(C, z, -1.0 / 24.0);
    C = fma3(C, z, 1.0 / 2.0);
    const double cs = fma(-z, C, 1.0);
    const uint32_t q = (uint32_t)j & 3u;
    const double cr = (q & 1u) ? sn : cs;
    const double sr = (q & 1u) ? cs : sn;
    c = (q == 1u || q == 2u) ? -cr : cr;
    s = (q >= 2u) ? -sr : sr;
}

__device__ __forceinline__ void normal_pair_f64(uint32_t w0, uint32_t w1, uint32_t w2,
                                                uint32_t w3, double &z0, double &z1) {
    const uint64_t x = ((uint64_t)w1 << 32) | w0;
    const uint64_t y = ((uint64_t)w3 << 32) | w2;
    const double l = ln_u1_f64((x >> 11) + 1);
    const double R = sqrt(fma(-2.0, l, 0.0));  // -2 ln u1 exactly; u1 = 1 gives +0
    double c, s;
    sincos_turn_f64(y >> 11, c, s);
    z0 = R * c;
    z1 = R * s;
}

// Convert a block of four words to the output words of its samples (bit
// patterns): four float32/u32 samples, or two float64 samples (little-endian
// word order) for D_F64U and D_F64N.
template <int D>
__device__ __forceinline__ void convert4(uint32_t w[4]) {
    if constexpr (D == D_UNIFORM) {
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = __float_as_uint(to_uniform(w[i]));
    } else if constexpr (D == D_NORMAL) {
        float a, b, c, d;
        normal_pair(w[0], w[1], a, b);
        normal_pair(w[2], w[3], c, d);
        w[0] = __float_as_uint(a); w[1] = __float_as_uint(b);
        w[2] = __float_as_uint(c); w[3] = __float_as_uint(d);
    } else if constexpr (D == D_F64U) {
        // halves taken as 32-bit values (no 64-bit view of w, which kept the
        // array out of registers)
        const double a = u01_f64(w[0], w[1]), b = u01_f64(w[2], w[3]);
        w[0] = (uint32_t)__double2loint(a); w[1] = (uint32_t)__double2hiint(a);
        w[2] = (uint32_t)__double2loint(b); w[3] = (uint32_t)__double2hiint(b);
    } else if constexpr (D == D_F64N) {
        double a, b;
        normal_pair_f64(w[0], w[1], w[2], w[3], a, b);
        w[0] = (uint32_t)__double2loint(a); w[1] = (uint32_t)__double2hiint(a);
        w[2] = (uint32_t)__double2loint(b); w[3] = (uint32_t)__double2hiint(b);
    }
}

// Integer sample in [lo, hi) from the word pair (w0, w1) of its two stream
// positions: lo + floor(((w1 << 32) | w0) r / 2^64), r = hi - lo < 2^32.  With
// x = w1 2^32 + w0, floor(x r / 2^64) = floor((w1 r + floor(w0 r / 2^32)) / 2^32):
// the high half of w0 r, then w1 r plus a 64-bit addend whose low word is that
// half and whose high word is lo -- adding lo 2^32 to the sum adds lo to its
// high word (a carry out of bit 63 is dropped, as a 32-bit add of lo drops
// it).  lo is passed as its two's-complement bits.
__device__ __forceinline__ uint32_t range_sample(uint32_t w0, uint32_t w1, uint32_t r,
                                                 uint32_t lo) {
    const uint32_t t = __umulhi(w0, r);
    const uint64_t s = (uint64_t)w1 * r + (((uint64_t)lo << 32) | t);
    return (uint32_t)(s >> 32);
}

// Words of counter block `blk` (positions 4*blk .. 4*blk+3) of stream ctr.
template <int G>
__device__ __forceinline__ void counter_block(uint32_t blk, uint32_t ctr, const KeySched &ks,
                                              uint32_t w[4]) {
    if constexpr (G == G_PHILOX) {
        philox_block(blk, ctr, ks, w);
    } else if constexpr (G == G_TF4X32) {
        tf4_block<20>(blk, ctr, ks, w);
    } else if constexpr (G == G_TF2X64) {
        tf2_block<20>(blk, ctr, ks, w);
    } else if constexpr (G == G_TF4X32_13) {
        tf4_block<13>(blk, ctr, ks, w);
    } else if constexpr (G == G_TF2X64_13) {
        tf2_block<13>(blk, ctr, ks, w);
    } else if constexpr (G == G_SQUARES64) {
        squares64_block(blk, ctr, ks.sqkey, w);
    } else if constexpr (G == G_PHILOX2X32) {
        philox2_block(blk, ctr, ks, w);
    } else {  // G_SQUARES
        squares_block(blk, ctr, ks.sqkey, w);
    }
}

}  // namespace orng
