// Seeds that share a Squares key.  The key of seed s is K(s) = z(s) | 1, where
// z is one SplitMix64 output step (add the golden-gamma increment, then two
// xor-shift-multiply steps and a final xor-shift), a bijection of 64-bit
// words.  So K(s) = K(s') for s != s' exactly when z(s') = z(s) ^ 1: every key
// belongs to two seeds, and the other seed of s is z^-1(z(s) ^ 1).
//
// This program walks every seed below 2^32 (the paper's Squares takes 32-bit
// seeds), forms its partner with the inverse step, and counts the seeds whose
// partner is below 2^32 too.  It checks the inverse and the oracle's key on a
// sample of seeds as it goes.  Output: "pairs <count> checked <n>", exit 0.
#include <cstdint>
#include <cstdio>
#include <thread>
#include <vector>

extern "C" uint64_t oracle_squares_key(uint64_t seed);

static const uint64_t GAMMA = 0x9E3779B97F4A7C15ull;
static const uint64_t M1 = 0xBF58476D1CE4E5B9ull, M2 = 0x94D049BB133111EBull;

static uint64_t z_of(uint64_t s) {
    uint64_t z = s + GAMMA;
    z = (z ^ (z >> 30)) * M1;
    z = (z ^ (z >> 27)) * M2;
    return z ^ (z >> 31);
}

// inverse of a -> a * m (mod 2^64) for odd m: Newton's iteration for m^-1
static uint64_t inverse_odd(uint64_t m) {
    uint64_t x = m;  // correct to 3 bits
    for (int i = 0; i < 6; ++i) x *= 2 - m * x;
    return x;
}

// inverse of x -> x ^ (x >> k)
static uint64_t unshift(uint64_t y, int k) {
    uint64_t x = y;
    for (int i = 0; i < 64 / k + 1; ++i) x = y ^ (x >> k);
    return x;
}

static uint64_t z_inverse(uint64_t z, uint64_t i1, uint64_t i2) {
    z = unshift(z, 31);
    z = unshift(z * i2, 27);
    z = unshift(z * i1, 30);
    return z - GAMMA;
}

int main() {
    const uint64_t i1 = inverse_odd(M1), i2 = inverse_odd(M2);
    if (M1 * i1 != 1 || M2 * i2 != 1) { std::puts("bad inverse"); return 1; }
    const unsigned T = std::thread::hardware_concurrency() ? std::thread::hardware_concurrency() : 8;
    std::vector<uint64_t> pairs(T, 0), bad(T, 0), checked(T, 0);
    std::vector<std::thread> th;
    const uint64_t N = 1ull << 32;
    for (unsigned t = 0; t < T; ++t) {
        th.emplace_back([&, t] {
            const uint64_t a = N * t / T, b = N * (t + 1) / T;
            for (uint64_t s = a; s < b; ++s) {
                const uint64_t z = z_of(s);
                const uint64_t p = z_inverse(z ^ 1ull, i1, i2);
                if (p < N) ++pairs[t];
                if ((s & 0xFFFFF) == 0x5A5A5) {  // sampled checks
                    ++checked[t];
                    if (z_inverse(z, i1, i2) != s || z_of(p) != (z ^ 1ull) || p == s ||
                        oracle_squares_key(s) != (z | 1ull) ||
                        oracle_squares_key(p) != oracle_squares_key(s))
                        ++bad[t];
                }
            }
        });
    }
    for (auto &x : th) x.join();
    uint64_t np = 0, nb = 0, nc = 0;
    for (unsigned t = 0; t < T; ++t) { np += pairs[t]; nb += bad[t]; nc += checked[t]; }
    if (nb) { std::printf("check failures %llu\n", (unsigned long long)nb); return 1; }
    std::printf("pairs %llu checked %llu\n", (unsigned long long)np, (unsigned long long)nc);
    return 0;
}
