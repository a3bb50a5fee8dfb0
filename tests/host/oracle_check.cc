// Runs every bulk entry point of the oracle on small inputs, with several
// threads, and writes each output as raw bytes to <dir>/<name>.bin.  Built
// with the address and undefined-behaviour sanitizers by the test-suite,
// which compares the files with the outputs of the ordinary oracle build.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../oracle/orng_oracle.h"

static std::string g_dir;

static void dump(const std::string &name, const void *p, size_t bytes) {
    FILE *f = std::fopen((g_dir + "/" + name + ".bin").c_str(), "wb");
    if (!f || std::fwrite(p, 1, bytes, f) != bytes) { std::printf("write failed\n"); std::exit(2); }
    std::fclose(f);
}

static void check(int rc, const char *what) {
    if (rc != 0) { std::printf("%s returned %d\n", what, rc); std::exit(3); }
}

int main(int argc, char **argv) {
    if (argc < 2) return 1;
    g_dir = argv[1];
    const int T = 3;  // threads: ranges split unevenly
    for (int g = 0; g <= 9; ++g) {
        const uint64_t seed = g == 9 ? 0x89ABCDEFull : 0x0123456789ABCDEFull;
        for (int d = 0; d <= 4; ++d) {
            const uint64_t n = 5001, off = 16380;
            std::vector<uint64_t> buf(n);  // 8 bytes per sample covers every distribution
            check(oracle_fill(g, d, seed, 7, off, n, buf.data(), T), "fill");
            dump("fill_" + std::to_string(g) + "_" + std::to_string(d), buf.data(),
                 n * (d >= 3 ? 8 : 4));
            std::vector<uint64_t> m(3 * 77);
            check(oracle_fill_multi(g, d, seed, 0xFFFFFFF0u, 3, 5, 77, m.data(), T), "fill_multi");
            dump("multi_" + std::to_string(g) + "_" + std::to_string(d), m.data(),
                 3 * 77 * (d >= 3 ? 8 : 4));
        }
        std::vector<int32_t> r(2 * 1001);
        check(oracle_fill_range(g, seed, 3, 2, 1, 1001, -1000, 999, r.data(), T), "fill_range");
        dump("range_" + std::to_string(g), r.data(), r.size() * 4);
        std::vector<uint32_t> ps(5 * 300 * 3);
        check(oracle_particle_streams(g, 100, 300, 3, 9, 5, ps.data(), T), "particle_streams");
        dump("particles_" + std::to_string(g), ps.data(), ps.size() * 4);
    }
    {
        std::vector<float> pos(3 * 500, 0.0f);
        std::vector<double> msd(4);
        check(oracle_brownian(0xABCDEF, 11, nullptr, 500, 3, 0, 40, 1e-3f, 1.0f, pos.data(),
                              msd.data(), 10, T), "brownian");
        dump("walk", pos.data(), pos.size() * 4);
    }
    {
        std::vector<double> st(4 * 700, 0.0);
        check(oracle_bd2(5, nullptr, 700, 1, 30, 1e-3, 1.0, st.data(), st.data() + 700,
                         st.data() + 1400, st.data() + 2100, T), "bd2");
        dump("bd2", st.data(), st.size() * 8);
    }
    {
        std::vector<uint32_t> x0(4096), x1(4096);
        for (uint32_t i = 0; i < 4096; ++i) { x0[i] = i * 2654435761u; x1[i] = i * 40503u + 7u; }
        std::vector<float> z0(4096), z1(4096);
        oracle_normal_pair_n(x0.data(), x1.data(), 4096, z0.data(), z1.data());
        dump("normal_pairs_z0", z0.data(), z0.size() * 4);
        dump("normal_pairs_z1", z1.data(), z1.size() * 4);
    }
    std::printf("OK\n");
    return 0;
}
