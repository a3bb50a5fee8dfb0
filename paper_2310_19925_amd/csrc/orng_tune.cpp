// Launch-parameter table and the autotuner that fills it.
//
// Launch parameters change speed only: every output is a function of its
// stream and position alone, so any workgroup size, span length, grid size,
// queue claim size or store kind gives identical results.  The table starts
// from defaults measured on MI355X and can be refined per (gen, dist) by
// orng_autotune, which times variants on the current device and keeps the
// fastest.  Entries persist in a small text file (one line per pair).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "../../include/orng.h"
#include "orng_internal.hpp"

namespace orng {

int fill_batched(const orng_req_t *reqs, size_t nreq, hipStream_t stream);

static std::mutex g_tune_mu;
static Tuned g_tuned[NGEN][NDIST];
static bool g_tuned_init = false;

// Measured on MI355X by orng_autotune (one entry per gen x dist, in
// enum order: u32, f32 uniform, f32 normal, f64 uniform, f64 normal): wg unroll max_wgs nontemporal | batched wg unroll chunk wgs/CU
// (wgs/CU 0 = static one-workgroup-per-tile schedule).
static const uint32_t kDefaultTable[NGEN * NDIST][8] = {
        {64, 4, 0, 2, 512, 8, 1, 0},
        {64, 4, 0, 1, 512, 8, 1, 0},
        {512, 2, 8192, 1, 128, 16, 1, 0},
        {64, 4, 0, 2, 512, 8, 1, 0},
        {512, 8, 8192, 1, 256, 16, 1, 4},
        {256, 8, 8192, 1, 128, 16, 1, 0},
        {512, 8, 8192, 1, 128, 16, 1, 0},
        {512, 8, 8192, 2, 128, 16, 1, 0},
        {512, 8, 8192, 1, 256, 16, 1, 0},
        {256, 8, 0, 1, 128, 16, 1, 8},
        {512, 4, 8192, 1, 128, 16, 1, 0},
        {512, 8, 8192, 1, 128, 16, 1, 0},
        {512, 4, 8192, 2, 128, 16, 1, 0},
        {512, 4, 8192, 1, 256, 16, 1, 0},
        {512, 4, 8192, 2, 128, 16, 1, 0},
        {64, 4, 0, 1, 256, 8, 1, 0},
        {64, 8, 0, 1, 256, 8, 1, 0},
        {256, 2, 8192, 1, 128, 16, 1, 0},
        {256, 8, 0, 1, 256, 16, 1, 0},
        {256, 2, 8192, 1, 128, 16, 1, 0},
        {64, 64, 0, 2, 512, 1, 1, 0},
        {64, 64, 0, 2, 512, 1, 1, 0},
        {256, 64, 0, 1, 128, 1, 1, 0},
        {512, 64, 0, 2, 128, 1, 1, 8},
        {256, 64, 0, 1, 128, 1, 1, 0},
        // 13-round Threefry
        {64, 8, 0, 1, 256, 8, 1, 0},
        {512, 4, 8192, 1, 128, 16, 1, 0},
        {512, 2, 8192, 1, 128, 16, 1, 0},
        {512, 8, 8192, 1, 256, 16, 1, 0},
        {512, 4, 8192, 1, 256, 16, 1, 0},
        {256, 8, 0, 2, 256, 8, 1, 0},
        {512, 8, 8192, 1, 128, 16, 1, 0},
        {256, 8, 0, 1, 256, 16, 1, 0},
        {256, 8, 8192, 1, 256, 16, 1, 0},
        {256, 8, 0, 1, 256, 16, 1, 4},
        // Tyche-i, Squares64 (started from Tyche's and Squares32's shapes)
        {64, 64, 0, 2, 512, 1, 1, 0},
        {64, 64, 0, 2, 512, 1, 1, 0},
        {256, 64, 0, 1, 128, 1, 1, 0},
        {64, 64, 0, 2, 128, 1, 1, 8},
        {256, 64, 0, 1, 128, 1, 1, 0},
        {64, 4, 0, 1, 256, 8, 1, 0},
        {64, 4, 0, 2, 512, 8, 1, 0},
        {256, 2, 8192, 1, 128, 16, 1, 0},
        {64, 4, 0, 1, 512, 8, 1, 0},
        {512, 4, 8192, 1, 256, 16, 1, 0},
        // Philox2x32-10
        {64, 4, 0, 2, 512, 8, 1, 0},
        {64, 4, 0, 2, 512, 8, 1, 0},
        {512, 2, 8192, 1, 128, 16, 1, 0},
        {128, 4, 0, 2, 512, 8, 1, 0},
        {512, 8, 8192, 1, 256, 16, 1, 4},
};

// Integer-range fills (orng_fill_range), one row per generator: workgroup
// size, groups of 256 samples per span (Tyche: one tile), grid cap (0: one
// wave per span), store kind (unused: ordinary stores).
// Measured on MI355X (a sweep of 64-512 threads, 1-16 groups per span, grid
// uncapped or 8 workgroups per CU, 2^30 samples; the fastest shape per
// generator).
static const uint32_t kRangeTable[NGEN][4] = {
        {128, 16, 0, 2},  {512, 1, 2048, 2}, {256, 16, 2048, 2}, {512, 16, 0, 2}, {64, 1, 0, 2},
        {256, 1, 2048, 2}, {256, 16, 0, 2},   {64, 1, 0, 2},      {256, 16, 0, 2}, {512, 16, 0, 2},
};
static Tuned g_range[NGEN];

static Tuned default_range(int gen) {
    Tuned t{};
    t.wg_size = kRangeTable[gen][0];
    t.unroll = kRangeTable[gen][1];
    t.max_wgs = kRangeTable[gen][2];
    t.nontemporal = kRangeTable[gen][3];
    return t;
}

static Tuned default_tuned(int gen, int dist) {
    const uint32_t *v = kDefaultTable[gen * NDIST + dist];
    Tuned t;
    t.wg_size = v[0];
    t.unroll = v[1];
    t.max_wgs = v[2];
    t.nontemporal = v[3];
    t.b_wg_size = v[4];
    t.b_unroll = v[5];
    t.b_chunk = v[6];
    t.b_wgs_per_cu = v[7];
    return t;
}

static void init_locked() {
    if (g_tuned_init) return;
    for (int g = 0; g < NGEN; ++g) {
        for (int d = 0; d < NDIST; ++d) g_tuned[g][d] = default_tuned(g, d);
        g_range[g] = default_range(g);
    }
    g_tuned_init = true;
}

static int load_locked(const char *path);

static void init_from_env_once() {
    static std::once_flag once;
    std::call_once(once, [] {
        const char *p = getenv("ORNG_TUNE_CACHE");
        std::lock_guard<std::mutex> lk(g_tune_mu);
        init_locked();
        if (p && *p) load_locked(p);
    });
}

Tuned tuned_fill(int gen, int dist) {
    init_from_env_once();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tuned[gen][dist];
}

Tuned tuned_range(int gen) {
    init_from_env_once();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_range[gen];
}

void set_tuned_range(int gen, const Tuned &t) {
    init_from_env_once();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_range[gen] = t;
}

void set_tuned(int gen, int dist, const Tuned &t) {
    init_from_env_once();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[gen][dist] = t;
}

static bool sane(const Tuned &t, int gen) {
    auto wg_ok = [](uint32_t w) { return w >= 64 && w <= 512 && w % 64 == 0; };
    return wg_ok(t.wg_size) && wg_ok(t.b_wg_size) && t.unroll >= 1 && t.unroll <= 64 &&
           t.b_unroll >= 1 && t.b_unroll <= 64 && t.b_chunk >= 1 && t.b_chunk <= 64 &&
           t.b_wgs_per_cu <= 64 && t.nontemporal >= 1 &&
           t.nontemporal <= 2 && (!tyche_like(gen) || t.unroll == 64);
}

static bool sane_range(const Tuned &t) {
    return t.wg_size >= 64 && t.wg_size <= 512 && t.wg_size % 64 == 0 && t.unroll >= 1 &&
           t.unroll <= 64 && t.nontemporal >= 1 && t.nontemporal <= 2;
}

static int load_locked(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) return ORNG_ENOENT;
    char line[256];
    int loaded = 0;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        int g, d;
        Tuned t;
        if (sscanf(line, "%d %d %u %u %u %u %u %u %u %u", &g, &d, &t.wg_size, &t.unroll,
                   &t.max_wgs, &t.nontemporal, &t.b_wg_size, &t.b_unroll, &t.b_chunk,
                   &t.b_wgs_per_cu) == 10 &&
            g >= 0 && g < NGEN && d >= 0 && d < NDIST && sane(t, g)) {
            g_tuned[g][d] = t;
            ++loaded;
        } else if (sscanf(line, "%d %d %u %u %u %u", &g, &d, &t.wg_size, &t.unroll, &t.max_wgs,
                          &t.nontemporal) == 6 &&
                   g >= 0 && g < NGEN && d == ORNG_TUNE_RANGE && sane_range(t)) {
            g_range[g] = t;  // an integer-range row: its batched fields are unused
            ++loaded;
        }
    }
    fclose(f);
    return loaded > 0 ? ORNG_OK : ORNG_EINVAL;
}

int load_tune_cache(const char *path) {
    init_from_env_once();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return load_locked(path);
}

int save_tune_cache(const char *path) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    init_locked();
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return ORNG_EINVAL;
    fprintf(f, "# orng launch table: gen dist wg unroll max_wgs nontemporal "
               "batched_wg batched_unroll batched_chunk batched_wgs_per_cu "
               "(dist %d: the integer-range fill, fill fields only)\n", ORNG_TUNE_RANGE);
    for (int g = 0; g < NGEN; ++g) {
        for (int d = 0; d < NDIST; ++d) {
            const Tuned &t = g_tuned[g][d];
            fprintf(f, "%d %d %u %u %u %u %u %u %u %u\n", g, d, t.wg_size, t.unroll, t.max_wgs,
                    t.nontemporal, t.b_wg_size, t.b_unroll, t.b_chunk, t.b_wgs_per_cu);
        }
        const Tuned &t = g_range[g];
        fprintf(f, "%d %d %u %u %u %u 0 0 0 0\n", g, ORNG_TUNE_RANGE, t.wg_size, t.unroll,
                t.max_wgs, t.nontemporal);
    }
    fclose(f);
    return rename(tmp.c_str(), path) == 0 ? ORNG_OK : ORNG_EINVAL;
}

// Median of `reps` timed runs of fn on stream s, in milliseconds.
template <class F>
static float time_ms(hipStream_t s, int reps, F fn, hipError_t *err) {
    hipEvent_t a, b;
    *err = hipEventCreate(&a);
    if (*err != hipSuccess) return 0;
    *err = hipEventCreate(&b);
    if (*err != hipSuccess) { hipEventDestroy(a); return 0; }
    std::vector<float> v;
    fn();  // warm-up
    for (int i = 0; i < reps && *err == hipSuccess; ++i) {
        hipEventRecord(a, s);
        fn();
        hipEventRecord(b, s);
        *err = hipEventSynchronize(b);
        float ms = 0;
        hipEventElapsedTime(&ms, a, b);
        v.push_back(ms);
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (v.empty()) return 1e30f;
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
}

// Second pass of a tuning search: the `keep` fastest candidates of a first
// pass (cands sorted by time) are timed again in interleaved rounds, one run
// of each per round, so that clock and power drift during the search hits all
// of them alike; returns the candidate with the lowest median.
template <class Apply, class Run>
static Tuned refine(std::vector<std::pair<float, Tuned>> cands, size_t keep, int rounds,
                    hipStream_t s, Apply apply, Run run, hipError_t *err) {
    std::stable_sort(cands.begin(), cands.end(),
                     [](const std::pair<float, Tuned> &a, const std::pair<float, Tuned> &b) {
                         return a.first < b.first;
                     });
    if (cands.size() > keep) cands.resize(keep);
    std::vector<std::vector<float>> t(cands.size());
    for (int r = 0; r < rounds && *err == hipSuccess; ++r)
        for (size_t i = 0; i < cands.size() && *err == hipSuccess; ++i) {
            apply(cands[i].second);
            t[i].push_back(time_ms(s, 1, run, err));
        }
    size_t best = 0;
    float best_ms = 1e30f;
    for (size_t i = 0; i < cands.size(); ++i) {
        if (t[i].empty()) continue;
        std::sort(t[i].begin(), t[i].end());
        const float m = t[i][t[i].size() / 2];
        if (m < best_ms) { best_ms = m; best = i; }
    }
    return cands.empty() ? Tuned{} : cands[best].second;
}

// Integer-range fill of gen: workgroup size x span length x grid cap, the
// entry in use competing too; 2^30 samples into buf.
static hipError_t tune_range(int gen, void *buf, uint64_t n, hipStream_t s) {
    hipError_t e = hipSuccess;
    const int cus = device_cu_count();
    Tuned best = tuned_range(gen);
    std::vector<std::pair<float, Tuned>> cands;
    cands.push_back({0.0f, best});
    auto run = [&] {
        orng_fill_range(gen, 0x5EED, 0, 1, 0, n, -1000000000, 1000000007,
                        static_cast<int32_t *>(buf), s);
    };
    for (uint32_t wg : {64u, 128u, 256u, 512u})
        for (uint32_t un : {1u, 2u, 4u, 8u, 16u}) {
            if (tyche_like(gen) && un != 1) continue;
            for (uint32_t cap : {0u, (uint32_t)cus * 8}) {
                if (e != hipSuccess) break;
                Tuned t = best;
                t.wg_size = wg;
                t.unroll = un;
                t.max_wgs = cap;
                set_tuned_range(gen, t);
                cands.push_back({time_ms(s, 3, run, &e), t});
            }
        }
    if (e == hipSuccess)
        best = refine(cands, 6, 9, s, [&](const Tuned &t) { set_tuned_range(gen, t); }, run, &e);
    set_tuned_range(gen, best);
    return e;
}

}  // namespace orng

using namespace orng;

extern "C" {

int orng_tune_load(const char *cache_path) {
    if (!cache_path) return ORNG_EINVAL;
    return load_tune_cache(cache_path);
}

int orng_autotune(int gen, int dist, const char *cache_path) {
    if (gen < 0 || gen >= NGEN || dist < 0 || (dist >= NDIST && dist != ORNG_TUNE_RANGE))
        return ORNG_EINVAL;
    if (dist == ORNG_TUNE_RANGE) {
        const uint64_t n = 1ull << 30;
        void *buf = nullptr;
        hipStream_t s = nullptr;
        hipError_t e = hipMalloc(&buf, n * 4);
        if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) { hipFree(buf); set_hip_error(e); return ORNG_EHIP; }
        const LaunchCfg saved_cfg = launch_cfg();
        set_launch_cfg(LaunchCfg{0, 0, 0, 0});
        e = tune_range(gen, buf, n, s);
        set_launch_cfg(saved_cfg);
        const hipError_t e2 = hipStreamSynchronize(s);
        hipStreamDestroy(s);
        hipFree(buf);
        if (e == hipSuccess) e = e2;
        if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
        if (cache_path) {
            const Tuned best = tuned_range(gen);
            load_tune_cache(cache_path);
            set_tuned_range(gen, best);
            return save_tune_cache(cache_path);
        }
        return ORNG_OK;
    }
    const uint64_t n = 1ull << 30;  // 4 GiB of samples: the size of a bulk fill
    void *buf = nullptr;
    hipStream_t s = nullptr;
    hipError_t e = hipMalloc(&buf, n * 4);
    if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) { hipFree(buf); set_hip_error(e); return ORNG_EHIP; }
    const LaunchCfg saved_cfg = launch_cfg();
    set_launch_cfg(LaunchCfg{0, 0, 0, 0});
    Tuned best = tuned_fill(gen, dist);
    const int cus = device_cu_count();

    // plain fill: workgroup size x span length x grid cap x store kind; the
    // entry in use competes too
    std::vector<std::pair<float, Tuned>> cands;
    cands.push_back({0.0f, best});  // time 0: always reaches the second pass
    const uint32_t wgs[] = {64, 128, 256, 512};
    const uint32_t unrolls[] = {1, 2, 4, 8};
    const uint32_t caps[] = {0, (uint32_t)cus * 8, (uint32_t)cus * 32};
    auto run_fill = [&] { launch_fill(gen, dist, 0x5EED, 0, 1, 0, n, buf, s); };
    for (uint32_t wg : wgs)
        for (uint32_t un : unrolls) {
            if (tyche_like(gen) && un != 1) continue;
            for (uint32_t cap : caps)
                for (uint32_t nt = 1; nt <= 2 && e == hipSuccess; ++nt) {
                    Tuned t = best;
                    t.wg_size = wg;
                    t.unroll = tyche_like(gen) ? 64 : un;
                    t.max_wgs = cap;
                    t.nontemporal = nt;
                    set_tuned(gen, dist, t);
                    cands.push_back({time_ms(s, 3, run_fill, &e), t});
                }
        }
    if (e == hipSuccess)
        best = refine(cands, 6, 9, s, [&](const Tuned &t) { set_tuned(gen, dist, t); }, run_fill,
                      &e);
    set_tuned(gen, dist, best);

    // batched: uneven requests packed back to back (lengths in samples; a
    // float64 sample takes two words of the buffer)
    std::mt19937_64 rng(12345);
    std::vector<orng_req_t> reqs;
    const uint64_t kw = words_per_sample(dist), lim = sample_limit(dist);
    uint64_t used = 0;  // words
    while (reqs.size() < 8192) {
        const double u = std::uniform_real_distribution<double>(0.0, 20.0)(rng);
        uint64_t len = (uint64_t)std::pow(2.0, u);
        if (len < 1) len = 1;
        if (used + len * kw > n) break;
        orng_req_t r{};
        r.seed = rng();
        r.ctr = (uint32_t)rng();
        r.offset = rng() % (lim - len + 1);
        r.n = len;
        r.out = static_cast<char *>(buf) + used * 4;
        r.gen = (uint32_t)gen;
        r.dist = (uint32_t)dist;
        r.flags = 0;
        reqs.push_back(r);
        used += len * kw;
    }
    std::vector<std::pair<float, Tuned>> bc;
    bc.push_back({0.0f, best});  // the entry in use
    auto run_batched = [&] { fill_batched(reqs.data(), reqs.size(), s); };
    for (uint32_t wg : {128u, 256u, 512u})
        for (uint32_t un : {1u, 2u, 4u, 8u, 16u})
            for (uint32_t ch : {1u, 4u})
                for (uint32_t wpc : {0u, 2u, 4u, 8u}) {  // 0: static schedule
                    if (e != hipSuccess) break;
                    if (tyche_like(gen) && un != 1) continue;
                    if (wpc == 0 && ch != 1) continue;  // chunk is a queue parameter
                    Tuned t = best;
                    t.b_wg_size = wg;
                    t.b_unroll = un;
                    t.b_chunk = ch;
                    t.b_wgs_per_cu = wpc;
                    set_tuned(gen, dist, t);
                    int st = ORNG_OK;
                    const float ms = time_ms(s, 3, [&] {
                        st = fill_batched(reqs.data(), reqs.size(), s);
                    }, &e);
                    if (st == ORNG_OK) bc.push_back({ms, t});
                }
    Tuned bt = best;
    if (e == hipSuccess)
        bt = refine(bc, 6, 9, s, [&](const Tuned &t) { set_tuned(gen, dist, t); }, run_batched,
                    &e);
    best.b_wg_size = bt.b_wg_size;
    best.b_unroll = bt.b_unroll;
    best.b_chunk = bt.b_chunk;
    best.b_wgs_per_cu = bt.b_wgs_per_cu;
    set_tuned(gen, dist, best);
    set_launch_cfg(saved_cfg);
    hipError_t e2 = hipStreamSynchronize(s);
    hipStreamDestroy(s);
    hipFree(buf);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
    if (cache_path) {
        load_tune_cache(cache_path);  // keep other pairs already in the file...
        set_tuned(gen, dist, best);   // ...but this pair's fresh result wins
        return save_tune_cache(cache_path);
    }
    return ORNG_OK;
}

}  // extern "C"
