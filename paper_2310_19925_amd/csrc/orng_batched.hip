// Batched fills: many streams of uneven lengths in one persistent launch.
//
// Every request's output equals orng_fill of the same (gen, dist, seed, ctr,
// offset, n) exactly: a sample depends only on its own stream and position
// (paper section 3.1), never on the other requests of the batch.
//
// Host: requests are validated, each is cut into tiles of W consecutive spans
// (a span is the fill kernels' unit: 64*U blocks of four words, or one Tyche
// tile; W = waves per workgroup, taken with the rest of the launch shape from
// the (generator, distribution) pair holding most of the batch's words), and
// a prefix sum gives every request its first tile number.  The header, the request table
// and a tile -> request map (and, for a batch with integer-range requests, a
// table of their bounds) are written into pinned staging and uploaded with
// two copies (three) into a device buffer whose layout is fixed for its capacity.
// Device: a persistent grid pulls tiles from an atomic cursor in the header
// (`chunk` tiles per pull), looks up the request of each tile in the map and
// generates it with the same span code as the plain fill.  A static schedule
// (one wave per tile, no queue) is the alternative the tuner may pick: short
// waves keep more stores in flight than long-lived ones on this part.  The launch is
// captured once into a hipGraph per (buffer, launch shape) and replayed.
// A small ring of such contexts per device lets consecutive calls overlap:
// a context is reused only after the event of its previous launch.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/orng.h"
#include "orng_internal.hpp"
#include "orng_span.hpp"

namespace orng {

struct DevReq {             // 64 bytes, read by the kernel with scalar loads
    char *out;
    uint64_t p0, n, seed;
    uint64_t first_span;    // absolute span number of the request's first tile
    uint64_t tile_start;    // number of the request's first tile in the batch
    uint32_t ctr;
    uint32_t unroll;        // blocks per lane per tile (counter generators)
    uint32_t flags;         // gen | dist << 4 | delta << 8
    uint32_t tiles;         // number of the request's tiles
};
static_assert(sizeof(DevReq) == 64, "DevReq layout");

struct BatchHdr {           // 64 bytes
    uint64_t total_tiles;
    uint64_t cursor;        // next unclaimed tile; uploaded as 0 with the header
    uint32_t nreq;
    uint32_t chunk;
    uint32_t spans_per_tile;  // W: a tile is W consecutive spans of one request
    uint32_t pad0;
    uint64_t pad[4];
};
static_assert(sizeof(BatchHdr) == 64, "BatchHdr layout");

struct BatchView {
    BatchHdr *hdr;
    const DevReq *reqs;
    const uint32_t *map;
    const uint32_t *bounds;  // request r: lo's bits at 2r, hi - lo at 2r + 1 (integer ranges)
};

__device__ __forceinline__ uint64_t bcast_lane0(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Generate spans j0, j0 + step, ... < W of tile t of the batch (wave-uniform).
// RNG: the variant with the integer-range cases, for batches that hold one.
template <bool NT, bool F64N, bool RNG>
__device__ __forceinline__ void run_tile(const BatchView &v, uint64_t t, uint32_t W, uint32_t j0,
                                         uint32_t step, uint32_t lane) {
    const uint32_t r = v.map[t];
    const DevReq q = v.reqs[r];
    const KeySched ks = make_keysched(q.seed);
    const int gen = (int)(q.flags & 15u), dist = (int)((q.flags >> 4) & 15u);
    uint32_t lo = 0, rr = 0;
    if constexpr (RNG) {
        if (dist == D_I32R) {
            lo = v.bounds[2 * (uint64_t)r];
            rr = v.bounds[2 * (uint64_t)r + 1];
        }
    }
    const uint64_t span0 = q.first_span + (t - q.tile_start) * W;
    for (uint32_t j = j0; j < W; j += step)
        process_span_any<NT, F64N, RNG>(gen, dist, ks, q.ctr, q.out, q.p0, q.p0 + q.n,
                                        span0 + j, q.unroll, (q.flags >> 8) & 3u, lane, lo, rr);
}

template <bool NT, bool F64N, bool RNG>
__global__ __launch_bounds__(512) void k_batched(BatchView v) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t total = v.hdr->total_tiles;
    const uint32_t chunk = v.hdr->chunk, W = v.hdr->spans_per_tile;
    for (;;) {
        uint64_t t0 = 0;
        if (lane == 0)
            t0 = atomicAdd(reinterpret_cast<unsigned long long *>(&v.hdr->cursor),
                           (unsigned long long)chunk);
        t0 = bcast_lane0(t0);
        if (t0 >= total) break;
        const uint64_t t1 = t0 + chunk < total ? t0 + chunk : total;
        for (uint64_t t = t0; t < t1; ++t) run_tile<NT, F64N, RNG>(v, t, W, 0, 1, lane);
    }
}

// Static schedule: workgroup t generates tile t, wave j of it span j of the
// tile (W = waves per workgroup), so every wave is short-lived like the plain
// fill's.  The grid is rounded up to a size bucket (a multiple of the XCD
// count) so that a captured graph serves many batch sizes; workgroups past the
// last tile exit at once.  Workgroup b takes tile b: workgroups are dealt to
// the 8 XCDs round-robin, so every XCD gets an even share of the batch's
// tiles and of their costs (on MI355X 5% faster than giving each XCD a
// contiguous eighth for L2 locality of the tile map, 8% on a batch that mixes
// generators and distributions).
template <bool NT, bool F64N, bool RNG>
__global__ __launch_bounds__(512) void k_batched_static(BatchView v) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t t = blockIdx.x;
    if (t >= v.hdr->total_tiles) return;
    const uint32_t j = wave_uniform(threadIdx.x >> 6);
    run_tile<NT, F64N, RNG>(v, t, blockDim.x >> 6, j, 0xFFFFu, lane);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BatchCtx {
    char *d_buf = nullptr;
    char *h_buf = nullptr;  // pinned staging, same layout
    uint64_t cap_req = 0, cap_tiles = 0;
    hipEvent_t done = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_key[4] = {0, 0, 0, 0};
};

struct DeviceBatch {
    std::mutex mu;
    std::vector<BatchCtx> ring;
    size_t next = 0;
    hipStream_t capture = nullptr;
};

static std::mutex g_dev_mu;
static std::vector<DeviceBatch *> g_devs;

static DeviceBatch *device_batch(int dev) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if ((int)g_devs.size() <= dev) g_devs.resize(dev + 1, nullptr);
    if (!g_devs[dev]) {
        g_devs[dev] = new DeviceBatch();  // lives until process exit
        g_devs[dev]->ring.resize(3);
    }
    return g_devs[dev];
}

// Buffer layout for a capacity: header, request rows, bounds (two words per
// request), tile map.
static size_t layout_bytes(uint64_t cap_req, uint64_t cap_tiles, size_t *map_off,
                           size_t *bounds_off) {
    *bounds_off = sizeof(BatchHdr) + cap_req * sizeof(DevReq);
    *map_off = *bounds_off + cap_req * 2 * sizeof(uint32_t);
    return *map_off + cap_tiles * sizeof(uint32_t);
}

static hipError_t ensure_capacity(BatchCtx &c, uint64_t nreq, uint64_t tiles) {
    if (nreq <= c.cap_req && tiles <= c.cap_tiles && c.d_buf) return hipSuccess;
    const uint64_t nr = std::max<uint64_t>(std::max<uint64_t>(nreq, c.cap_req * 3 / 2), 1024);
    const uint64_t nt = std::max<uint64_t>(std::max<uint64_t>(tiles, c.cap_tiles * 3 / 2), 65536);
    size_t map_off, bounds_off;
    const size_t bytes = layout_bytes(nr, nt, &map_off, &bounds_off);
    hipError_t e;
    if (c.exec) { hipGraphExecDestroy(c.exec); c.exec = nullptr; }
    if (c.graph) { hipGraphDestroy(c.graph); c.graph = nullptr; }
    if (c.d_buf) { hipFree(c.d_buf); c.d_buf = nullptr; }
    if (c.h_buf) { hipHostFree(c.h_buf); c.h_buf = nullptr; }
    c.cap_req = c.cap_tiles = 0;
    if ((e = hipMalloc(&c.d_buf, bytes)) != hipSuccess) return e;
    if ((e = hipHostMalloc(&c.h_buf, bytes, hipHostMallocDefault)) != hipSuccess) return e;
    c.cap_req = nr;
    c.cap_tiles = nt;
    return hipSuccess;
}

// Launch shape shared by the batched and served kernels.
struct BatchShape {
    uint32_t wg, grid, chunk;
    bool nt;
    bool persistent;
};

// Smallest bucket >= x with 1/8 granularity (keeps captured graphs reusable).
static uint64_t bucket(uint64_t x) {
    if (x <= 64) return x;
    int k = 63 - __builtin_clzll(x);
    const uint64_t step = 1ull << (k - 3);
    return (x + step - 1) / step * step;
}

uint32_t batch_wg(int gen, int dist) {
    const LaunchCfg cfg = launch_cfg();
    return cfg.wg_size ? cfg.wg_size : tuned_fill(gen, dist).b_wg_size;
}

static BatchShape batch_shape(int gen, int dist, uint64_t tiles) {
    const Tuned tu = tuned_fill(gen, dist);
    const LaunchCfg cfg = launch_cfg();
    BatchShape s;
    s.wg = batch_wg(gen, dist);
    s.chunk = tu.b_chunk ? tu.b_chunk : 1;
    s.nt = false;
    const uint64_t wpg = s.wg / 64;
    // b_wgs_per_cu == 0 selects the static one-workgroup-per-tile schedule,
    // unless its grid would pass the dispatch limit of 2^32 work-items per
    // dimension (batches of 2^23 tiles and more, 16 GiB or more of output)
    const bool static_fits = (bucket(tiles) + XCDS - 1) / XCDS * XCDS <= max_wgs_1d(s.wg);
    s.persistent = tu.b_wgs_per_cu != 0 || cfg.max_wgs != 0 || !static_fits;
    if (s.persistent) {
        uint64_t grid = (uint64_t)device_cu_count() * (tu.b_wgs_per_cu ? tu.b_wgs_per_cu : 4);
        if (cfg.max_wgs) grid = cfg.max_wgs;
        const uint64_t need = (tiles + wpg - 1) / wpg;  // one tile per wave at a time
        s.grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(grid, need));
    } else {
        s.grid = (uint32_t)((bucket(tiles) + XCDS - 1) / XCDS * XCDS);  // one workgroup per tile
    }
    return s;
}

template <bool F64N, bool RNG>
static void *batched_kernel_v(const BatchShape &s) {
    if (s.persistent)
        return s.nt ? reinterpret_cast<void *>(&k_batched<true, F64N, RNG>)
                    : reinterpret_cast<void *>(&k_batched<false, F64N, RNG>);
    return s.nt ? reinterpret_cast<void *>(&k_batched_static<true, F64N, RNG>)
                : reinterpret_cast<void *>(&k_batched_static<false, F64N, RNG>);
}

// The variants with the float64 normal cases, or with the integer-range cases,
// only for batches that hold such a request (each set of cases raises the
// kernel's register count, so its occupancy, for every other request).
static void *batched_kernel(const BatchShape &s, bool f64n, bool rng) {
    if (f64n)
        return rng ? batched_kernel_v<true, true>(s) : batched_kernel_v<true, false>(s);
    return rng ? batched_kernel_v<false, true>(s) : batched_kernel_v<false, false>(s);
}

// Tile decomposition of one request: spans of `unroll` blocks per lane,
// W spans per tile.
// (Span and tile sizes are powers of two at every built-in launch shape; the
// quotients are then shifts, which halves the tiling pass over 10^5 requests.)
void request_tiles(const orng_req_t &r, uint32_t unroll, uint32_t W, uint64_t *first_span,
                   uint64_t *count) {
    const uint64_t sb = span_blocks((int)r.gen, unroll);
    const uint64_t k = words_per_sample((int)r.dist);
    const uint64_t fb = r.offset * k / 4, lb = ((r.offset + r.n) * k - 1) / 4;
    uint64_t spans;
    if ((sb & (sb - 1)) == 0 && (W & (W - 1)) == 0) {
        const int s = __builtin_ctzll(sb), w = __builtin_ctz(W);
        *first_span = fb >> s;
        spans = (lb >> s) - *first_span + 1;
        *count = (spans + W - 1) >> w;
        return;
    }
    *first_span = fb / sb;
    spans = lb / sb - *first_span + 1;
    *count = (spans + W - 1) / W;
}

// Host worker threads for the batched path's preparation passes: started on
// first use and kept (detached, waiting on a condition variable) until the
// process ends, so a call pays a wake-up instead of thread creation.  One
// job at a time; run(T, f) calls f(t) for t in [0, T), t = 0 on the caller.
class HostPool {
  public:
    static HostPool &get() {
        static HostPool *p = new HostPool();  // never destroyed: workers outlive main
        return *p;
    }
    size_t size() const { return workers_ + 1; }
    template <class F>
    void run(size_t T, F f) {
        T = std::min(T, size());
        if (T <= 1) { f(size_t(0)); return; }
        std::lock_guard<std::mutex> one(job_mu_);  // one job at a time
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = [&f](size_t t) { f(t); };
            parts_ = T;
            pending_ = T - 1;
            ++gen_;
        }
        cv_.notify_all();
        f(size_t(0));
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return pending_ == 0; });
        job_ = nullptr;
    }

  private:
    HostPool() {
        const size_t hw = std::max(1u, std::thread::hardware_concurrency());
        workers_ = std::min<size_t>(7, hw > 1 ? hw - 1 : 0);
        for (size_t w = 1; w <= workers_; ++w) std::thread([this, w] { loop(w); }).detach();
    }
    void loop(size_t w) {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (w >= parts_) continue;
            auto job = job_;
            lk.unlock();
            job(w);
            lk.lock();
            if (--pending_ == 0) done_.notify_one();
        }
    }
    size_t workers_ = 0;
    std::mutex job_mu_, mu_;
    std::condition_variable cv_, done_;
    std::function<void(size_t)> job_;
    size_t parts_ = 0, pending_ = 0;
    uint64_t gen_ = 0;
};

// Contiguous ranges [begin(t), begin(t+1)) of [0, n) for up to eight host
// threads (one for small n); run(f) calls f(t, begin, end) for every range.
struct Ranges {
    size_t n, T;
    explicit Ranges(size_t n_) : n(n_) {
        T = n < 8192 ? 1 : std::min<size_t>(HostPool::get().size(), n / 4096);
    }
    size_t begin(size_t t) const { return n * t / T; }
    template <class F>
    void run(F f) const {
        HostPool::get().run(T, [&](size_t t) { f(t, begin(t), begin(t + 1)); });
    }
};

static bool use_graphs() {
    static const bool on = [] {
        const char *e = getenv("ORNG_NO_GRAPH");
        return !(e && *e && *e != '0');
    }();
    return on;
}

// Table row of one request; `ts` is its first tile, `cnt` its tile count;
// bounds[0..1] receive its integer-range bounds.
static void make_row(DevReq &d, uint32_t *bounds, const orng_req_t &r, uint32_t unroll,
                     uint64_t first_span, uint64_t ts, uint64_t cnt) {
    const uint64_t kw = words_per_sample((int)r.dist);
    d.out = static_cast<char *>(r.out);
    d.p0 = r.offset * kw;  // positions and counts in stream words from here on
    d.n = r.n * kw;
    d.seed = r.seed;
    d.first_span = first_span;
    d.tile_start = ts;
    d.ctr = r.ctr;
    d.unroll = unroll;
    d.flags = r.gen | (r.dist << 4) | (output_delta(r, r.out) << 8);
    d.tiles = (uint32_t)cnt;
    range_bounds(r, &bounds[0], &bounds[1]);
}

// The (generator, distribution) pair holding most of a batch's words picks the
// batch's launch shape (workgroup size, so the tile size, and the schedule);
// ties go to the lower pair number.
static int dominant_pair(const uint64_t *words) {
    int best = 0;
    for (int k = 1; k < NGEN * NDIST; ++k)
        if (words[k] > words[best]) best = k;
    return best;
}

// Blocks per lane per tile of every (generator, request distribution); an
// integer-range request takes its launch row from the float64 uniform one.
static void unroll_table(uint32_t unroll_of[NGEN][NREQDIST]) {
    for (int g = 0; g < NGEN; ++g)
        for (int d = 0; d < NREQDIST; ++d)
            unroll_of[g][d] = tyche_like(g) ? 64 : tuned_fill(g, shape_dist(d)).b_unroll;
}

int fill_batched(const orng_req_t *reqs, size_t nreq, hipStream_t stream) {
    if (nreq && !reqs) return ORNG_EINVAL;
    if (!nreq) return ORNG_OK;
    if (nreq > 0xFFFFFFFFull) return ORNG_ENOMEM;  // the tile map holds 32-bit request numbers
    // Host preparation in three parallel passes over contiguous ranges of the
    // request list: (1) validate every request and count the words of each
    // (generator, distribution) pair, which picks the launch shape; (2) tile
    // every request, summing each range's tiles; then, after a scan over the
    // ranges, (3) write each request's table row and its tiles' entries of
    // the tile map.  Every request keeps its own row (one without work owns no
    // tiles).
    const Ranges rg(nreq);
    constexpr int NP = NGEN * NDIST;
    std::vector<uint64_t> range_words(rg.T * NP, 0);
    std::vector<size_t> range_bad(rg.T, nreq);  // first invalid request of each range
    std::vector<int> range_st(rg.T, ORNG_OK);
    std::vector<char> range_rng(rg.T, 0);       // the range holds an integer-range request
    rg.run([&](size_t t, size_t a, size_t b) {
        uint64_t *w = &range_words[t * NP];
        for (size_t i = a; i < b; ++i) {
            const int st = validate_request(reqs[i]);
            if (st != ORNG_OK) { range_bad[t] = i; range_st[t] = st; return; }
            w[reqs[i].gen * NDIST + shape_dist((int)reqs[i].dist)] +=
                reqs[i].n * words_per_sample((int)reqs[i].dist);
            if (reqs[i].dist == ORNG_I32_RANGE && reqs[i].n) range_rng[t] = 1;
        }
    });
    for (size_t t = 0; t < rg.T; ++t)
        if (range_bad[t] < nreq) return range_st[t];  // ranges are in list order
    uint64_t words[NP] = {0};
    for (size_t t = 0; t < rg.T; ++t)
        for (int k = 0; k < NP; ++k) words[k] += range_words[t * NP + k];
    const bool f64n = [&] {
        for (int g = 0; g < NGEN; ++g)
            if (words[g * NDIST + ORNG_F64_NORMAL]) return true;
        return false;
    }();
    const bool rng = std::find(range_rng.begin(), range_rng.end(), 1) != range_rng.end();
    const int pair = dominant_pair(words);
    const uint32_t W = batch_wg(pair / NDIST, pair % NDIST) / 64;
    uint32_t unroll_of[NGEN][NREQDIST];  // one table lookup per pair, not per request
    unroll_table(unroll_of);

    // per-request first span and tile count: for batches of up to 2^20
    // requests in arrays kept by the calling thread across calls (fresh ones
    // cost a page fault per 4 KiB on first touch; at most 16 MiB per thread),
    // for larger ones in arrays of this call
    constexpr size_t KEEP = size_t(1) << 20;
    static thread_local std::vector<uint64_t> t_fspan, t_cnt;
    std::vector<uint64_t> big_fspan, big_cnt;
    uint64_t *fspan, *cnt;
    if (nreq <= KEEP) {
        if (t_fspan.size() < nreq) {
            t_fspan.resize(nreq);
            t_cnt.resize(nreq);
        }
        fspan = t_fspan.data();
        cnt = t_cnt.data();
    } else {
        big_fspan.resize(nreq);
        big_cnt.resize(nreq);
        fspan = big_fspan.data();
        cnt = big_cnt.data();
    }
    std::vector<uint64_t> range_tiles(rg.T + 1, 0);
    rg.run([&](size_t t, size_t a, size_t b) {
        uint64_t sum = 0;
        for (size_t i = a; i < b; ++i) {
            cnt[i] = 0;
            fspan[i] = 0;
            if (!reqs[i].n) continue;
            request_tiles(reqs[i], unroll_of[reqs[i].gen][reqs[i].dist], W, &fspan[i], &cnt[i]);
            sum += cnt[i];
        }
        range_tiles[t + 1] = sum;
    });
    for (size_t t = 0; t < rg.T; ++t) range_tiles[t + 1] += range_tiles[t];
    const uint64_t tiles = range_tiles[rg.T];
    if (tiles == 0) return ORNG_OK;
    if (tiles > (1ull << 28)) return ORNG_ENOMEM;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
    DeviceBatch *db = device_batch(dev);
    std::lock_guard<std::mutex> lk(db->mu);
    BatchCtx &c = db->ring[db->next];
    db->next = (db->next + 1) % db->ring.size();
#define ORNG_TRY(x) do { e = (x); if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; } } while (0)
    if (!c.done) ORNG_TRY(hipEventCreateWithFlags(&c.done, hipEventDisableTiming));
    else ORNG_TRY(hipEventSynchronize(c.done));  // staging and tables of its last use are free
    ORNG_TRY(ensure_capacity(c, nreq, tiles));
    if (!db->capture) ORNG_TRY(hipStreamCreateWithFlags(&db->capture, hipStreamNonBlocking));

    const BatchShape sh = batch_shape(pair / NDIST, pair % NDIST, tiles);
    size_t map_off, bounds_off;
    layout_bytes(c.cap_req, c.cap_tiles, &map_off, &bounds_off);
    BatchHdr *hdr = reinterpret_cast<BatchHdr *>(c.h_buf);
    DevReq *dq = reinterpret_cast<DevReq *>(c.h_buf + sizeof(BatchHdr));
    uint32_t *bounds = reinterpret_cast<uint32_t *>(c.h_buf + bounds_off);
    uint32_t *map = reinterpret_cast<uint32_t *>(c.h_buf + map_off);
    std::memset(hdr, 0, sizeof(BatchHdr));
    hdr->total_tiles = tiles;
    hdr->cursor = 0;
    hdr->nreq = (uint32_t)nreq;
    hdr->chunk = sh.chunk;
    hdr->spans_per_tile = W;
    rg.run([&](size_t t, size_t a, size_t b) {
        uint64_t ts = range_tiles[t];
        for (size_t i = a; i < b; ++i) {
            const orng_req_t &r = reqs[i];
            make_row(dq[i], bounds + 2 * i, r, r.n ? unroll_of[r.gen][r.dist] : 0, fspan[i], ts,
                     cnt[i]);
            std::fill_n(map + ts, cnt[i], (uint32_t)i);
            ts += cnt[i];
        }
    });
    ORNG_TRY(hipMemcpyAsync(c.d_buf, c.h_buf, sizeof(BatchHdr) + nreq * sizeof(DevReq),
                            hipMemcpyHostToDevice, stream));
    ORNG_TRY(hipMemcpyAsync(c.d_buf + map_off, c.h_buf + map_off, tiles * sizeof(uint32_t),
                            hipMemcpyHostToDevice, stream));
    if (rng)
        ORNG_TRY(hipMemcpyAsync(c.d_buf + bounds_off, c.h_buf + bounds_off,
                                nreq * 2 * sizeof(uint32_t), hipMemcpyHostToDevice, stream));

    BatchView v;
    v.hdr = reinterpret_cast<BatchHdr *>(c.d_buf);
    v.reqs = reinterpret_cast<const DevReq *>(c.d_buf + sizeof(BatchHdr));
    v.map = reinterpret_cast<const uint32_t *>(c.d_buf + map_off);
    v.bounds = reinterpret_cast<const uint32_t *>(c.d_buf + bounds_off);
    void *args[] = {&v};
    if (use_graphs()) {
        const uint64_t key[4] = {reinterpret_cast<uintptr_t>(c.d_buf), sh.wg, sh.grid,
                                 (uint64_t)sh.nt | ((uint64_t)sh.persistent << 1) |
                                     ((uint64_t)f64n << 2) | ((uint64_t)rng << 3)};
        if (!c.exec || std::memcmp(key, c.graph_key, sizeof key) != 0) {
            if (c.exec) { hipGraphExecDestroy(c.exec); c.exec = nullptr; }
            if (c.graph) { hipGraphDestroy(c.graph); c.graph = nullptr; }
            ORNG_TRY(hipStreamBeginCapture(db->capture, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipLaunchKernel(batched_kernel(sh, f64n, rng), dim3(sh.grid),
                                            dim3(sh.wg), args, 0, db->capture);
            hipError_t ce = hipStreamEndCapture(db->capture, &c.graph);
            ORNG_TRY(le);
            ORNG_TRY(ce);
            ORNG_TRY(hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0));
            std::memcpy(c.graph_key, key, sizeof key);
        }
        ORNG_TRY(hipGraphLaunch(c.exec, stream));
    } else {
        ORNG_TRY(hipLaunchKernel(batched_kernel(sh, f64n, rng), dim3(sh.grid), dim3(sh.wg), args,
                                 0, stream));
    }
    ORNG_TRY(hipEventRecord(c.done, stream));
#undef ORNG_TRY
    return ORNG_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free variant of fill_batched
// ---------------------------------------------------------------------------
// For callers that cannot allocate: the batch's header, request table and tile
// map live in `scratch`, a device array of fixed size defined here, instead of
// a buffer the library allocates.  Host code never passes the array's name to
// a kernel or a copy (in host code it is a host-side stand-in, not a device
// address): the address is looked up once per device with
// hipGetSymbolAddress, while that device is current, and only that address is
// used.  The host writes the header and the request rows in one serial pass
// into a static host array; the upload from that pageable array is done before
// hipMemcpyAsync returns, so the array is free again when the call returns.  A
// small kernel then writes the tile map from the rows, and the generation
// kernel is the one orng_fill_batched runs (launched directly, no graph).
// Every call on a device shares its scratch: calls on one stream follow each
// other in stream order; calls that overlap on one device race.
constexpr uint64_t NOALLOC_ROWS_END =
    sizeof(BatchHdr) + (uint64_t)ORNG_NOALLOC_MAX_REQUESTS * sizeof(DevReq);
constexpr uint64_t NOALLOC_BOUNDS_OFF = NOALLOC_ROWS_END;  // two words per request
constexpr uint64_t NOALLOC_STAGE_END =
    NOALLOC_BOUNDS_OFF + (uint64_t)ORNG_NOALLOC_MAX_REQUESTS * 2 * sizeof(uint32_t);
constexpr uint64_t NOALLOC_MAP_OFF = (NOALLOC_STAGE_END + 255) / 256 * 256;
constexpr uint64_t NOALLOC_BYTES =
    NOALLOC_MAP_OFF + (uint64_t)ORNG_NOALLOC_MAX_TILES * sizeof(uint32_t);

static __device__ __align__(256) char scratch[NOALLOC_BYTES];

static std::mutex g_na_mu;                        // one allocation-free call at a time per process
alignas(64) static char g_na_stage[NOALLOC_STAGE_END];  // host: header, rows, bounds
constexpr int NOALLOC_MAX_DEVICES = 64;
static char *g_na_ptr[NOALLOC_MAX_DEVICES];       // device address of `scratch`, per device

// Tile map from the request rows: wave r writes the entries of request r.
__global__ __launch_bounds__(256) void k_tile_map(const DevReq *reqs, uint32_t nreq,
                                                  uint32_t *map) {
    const uint32_t r = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (r >= nreq) return;
    const uint64_t t0 = reqs[r].tile_start;
    const uint32_t cnt = reqs[r].tiles;
    for (uint32_t k = threadIdx.x & 63u; k < cnt; k += 64u) map[t0 + k] = r;
}

int fill_batched_noalloc(const orng_req_t *reqs, size_t nreq, hipStream_t stream) {
    if (nreq && !reqs) return ORNG_EINVAL;
    if (!nreq) return ORNG_OK;
    constexpr int NP = NGEN * NDIST;
    uint64_t words[NP] = {0};
    bool rng = false;
    for (size_t i = 0; i < nreq; ++i) {
        const int st = validate_request(reqs[i]);
        if (st != ORNG_OK) return st;
        words[reqs[i].gen * NDIST + shape_dist((int)reqs[i].dist)] +=
            reqs[i].n * words_per_sample((int)reqs[i].dist);
        rng = rng || (reqs[i].dist == ORNG_I32_RANGE && reqs[i].n);
    }
    if (nreq > ORNG_NOALLOC_MAX_REQUESTS) return ORNG_ENOMEM;
    bool f64n = false;
    for (int g = 0; g < NGEN; ++g) f64n = f64n || words[g * NDIST + ORNG_F64_NORMAL] != 0;
    const int pair = dominant_pair(words);
    const uint32_t W = batch_wg(pair / NDIST, pair % NDIST) / 64;
    uint32_t unroll_of[NGEN][NREQDIST];
    unroll_table(unroll_of);

    std::lock_guard<std::mutex> lk(g_na_mu);
    DevReq *rows = reinterpret_cast<DevReq *>(g_na_stage + sizeof(BatchHdr));
    uint32_t *bounds = reinterpret_cast<uint32_t *>(g_na_stage + NOALLOC_BOUNDS_OFF);
    uint64_t tiles = 0;
    for (size_t i = 0; i < nreq; ++i) {
        const orng_req_t &r = reqs[i];
        uint64_t fs = 0, cnt = 0;
        if (r.n) request_tiles(r, unroll_of[r.gen][r.dist], W, &fs, &cnt);
        if (cnt > ORNG_NOALLOC_MAX_TILES - tiles) return ORNG_ENOMEM;
        make_row(rows[i], bounds + 2 * i, r, r.n ? unroll_of[r.gen][r.dist] : 0, fs, tiles, cnt);
        tiles += cnt;
    }
    if (tiles == 0) return ORNG_OK;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return ORNG_ENOMEM;
    if (!g_na_ptr[dev]) {  // set-up, once per device, with that device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) { set_hip_error(e); return ORNG_EHIP; }
        g_na_ptr[dev] = static_cast<char *>(p);
    }
    char *base = g_na_ptr[dev];

    const BatchShape sh = batch_shape(pair / NDIST, pair % NDIST, tiles);
    BatchHdr *hdr = reinterpret_cast<BatchHdr *>(g_na_stage);
    std::memset(hdr, 0, sizeof(BatchHdr));
    hdr->total_tiles = tiles;
    hdr->cursor = 0;  // the work queue starts empty on every call
    hdr->nreq = (uint32_t)nreq;
    hdr->chunk = sh.chunk;
    hdr->spans_per_tile = W;
#define ORNG_TRY(x) do { e = (x); if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; } } while (0)
    ORNG_TRY(hipMemcpyAsync(base, g_na_stage, sizeof(BatchHdr) + nreq * sizeof(DevReq),
                            hipMemcpyHostToDevice, stream));
    if (rng)
        ORNG_TRY(hipMemcpyAsync(base + NOALLOC_BOUNDS_OFF, g_na_stage + NOALLOC_BOUNDS_OFF,
                                nreq * 2 * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    BatchView v;
    v.hdr = reinterpret_cast<BatchHdr *>(base);
    v.reqs = reinterpret_cast<const DevReq *>(base + sizeof(BatchHdr));
    v.map = reinterpret_cast<const uint32_t *>(base + NOALLOC_MAP_OFF);
    v.bounds = reinterpret_cast<const uint32_t *>(base + NOALLOC_BOUNDS_OFF);
    uint32_t *map = reinterpret_cast<uint32_t *>(base + NOALLOC_MAP_OFF);
    const uint32_t nr = (uint32_t)nreq;
    void *margs[] = {&v.reqs, const_cast<uint32_t *>(&nr), &map};
    ORNG_TRY(hipLaunchKernel(reinterpret_cast<void *>(&k_tile_map), dim3((nr + 3) / 4), dim3(256),
                             margs, 0, stream));
    void *args[] = {&v};
    ORNG_TRY(hipLaunchKernel(batched_kernel(sh, f64n, rng), dim3(sh.grid), dim3(sh.wg), args, 0,
                             stream));
#undef ORNG_TRY
    return ORNG_OK;
}

}  // namespace orng

extern "C" {

int orng_fill_batched(const orng_req_t *h_reqs, size_t nreq, void *stream) {
    return orng::fill_batched(h_reqs, nreq, static_cast<hipStream_t>(stream));
}

int orng_fill_batched_noalloc(const orng_req_t *h_reqs, size_t nreq, void *stream) {
    return orng::fill_batched_noalloc(h_reqs, nreq, static_cast<hipStream_t>(stream));
}

int orng_fill_each(const orng_req_t *h_reqs, size_t nreq, void *stream) {
    if (nreq && !h_reqs) return ORNG_EINVAL;
    for (size_t i = 0; i < nreq; ++i) {
        const int st = orng::validate_request(h_reqs[i]);
        if (st != ORNG_OK) return st;
    }
    for (size_t i = 0; i < nreq; ++i) {
        const orng_req_t &r = h_reqs[i];
        if (!r.n) continue;
        if (r.dist == ORNG_I32_RANGE) {
            const int st = orng_fill_range((int)r.gen, r.seed, r.ctr, 1, r.offset, r.n, r.lo,
                                           r.hi, static_cast<int32_t *>(r.out), stream);
            if (st != ORNG_OK) return st;
            continue;
        }
        const uint64_t k = orng::words_per_sample((int)r.dist);
        hipError_t e = orng::launch_fill((int)r.gen, (int)r.dist, r.seed, r.ctr, 1, r.offset * k,
                                         r.n * k, r.out, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) {
            orng::set_hip_error(e);
            return ORNG_EHIP;
        }
    }
    return ORNG_OK;
}

}  // extern "C"
