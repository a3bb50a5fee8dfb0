/*
 * orng.h -- C interface of liborng, counter-based random number generation
 * on MI355X (gfx950).
 *
 * Stream model (OpenRAND paper, section 3.1 "API Design"): a generator is
 * addressed by a 64-bit seed and a 32-bit counter; together they name one
 * stream of period 2^32 words.  The seed identifies a processing element (a
 * particle, a pixel), the counter gives it as many independent streams as it
 * needs.  Generation is stateless (section 3.1, second paragraph): every
 * output is a pure function of (generator, distribution, seed, counter,
 * position), so results never depend on launch geometry, thread count,
 * batching, other requests or timing (section 4).
 *
 * Generators (section 3.1): Philox4x32-10 and Threefry (4x32-20, 2x64-20)
 * after Salmon et al. SC'11, Squares (32-bit output, four rounds) after
 * Widynski 2020, Tyche after Neves and Araujo 2012; and the variants
 * Threefry 13-round, Tyche-i, Squares64 and Philox2x32-10.
 *
 * Conventions shared by every call:
 *  - Device pointers are caller-owned HIP device allocations; the library never
 *    frees caller memory.  Output pointers must be 4-byte aligned; 16-byte
 *    alignment of the block grid (out address in words minus offset being a
 *    multiple of 4) is the fast path.
 *  - `stream` is a hipStream_t passed as an opaque pointer (NULL: the null
 *    stream).  Calls that take a stream enqueue work on it and return at once.
 *  - Every call returns ORNG_OK (0) or a negative status; none aborts.  After
 *    ORNG_EHIP, orng_last_hip_error() gives the HIP error code (per thread).
 *  - n == 0 is a no-op that returns ORNG_OK (pointers may then be NULL).
 */
#ifndef ORNG_H
#define ORNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* generators */
enum {
    ORNG_PHILOX4X32_10 = 0,
    ORNG_THREEFRY4X32_20 = 1,
    ORNG_THREEFRY2X64_20 = 2,
    ORNG_SQUARES32 = 3,
    ORNG_TYCHE = 4,
    ORNG_THREEFRY4X32_13 = 5, /* the Threefry rounds stopped after round 13 */
    ORNG_THREEFRY2X64_13 = 6,
    ORNG_TYCHE_I = 7,         /* Tyche on the inverse of its mixing round */
    ORNG_SQUARES64 = 8,       /* five-round Squares, 64 bits (two words) per call */
    ORNG_PHILOX2X32 = 9       /* two-word Philox; one 32-bit key word: seeds < 2^32 */
};

/* distributions; samples are 4 bytes, 8 for the two float64 ones */
enum {
    ORNG_U32 = 0,         /* raw 32-bit word */
    ORNG_F32_UNIFORM = 1, /* (word >> 8) * 2^-24, in [0, 1) */
    ORNG_F32_NORMAL = 2,  /* Box-Muller, one member of a pair per sample */
    ORNG_F64_UNIFORM = 3, /* two words per sample: ((w1 << 32 | w0) >> 11) * 2^-53, in [0, 1) */
    ORNG_F64_NORMAL = 4,  /* float64 Box-Muller, pair m from the four words 4m..4m+3 */
    ORNG_I32_RANGE = 5    /* int32 in [lo, hi) from the word pair 2p, 2p+1 (orng_fill_range);
                             request records only: they carry the bounds */
};

/* status codes */
enum {
    ORNG_OK = 0,
    ORNG_EINVAL = -1, /* bad enum, NULL pointer with work to do, misalignment, bad dim */
    ORNG_ERANGE = -2, /* position past the stream period, counter overflow */
    ORNG_ENOMEM = -3, /* request larger than the memory it may use */
    ORNG_EAGAIN = -4, /* resources momentarily exhausted (non-blocking calls) */
    ORNG_EBUSY = -5,  /* result not ready yet */
    ORNG_EHIP = -6,   /* HIP runtime error, see orng_last_hip_error() */
    ORNG_ENOENT = -7  /* unknown ticket / object */
};

/*
 * orng_fill -- out[j] = sample (offset + j) of stream (seed, ctr), j < n.
 *
 * Paper section 3.1 (stream = seed + counter, period 2^32).  Sample p of a
 * distribution uses word p (U32, F32_UNIFORM); F64_UNIFORM sample p uses
 * words 2p (w0) and 2p+1 (w1), so its samples end at 2^31 (the float64 draw
 * of the paper's example, section 4 Fig. 1); for F32_NORMAL, sample p is
 * member p mod 2 of the Box-Muller pair built from words 2*(p/2) and
 * 2*(p/2)+1.  For F64_NORMAL, sample p is member p mod 2 of the pair built
 * from words 4*(p/2) .. 4*(p/2)+3: x = (w1 << 32) | w0, y = (w3 << 32) | w2,
 * u1 = ((x >> 11) + 1) 2^-53, u2 = (y >> 11) 2^-53, R = sqrt(-2 ln u1),
 * (R cos 2 pi u2, R sin 2 pi u2), with the library's own float64 ln, cos and
 * sin (each within 2 ulp; results are reproducible bit for bit).  Both float64
 * distributions use two words per sample, so their samples end at 2^31.
 * The stream's words are:
 *   Philox4x32-10  : word p = word p%4 of Philox(counter (p/4, ctr, 0, 0),
 *                    key (lo32 seed, hi32 seed))
 *   Threefry4x32-20: same counter, key (lo32 seed, hi32 seed, 0, 0)
 *   Threefry2x64-20: counter (p/4, ctr) as 64-bit words, key (seed, 0);
 *                    words lo X0, hi X0, lo X1, hi X1
 *   Threefry4x32-13, Threefry2x64-13: as their 20-round forms, with the
 *                    key injections after rounds 4, 8 and 12 and 13 rounds
 *   Squares32      : squares32(counter (ctr << 32) | p, key K(seed)),
 *                    K = SplitMix64 output step of seed, low bit set (two
 *                    seeds per key: those whose SplitMix64 outputs differ
 *                    only in bit 0; below 2^32 only 369106595 and
 *                    2888123536 pair up)
 *   Tyche          : tiles of 16384 words; word p of tile t = p / 16384,
 *                    r = p % 16384 is output 4*(r/256) + r%4 of the Tyche
 *                    instance seeded with (seed, ctr) whose c word is XORed
 *                    with t*64 + (r/4)%64.
 *   Tyche-i        : the Tyche layout and seeding with MIX-i, the inverse of
 *                    Tyche's MIX (its four steps undone in reverse order)
 *   Squares64      : word p = low (p even) or high half of
 *                    squares64(counter (ctr << 32) | p/2, key K(seed))
 *   Philox2x32-10  : word p = word p%2 of Philox2x32(counter (p/2, ctr),
 *                    key seed); its key is one 32-bit word, so it takes
 *                    seeds below 2^32 only (as the paper's Squares takes
 *                    32-bit seeds, section 3.1)
 * Arguments: gen, dist (enums above); d_out: device buffer of n samples
 * (n * 4 bytes, 4-byte aligned; n * 8 bytes, 8-byte aligned for the float64
 * distributions).
 * Errors: EINVAL (enum, NULL, alignment, a Philox2x32 seed of 2^32 or more;
 *         ORNG_I32_RANGE too, which needs bounds: orng_fill_range),
 *         ERANGE (offset + n past the last sample: 2^32, or 2^31 for the
 *         float64 distributions).
 */
int orng_fill(int gen, int dist, uint64_t seed, uint32_t ctr, uint64_t offset, uint64_t n,
              void *d_out, void *stream);

/*
 * orng_fill_multi -- out[i * per_stream + j] = sample (offset + j) of stream
 * (seed, ctr0 + i), for i < n_streams, j < per_stream.  One seed, many
 * counters: the "multiple streams per seed" use of section 3.1.
 * Errors: as orng_fill, plus ERANGE when ctr0 + n_streams - 1 overflows 32 bits.
 */
int orng_fill_multi(int gen, int dist, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                    uint64_t offset, uint64_t per_stream, void *d_out, void *stream);

/*
 * orng_particle_streams -- parallel micro-streams for statistical testing of
 * parallel streams (section 5.2, after the procedure it cites):
 *   out[(t * n_particles + p) * draws + k] = word k of stream
 *                                           (seed0 + p, ctr0 + t)
 * for t < n_iters, p < n_particles, k < draws: each particle draws a
 * micro-stream of `draws` words per iteration from its own stream, keyed as
 * in the paper's example (seed = particle id, counter = iteration); an
 * iteration's micro-streams are concatenated in particle order.  Word k is
 * orng_fill's word at position k of the same stream.
 * d_out: device buffer of n_iters * n_particles * draws 32-bit words.
 * Errors: EINVAL (gen, draws not in 1..16, NULL or misaligned d_out), ERANGE
 *         (ctr0 + n_iters - 1 > 2^32 - 1, seed0 + n_particles - 1 overflows
 *         64 bits, or for Philox2x32 exceeds 2^32 - 1).  n_particles = 0 or
 *         n_iters = 0 does nothing.
 */
int orng_particle_streams(int gen, uint64_t seed0, uint32_t n_particles, uint32_t draws,
                          uint32_t ctr0, uint32_t n_iters, void *d_out, void *stream);

/*
 * orng_fill_range -- integers in [lo, hi): d_out[i * per_stream + j] = sample
 * (offset + j) of stream (seed, ctr0 + i), for i < n_streams, j < per_stream.
 * The generators are meant to feed standard distributions (section 3); this is
 * the integer one.  Sample p takes x = (w1 << 32) | w0 from the words w0, w1 at
 * positions 2p and 2p+1 of the stream (the word pair of ORNG_F64_UNIFORM) and
 * returns lo + floor(x * (hi - lo) / 2^64).  Every value's probability is
 * within 2^-64 of 1 / (hi - lo): no remainder is taken (x mod r of one word
 * favours low values by up to 2:1) and nothing is rejected, so each sample
 * keeps its fixed positions and any range of samples can be made directly.
 * Positions: offset + per_stream <= 2^31 samples per stream.
 * d_out: device buffer of n_streams * per_stream int32 (caller-owned, 4-byte
 *   aligned; 16-byte alignment of d_out + offset is the fast path).
 * Errors: EINVAL (gen, lo >= hi, a Philox2x32 seed of 2^32 or more, NULL or
 *         misaligned d_out with work to do),
 *         ERANGE (offset + per_stream > 2^31, ctr0 + n_streams - 1 > 2^32 - 1).
 *         n_streams = 0 or per_stream = 0 does nothing.
 */
int orng_fill_range(int gen, uint64_t seed, uint32_t ctr0, uint32_t n_streams, uint64_t offset,
                    uint64_t per_stream, int32_t lo, int32_t hi, int32_t *d_out, void *stream);

/*
 * orng_brownian -- fused overdamped Brownian walk (paper section 4, Fig. 1;
 * section 5.1), all steps in one launch.
 * Particle i (0 <= i < n_particles) owns the Philox4x32-10 stream
 * (seed, ctr0 + i).  Global step g = step0 + s (s < n_steps) uses F32_NORMAL
 * samples dim*g .. dim*g + dim - 1 of that stream and updates
 * x_d = fmaf(sigma, normal_d, x_d), sigma = (float)sqrt(2.0 * D * dt).
 * d_pos: float SoA [dim][n_particles], read and written in place.
 * d_msd: NULL, or n_steps / msd_every doubles; entry q receives the sum over
 *        all particles of |x|^2 after local step (q + 1) * msd_every (the
 *        library zeroes it first).  Summation order is not fixed, so d_msd is
 *        reproducible only to rounding.
 * Resuming from saved positions with step0 = k continues the same walk.
 * Errors: EINVAL (dim not 1..3, NULL d_pos), ERANGE (dim*(step0+n_steps) >
 *         2^32 or ctr0 + n_particles - 1 overflows).
 */
int orng_brownian(uint64_t seed, uint32_t ctr0, uint32_t n_particles, uint32_t dim,
                  uint64_t step0, uint32_t n_steps, float dt, float D, float *d_pos,
                  double *d_msd, uint32_t msd_every, void *stream);

/*
 * orng_bd2 -- the paper's 2-D Brownian dynamics example (section 4, Fig. 1,
 * run as the GPU benchmark of section 5.1), in float64.
 * Particle i (0 <= i < n) has id pid = pid0 + i, which is its generator's
 * seed; step s (s < n_steps) uses counter step0 + s.  Per step, with r.x from
 * words 0, 1 and r.y from words 2, 3 of Philox4x32-10 stream (pid, step0 + s),
 * each word pair (w0, w1) read as the double ((w1 << 32 | w0) >> 11) * 2^-53
 * in [0, 1): the velocity relaxes at the rate gamma_over_m and takes a
 * uniform kick on [-sqrt(dt), sqrt(dt)), and the position integrates it,
 * evaluated for both components as
 *   v <- a * v + (r - 0.5) * w        a = 1 - gamma_over_m * dt, w = 2 sqrt(dt)
 *   x <- x + v * dt
 * with a and w formed once per call and every operation one IEEE float64
 * operation (r - 0.5 is exact).
 * d_x, d_y, d_vx, d_vy: device float64 arrays of n entries (SoA), read and
 *   written in place; 8-byte aligned, not overlapping.
 * steps_per_launch: steps run per kernel launch with the particle kept in
 *   registers; 1 is the paper's one launch per step, 0 runs all steps in one
 *   launch.  Results are identical for every value.
 * Resuming from saved state with step0 = k continues the same run.
 * Errors: EINVAL (NULL or misaligned array, dt negative or not finite,
 *         gamma_over_m not finite), ERANGE (step0 + n_steps - 1 > 2^32 - 1, or
 *         pid0 + n - 1 overflows 64 bits).  n = 0 or n_steps = 0 does nothing.
 */
int orng_bd2(uint64_t pid0, uint32_t n, uint32_t step0, uint32_t n_steps, double dt,
             double gamma_over_m, double *d_x, double *d_y, double *d_vx, double *d_vy,
             uint32_t steps_per_launch, void *stream);

/*
 * orng_normal_pairs -- the library's Box-Muller transform applied to
 * caller-supplied 32-bit words: (z0[i], z1[i]) is the normal pair made from
 * (x0[i], x1[i]) exactly as F32_NORMAL samples 2m and 2m+1 are made from
 * words 2m and 2m+1 (u1 = ((x0 >> 8) + 1) 2^-24, u2 = (x1 >> 8) 2^-24,
 * z0 = R cos 2 pi u2, z1 = R sin 2 pi u2, R = sqrt(-2 ln u1)).
 * All four arrays are device buffers of n elements, 4-byte aligned.
 * Errors: EINVAL (NULL or misaligned pointer with n > 0), ERANGE (n > 2^40).
 */
int orng_normal_pairs(const uint32_t *d_x0, const uint32_t *d_x1, uint64_t n, float *d_z0,
                      float *d_z1, void *stream);

/*
 * Fill request: the arguments of one orng_fill, as a record.  56 bytes.
 *   out    : device buffer of n samples (caller-owned): n * 4 bytes, 4-byte
 *            aligned; n * 8 bytes, 8-byte aligned for the float64 distributions
 *   flags  : reserved, must be 0
 *   lo, hi : dist == ORNG_I32_RANGE only: the request is the single-stream
 *            orng_fill_range(gen, seed, ctr, 1, offset, n, lo, hi, out), so
 *            lo < hi, offsets and counts are in samples of two words (at
 *            most 2^31 per stream) and out holds n int32; ignored for every
 *            other distribution
 */
typedef struct {
    uint64_t seed;
    uint64_t offset;
    uint64_t n;
    void *out;
    uint32_t ctr;
    uint32_t gen;
    uint32_t dist;
    uint32_t flags;
    int32_t lo;
    int32_t hi;
} orng_req_t;

/*
 * orng_fill_batched -- every request r of h_reqs[0 .. nreq) is filled exactly
 * as orng_fill(r.gen, r.dist, r.seed, r.ctr, r.offset, r.n, r.out) would fill
 * it (orng_fill_range with r.lo, r.hi for ORNG_I32_RANGE; each sample depends
 * only on its own stream and position, section 3.1),
 * in one persistent launch that pulls fixed-size tiles of all requests from a
 * device work queue; the launch is replayed from a captured hipGraph.
 * h_reqs is host memory, copied before the call returns.  Output ranges of
 * different requests must not overlap.  Requests with n == 0 are skipped.
 * Errors: EINVAL / ERANGE as orng_fill (orng_fill_range for ORNG_I32_RANGE:
 *         EINVAL when lo >= hi) for the first bad request (nothing is
 *         enqueued then); ENOMEM if the batch needs more than 2^28 tiles or
 *         holds 2^32 or more requests.
 */
int orng_fill_batched(const orng_req_t *h_reqs, size_t nreq, void *stream);

/*
 * orng_fill_batched_noalloc -- orng_fill_batched for callers that cannot
 * allocate memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same results, the same generation kernels, and
 * no allocation of any kind by the call.  The batch's header, request table
 * (64 bytes per request, plus 8 for integer-range bounds) and tile map (4
 * bytes per tile) live in a fixed device array of the library (about 25 MiB,
 * held by every device the call runs on until the process ends), and the
 * rows are staged in a fixed host array.  Limits: at most ORNG_NOALLOC_MAX_REQUESTS requests and
 * ORNG_NOALLOC_MAX_TILES tiles (a tile is 2,048 to 65,536 words at the
 * built-in launch shapes; any request with work needs at least one).
 * Behaviour: the call returns after the request rows are uploaded, which
 * waits for work queued earlier on `stream`; the kernels then run on `stream`
 * without a captured graph.  Every call on a device shares that device's
 * array, which keeps the last call's contents: calls on one stream run one
 * after the other; calls that overlap on one device (other streams, other
 * host threads' streams) race and must not be made.
 * Errors: EINVAL / ERANGE as orng_fill_batched for the first bad request;
 *         ENOMEM if nreq > ORNG_NOALLOC_MAX_REQUESTS or the batch needs more
 *         than ORNG_NOALLOC_MAX_TILES tiles (nothing is enqueued then).
 */
enum { ORNG_NOALLOC_MAX_REQUESTS = 131072, ORNG_NOALLOC_MAX_TILES = 4194304 };
int orng_fill_batched_noalloc(const orng_req_t *h_reqs, size_t nreq, void *stream);

/*
 * orng_fill_each -- the plain path for the same request list: one fill launch
 * per request, in order (the baseline the batched and served paths are
 * compared with).  Same results and errors as orng_fill_batched.
 */
int orng_fill_each(const orng_req_t *h_reqs, size_t nreq, void *stream);

/*
 * orng_autotune -- time launch variants of the fill and batched kernels for
 * (gen, dist) on the current device (workgroup size, blocks of four words per
 * lane per tile, tiles per queue claim, persistent workgroups per CU), or with
 * dist = ORNG_TUNE_RANGE those of orng_fill_range for gen, and keep
 * the fastest (a first pass over all variants, then the fastest few and the
 * entry in use re-timed against each other in interleaved rounds); results
 * never change, only speed.  Allocates 4 GiB of device memory for the
 * duration of the call and synchronizes the device.
 * cache_path (nullable): text file that receives the table of tuned entries
 * (existing entries for other pairs are kept).  orng_tune_load reads such a
 * file; the library also reads $ORNG_TUNE_CACHE at first use.
 */
enum { ORNG_TUNE_RANGE = 5 };
int orng_autotune(int gen, int dist, const char *cache_path);
int orng_tune_load(const char *cache_path);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of fill requests (the request loop built on the
 * stream model of section 3.1).  A server owns one HIP stream on the device
 * that is current at orng_serve_create, an HBM arena for outputs it
 * allocates, and a table of device-resident slots holding the stream state of
 * every admitted request (seed, counter, position range, output).  Requests
 * are admitted in arrival order as slots and arena space free up; each device
 * step generates tiles of all admitted requests in one launch, and up to three
 * steps are in flight, so requests that arrive while others run join the next
 * step and their work overlaps on the device.  Results are bit-identical to
 * orng_fill of the same request, alone or in any mix.
 * Failures: if a step cannot be enqueued (an upload or launch error on the
 * host), the steps already queued are waited for and the requests they finish
 * end done; every other unfinished request ends with that error (its poll or
 * wait returns it, e.g. ORNG_EHIP), later submits return it, and
 * orng_serve_destroy returns it after freeing the server.  A device fault ends
 * every unfinished request at once.  For tests of this path, the environment
 * variable ORNG_SERVE_FAIL_STEP=k (read by orng_serve_create) makes the k-th
 * step of the server fail that way.
 * ------------------------------------------------------------------------- */
typedef struct orng_server orng_server_t;

typedef struct {
    void *arena;            /* device memory for server-allocated outputs; NULL: the
                               server allocates arena_bytes itself */
    uint64_t arena_bytes;   /* HBM budget for outputs in flight (> 0) */
    uint32_t max_slots;     /* requests resident on the device at once (0: 4096) */
    uint32_t flags;         /* reserved, 0 */
    uint64_t step_words;    /* most words generated per device step (0: automatic, 2^30;
                               at most 2^34) */
} orng_serve_cfg_t;

typedef struct {
    void *d_out;            /* device address of the result (arena or caller buffer) */
    uint64_t n;             /* samples */
    int64_t t_submit_ns;    /* CLOCK_MONOTONIC time of orng_serve_submit */
    int64_t t_admit_ns;     /* time the request got a slot (and arena space) */
    int64_t t_done_ns;      /* time the server observed its last tile complete */
    int32_t status;         /* ORNG_OK, or the error that ended the request */
    int32_t pad;
} orng_result_t;

typedef struct {
    uint64_t submitted, admitted, completed, released, failed;
    uint64_t samples_done;  /* samples of completed requests */
    uint64_t steps;         /* device launches */
    uint64_t arena_peak_bytes;
    uint32_t active_peak;   /* most requests resident at once */
    uint32_t queued;        /* waiting for admission now */
    double latency_p50_ms, latency_p99_ms, latency_mean_ms; /* submit -> done, nearest rank,
                                                                over the latest 2^20 completed */
    double first_submit_to_last_done_s;
} orng_serve_stats_t;

/* Create a server.  Errors: EINVAL (cfg: arena_bytes < 256, a misaligned arena,
   flags != 0, step_words > 2^34), EHIP (stream/arena allocation). */
int orng_serve_create(const orng_serve_cfg_t *cfg, orng_server_t **srv);
/* Queue a request; never blocks on the device.  req->out == NULL asks the
   server for an arena output (released by orng_serve_release); otherwise the
   caller's buffer is written.  The server writes from streams of its own,
   which do not wait for work queued on the caller's streams: a caller buffer
   must have no pending reads or writes on any stream when it is submitted
   (synchronize first).  Errors: EINVAL/ERANGE (as orng_fill), ENOMEM
   (output larger than the arena), EBUSY (server shutting down). */
int orng_serve_submit(orng_server_t *srv, const orng_req_t *req, uint64_t *ticket);
/* Non-blocking submit: the request is queued only if the server can admit it
   at once (no request waits ahead of it, a device slot is free and, when
   req->out == NULL, its arena range is free; the range is taken by this
   call).  Otherwise nothing is queued and ORNG_EAGAIN is returned.  Other
   errors as orng_serve_submit. */
int orng_serve_try_submit(orng_server_t *srv, const orng_req_t *req, uint64_t *ticket);
/* Queue n requests in one call (one arrival of many); tickets[i] receives the
   ticket of reqs[i].  All requests are validated first: on an error nothing is
   queued and the status is that of the first bad request. */
int orng_serve_submit_many(orng_server_t *srv, const orng_req_t *reqs, size_t n,
                           uint64_t *tickets);
/* Wait for each of tickets[0 .. n) in order and release it as soon as it is
   done (up to timeout_ns in total, < 0: forever).  *released (nullable) gets
   how many were released; EBUSY on timeout, ENOENT at an unknown ticket. */
int orng_serve_release_many(orng_server_t *srv, const uint64_t *tickets, size_t n,
                            int64_t timeout_ns, size_t *released);
/* ORNG_OK and *res when done, ORNG_EBUSY while queued or running, ENOENT for
   unknown or released tickets. */
int orng_serve_poll(orng_server_t *srv, uint64_t ticket, orng_result_t *res);
/* As poll, waiting up to timeout_ns (< 0: forever). */
int orng_serve_wait(orng_server_t *srv, uint64_t ticket, int64_t timeout_ns, orng_result_t *res);
/* Forget a finished ticket and return its arena range.  EBUSY if not finished. */
int orng_serve_release(orng_server_t *srv, uint64_t ticket);
/* Counters and latency percentiles (nearest rank over completed requests). */
int orng_serve_stats(orng_server_t *srv, orng_serve_stats_t *st);
/* Drain queued and in-flight work, then free the server (caller memory untouched). */
int orng_serve_destroy(orng_server_t *srv);

/* Launch knobs for the fill kernels (0 = automatic).  They change speed
   only, never results.  Process-wide; NULL restores the defaults. */
typedef struct {
    uint32_t wg_size;     /* threads per workgroup: 64..512, multiple of 64 */
    uint32_t unroll;      /* blocks of 4 words per lane per span: 1..64 */
    uint32_t max_wgs;     /* cap on the grid; larger work loops grid-stride */
    uint32_t nontemporal; /* 1 nontemporal stores, 2 ordinary stores */
} orng_launch_t;
int orng_set_launch(const orng_launch_t *cfg);
int orng_get_launch(orng_launch_t *cfg);

/* Text for a status code (static storage). */
const char *orng_strerror(int status);
/* HIP error code behind the last ORNG_EHIP on this thread (0 if none). */
int orng_last_hip_error(void);
/* Library version, e.g. 0x000100 for 0.1.0. */
int orng_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ORNG_H */
