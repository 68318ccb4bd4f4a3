/*
 * mtgp.h -- C ABI of the MTGP library for AMD Instinct MI355X (gfx950).
 *
 * MTGP (Saito & Matsumoto, "Variants of Mersenne Twister Suitable for Graphic
 * Processors") is an F2-linear generator whose state is N = ceil(p/32) 32-bit
 * words for a Mersenne exponent p (section 3.3); each new word is
 *     x_{N+i} = g(x_{M+i}, x_{1+i}, x_i)            (section 3.6, Definition
 *                                                      "recursion parameters")
 * and each output is tempered with x_{M-1+i}        (section 3.7, Definition
 *                                                      "tempering parameter").
 * Outputs are produced on the GPU by evaluating up to N-M mutually independent
 * steps of the recursion at once (section 3.2).
 *
 * Conventions for every call below:
 *   - Device pointers (`out`) are caller-owned device memory (e.g. a torch
 *     tensor's data pointer) of at least 4*n bytes, 4-byte aligned.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Generation calls are asynchronous and stream-ordered; calls on one
 *     handle must be issued in order on one stream, or the caller must
 *     synchronise when switching streams. Handles are not thread-safe;
 *     distinct handles are independent.
 *   - Output k of a fresh generator is o_{N+k}: the N seed words are never
 *     emitted. All output kinds share one position counter: k outputs of any
 *     kind advance the stream by k steps, and the float outputs at position k
 *     are derived from the uint32 output at position k (section 6).
 *   - Any n >= 0 is allowed; n = 0 is a successful no-op. Consecutive calls
 *     continue the stream exactly (section 8): gen(a) then gen(b) equals the
 *     first a+b outputs of gen(a+b).
 *   - Return codes: MTGP_OK, or a negative MTGP_E* code. mtgp_last_error()
 *     holds the code of the last failing call on the calling thread.
 *     MTGP_EDEVICE reports a HIP error met while the call set up or enqueued
 *     its work: streams whose work was not enqueued keep their position (a
 *     plain batch call, one launch per request, may have enqueued and
 *     advanced its earlier requests). States are updated
 *     in place by the kernels, so an error raised later by the device (a
 *     fault reported at a following synchronisation) can leave them partly
 *     written; such a generator should be re-seeded or restored with
 *     set_state before further use.
 */
#ifndef MTGP_H
#define MTGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MTGP_OK        0
#define MTGP_EINVAL   (-1)   /* bad parameter set, bad argument or alignment */
#define MTGP_ENOMEM   (-2)   /* host or device allocation failed */
#define MTGP_EDEVICE  (-3)   /* HIP error while setting up or enqueueing; position unchanged */
#define MTGP_ENOTFOUND (-4)  /* parameter search: no set within max_draws */

/* Output kinds (section 6). */
#define MTGP_KIND_UINT32        0   /* tempered 32-bit word o_{N+k} */
#define MTGP_KIND_FLOAT32_1TO2  1   /* bits 0x3f800000 | (o >> 9): float in [1,2) */
#define MTGP_KIND_FLOAT32_0TO1  2   /* the [1,2) value minus 1.0f: float in [0,1) */
/* Gaussian float32 by the Box-Muller transform of float [1,2) outputs, which
 * section 6 names as a direct use of that range: for the pair (a, b) of
 * [1,2) values at positions 2j, 2j+1 counted from the start of the call or
 * request, r = sqrt(-2 ln(2 - a)); output 2j = r cos(2 pi (b - 1)) and
 * output 2j+1 = r sin(2 pi (b - 1)). n outputs consume n steps. Requires an
 * even n and N - M >= 2 (MTGP_EINVAL otherwise). Computed in binary32 with
 * the hardware approximations v_log_f32, v_sqrt_f32 and v_sin_f32 (each
 * checked exhaustively over its 2^23 inputs here on gfx950): the result is
 * within about 1.5e-6 absolute of the exact transform of the same a and b
 * (an absolute bound, not a few ulp: near z = 0 it is many ulp), and the
 * tests accept 1.5e-5 absolute. Not bit-exact against a reference. */
#define MTGP_KIND_NORMAL_FLOAT32 3

/*
 * Parameter set (section 3.6 and 3.7). Copied at create time; the caller
 * keeps ownership.
 *   mexp       Mersenne exponent p; N = ceil(p/32), r = 32N - p. Accepted:
 *              65 <= p <= 65536 (3 <= N <= 2048). The released periods are
 *              p = 11213, 23209, 44497 (N = 351, 726, 1391).
 *   pos        middle position M, 2 <= M <= N-1 (section 3.1 requires 1<M<N;
 *              M >= 2 keeps the tempering word x_{M-1+i} a full state word).
 *   sh1, sh2   shift amounts, 0..31.
 *   param_tbl  recursion table: entry v is (v as a 4-bit row vector) * R for
 *              the 4x32 matrix R. Must be F2-linear: tbl[0] = 0 and
 *              tbl[a ^ b] = tbl[a] ^ tbl[b].
 *   temper_tbl tempering table, entry v = (v as a 4-bit row vector) * T; same
 *              linearity rule.
 */
typedef struct mtgp_param_set {
    uint32_t mexp;
    uint32_t pos;
    uint32_t sh1;
    uint32_t sh2;
    uint32_t param_tbl[16];
    uint32_t temper_tbl[16];
} mtgp_param_set;

typedef struct mtgp mtgp_t;               /* one generator; owns its device state */
typedef struct mtgp_batch mtgp_batch_t;   /* many generators; states resident in one device array */

/* Number of state words N for a Mersenne exponent (0 if outside 65..65536). */
uint32_t mtgp_state_words(uint32_t mexp);

/*
 * Create a generator on the current HIP device. The state x_0..x_{N-1} is
 * seeded on the host (the paper leaves seeding open; the MT19937
 * initialisation recurrence x_0 = seed, x_i = 1812433253 (x_{i-1} ^
 * (x_{i-1} >> 30)) + i is used) and copied to device memory owned by the
 * handle. Returns NULL on error (see mtgp_last_error()).
 */
mtgp_t *mtgp_create(const mtgp_param_set *ps, uint32_t seed);

/*
 * Generate n outputs into device memory `out` on `stream` (section 8: load
 * the state, run rounds of the recursion, store outputs, store the state
 * back). One kernel launch with one workgroup.
 */
int mtgp_generate_uint32(mtgp_t *g, size_t n, uint32_t *out, void *stream);
int mtgp_generate_float32_1to2(mtgp_t *g, size_t n, float *out, void *stream);
int mtgp_generate_float32_0to1(mtgp_t *g, size_t n, float *out, void *stream);
int mtgp_generate_normal_float32(mtgp_t *g, size_t n, float *out, void *stream);   /* n even */

/*
 * Jump-ahead for this generator's calls (section 7 discusses jumping ahead):
 * with max_rounds > 0, a call that needs more than max_rounds rounds runs as
 * S segments that generate concurrently -- segment k starts from F^{kJ} S,
 * computed on the device from the current state's raw words and
 * h_k = x^{kJ} mod psi (psi annihilates the state's orbit, found on the host
 * with Berlekamp-Massey on the first split call, and again after
 * mtgp_set_state). The jump polynomials and device buffers are kept for the
 * last segment length, so repeated calls of one length pay only the
 * kernels. Outputs are identical to the unsplit stream. The first split call
 * synchronises `stream` once (to read the raw words back). 0 (default)
 * disables.
 */
int mtgp_set_split(mtgp_t *g, uint32_t max_rounds);

/* Release the handle (NULL-safe); waits for work queued on its last stream. */
void mtgp_destroy(mtgp_t *g);

/*
 * Checkpoint / restore. get_state waits for the last stream used, then copies
 * the N state words x_c..x_{c+N-1} (sequence order) to host memory and the
 * number c of outputs produced so far to *consumed (may be NULL).
 * set_state installs N words (any values; the r low bits of word 0 are
 * ignored by the recursion) and a position counter.
 */
int mtgp_get_state(mtgp_t *g, uint32_t *host_words, uint64_t *consumed);
int mtgp_set_state(mtgp_t *g, const uint32_t *host_words, uint64_t consumed);

/* ---------------------------------------------------------------------------
 * Batches: many independent generators (section 4.3 runs one block per
 * generator with distinct parameter sets; here one persistent launch serves
 * a list of requests of uneven length, ordered longest first).
 * ------------------------------------------------------------------------- */

/* One request: `n` outputs of `kind` from generator `gen` into device `out`. */
typedef struct mtgp_request {
    uint32_t gen;
    uint32_t kind;
    uint64_t n;
    void *out;
} mtgp_request;

/*
 * Create `count` generators from ps[0..count-1] (each validated as for
 * mtgp_create) seeded with seeds[0..count-1]. All states live in one device
 * array that stays resident until mtgp_batch_destroy.
 */
mtgp_batch_t *mtgp_batch_create(const mtgp_param_set *ps, const uint32_t *seeds, uint32_t count);

/*
 * Serve `nreq` requests in one persistent kernel launch on `stream`. A
 * generator may appear at most once per call (requests for one generator
 * must be split across calls, which run in stream order). Requests with
 * n = 0 are skipped. With a split limit set (mtgp_batch_set_split) and a
 * request longer than it, the call runs as a one-off plan of jump-ahead
 * segments: it then waits for the batch's last stream (and, the first time
 * for a generator, reads its raw words back to find the annihilator) before
 * the launch is enqueued; the plan is kept until the next such call or
 * mtgp_batch_destroy. Returns MTGP_EINVAL for a bad generator index, kind,
 * duplicate generator or misaligned output.
 */
int mtgp_batch_generate(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream);

/*
 * For callers that cannot allocate -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation: the same call as
 * mtgp_batch_generate without jump-ahead segments (a split limit is
 * ignored), making no device or host allocation. Its work items (at most
 * MTGP_STATIC_MAX_ITEMS requests with n > 0) and queue counters live in a
 * fixed array of MTGP_STATIC_SCRATCH_BYTES in this library's device code, one
 * copy per GPU held until the process ends; the batch's pinned staging for
 * the items is made by mtgp_batch_create. Every call on one GPU uses that
 * GPU's copy, so calls that overlap on a GPU (other streams, other batches,
 * other threads) race and must be serialised by the caller; calls on one
 * stream are ordered. A call waits on the host until the previous such
 * call of this batch has uploaded its items. Returns MTGP_EINVAL for
 * nreq > MTGP_STATIC_MAX_ITEMS and as mtgp_batch_generate does, and
 * MTGP_EDEVICE on a HIP error.
 */
#define MTGP_STATIC_MAX_ITEMS 4096
#define MTGP_STATIC_SCRATCH_BYTES (256 + 32 * MTGP_STATIC_MAX_ITEMS)
int mtgp_batch_generate_static(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream);

/*
 * Same work as mtgp_batch_generate, but as one launch per request on
 * `stream` (the plain form, for comparison).
 */
int mtgp_batch_generate_plain(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream);

int mtgp_batch_get_state(mtgp_batch_t *b, uint32_t gen, uint32_t *host_words, uint64_t *consumed);
int mtgp_batch_set_state(mtgp_batch_t *b, uint32_t gen, const uint32_t *host_words, uint64_t consumed);
uint32_t mtgp_batch_size(const mtgp_batch_t *b);
void mtgp_batch_destroy(mtgp_batch_t *b);

/* ---------------------------------------------------------------------------
 * Plans: a fixed request list for repeated replay. Creation validates the
 * requests, orders them longest critical path first, uploads the list once
 * and captures the persistent launch into a HIP graph. Each mtgp_plan_launch
 * continues every listed generator by its request's n outputs, written to
 * the same output buffers. The batch must outlive its plans; plan launches
 * and other calls on the same batch must be stream-ordered. Returns NULL on
 * error (see mtgp_last_error()).
 * ------------------------------------------------------------------------- */
typedef struct mtgp_plan mtgp_plan_t;

/*
 * Jump-ahead for plans (the paper's section 7 discusses jumping ahead).
 * With max_rounds > 0, mtgp_batch_plan_create (and mtgp_batch_generate, as a
 * one-off plan) splits every request whose
 * generator would need more than max_rounds rounds into S segments of J
 * outputs that run concurrently: segment k starts from the state F^{kJ} S,
 * computed on the GPU at each launch as the XOR of the states S, F S, ...
 * selected by h_k = x^{kJ} mod psi, where psi annihilates the generator's
 * orbit (found once per generator on the host from the minimal polynomials of
 * the bit planes of its raw words -- Berlekamp-Massey, section 5 -- and
 * verified on every state word). Outputs are identical to the unsplit
 * stream. A generator for which no annihilator is found is not split.
 * mtgp_batch_set_state on a split generator makes existing plans stale
 * (mtgp_plan_launch then returns MTGP_EINVAL). 0 (the default) disables it.
 */
int mtgp_batch_set_split(mtgp_batch_t *b, uint32_t max_rounds);
mtgp_plan_t *mtgp_batch_plan_create(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq);
int mtgp_plan_launch(mtgp_plan_t *p, void *stream);

/*
 * One phase of a plan launch, for callers that time or overlap the phases.
 * MTGP_PHASE_PREPARE computes the start states of the segments (the raw
 * prefix and jump kernels; nothing for a plan without segments);
 * MTGP_PHASE_GENERATE runs the persistent generation and advances the
 * generators. A replay is PREPARE then GENERATE, stream-ordered, each once;
 * MTGP_PHASE_ALL (what mtgp_plan_launch does) is both in one graph launch.
 * Returns MTGP_EINVAL for an unknown phase or a stale plan.
 */
#define MTGP_PHASE_ALL 0
#define MTGP_PHASE_PREPARE 1
#define MTGP_PHASE_GENERATE 2
int mtgp_plan_launch_phase(mtgp_plan_t *p, int phase, void *stream);
void mtgp_plan_destroy(mtgp_plan_t *p);   /* NULL-safe; waits for the batch's last stream */

/*
 * What a plan launches (for callers that report or profile it): the launch
 * shape its generation kernel was resolved to (mode as in
 * mtgp_batch_set_launch, never -1; for the chunked form spl is the
 * read-ahead depth and lds_words the ring length), its work items
 * (requests and segments), and of these the segments whose start state a
 * jump computes. Host only. MTGP_EINVAL for NULL arguments.
 */
typedef struct {
    int32_t mode;
    uint32_t threads;
    uint32_t spl;
    uint32_t lds_words;
    uint32_t grid;       /* workgroups of the generation launch */
    uint32_t items;      /* work items of the generation launch */
    uint32_t jumps;      /* segments started from a jump */
} mtgp_plan_info;
int mtgp_plan_describe(const mtgp_plan_t *p, mtgp_plan_info *info);

/*
 * The generation launch's work items in queue order: output device address
 * and output count of item i in outs[i] and ns[i], for the first
 * min(cap, items) items. Returns that count, or MTGP_EINVAL for NULL
 * arguments. Host only.
 */
int mtgp_plan_items(const mtgp_plan_t *p, uint64_t *outs, uint64_t *ns, uint32_t cap);

/*
 * Autotuner for a request list (unique generators, as for plans). Times `reps`
 * plan launches on `stream` for each candidate configuration -- the automatic
 * launch shape with no split, with the split limits of one unit's fair share
 * (all rounds of the request list over the automatic launch's wavefronts or
 * workgroups) and three quarters of it, and with split limits halving from
 * the longest request's round count down to 128 rounds (rounds of the
 * automatic shape; seven halvings, then more only while each one is the
 * fastest so far),
 * then the chunked form (mode 2) with 64/256/1024 lanes per workgroup and
 * read-ahead 2 (and 256 lanes with read-ahead 1), workgroup forms of
 * 128/256/512/1024 lanes with 1-4 steps per lane and the wavefront form, each
 * at the split limit that cuts the same segment lengths as the best one so
 * far (split limits count rounds of the shape in use) and at half of it,
 * then the best of these with the other recursion-table
 * form (MTGP_MODE_REC_BASIS), then the best so far with its split limit
 * times 1.3 and divided by 1.3 -- and keeps the fastest (a later candidate must be at least
 * 2 % faster than the one it replaces) as the batch's launch shape
 * (mtgp_batch_set_launch) and split limit (mtgp_batch_set_split). Outputs are
 * identical under every configuration; the generators' states and counters
 * are restored after each trial, so the call leaves the streams where they
 * were. The request outputs are overwritten. The result is written to *best
 * if non-NULL: mode -1 (threads, spl 0) means the automatic shape. Returns
 * MTGP_EINVAL for bad requests or reps == 0, MTGP_ENOMEM, or MTGP_EDEVICE (the
 * previous settings are then kept).
 */
typedef struct {
    int mode, threads, spl;   /* chosen shape; mode -1: the automatic shape (mode may carry MTGP_MODE_REC_BASIS) */
    uint32_t split_rounds;    /* chosen split limit (0: no split) */
    float ms;                 /* its mean plan launch time */
    uint32_t trials;          /* configurations timed */
} mtgp_tuning;
int mtgp_batch_autotune(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream, uint32_t reps,
                        mtgp_tuning *best);

/* ---------------------------------------------------------------------------
 * Launch shape (for tuning; results are identical for every valid shape).
 *   mode 0: one workgroup of `threads` lanes per generator, a barrier between
 *           rounds; steps per lane per round up to `spl` (1, 2 or 4).
 *   mode 1: one wavefront per generator, `threads`/64 wavefronts per
 *           workgroup, no barriers; spl up to 1, 2, 4, 6, 8, 12 or 16.
 *   mode 2: chunked form: one wavefront per generator, `threads`/64
 *           wavefronts per workgroup, no barriers. Each wavefront takes the
 *           steps 64 at a time (one per lane) and keeps three such chunks in
 *           flight: the LDS reads of chunk q + spl + 1, the recursion of
 *           chunk q + 1 up to its table lookups, and the write-back and
 *           output of chunk q; spl (1 or 2) is the read-ahead in chunks and
 *           needs N - M >= 64 (spl + 2) for every generator served (the
 *           steps of a chunk then never depend on the two chunks before it,
 *           section 3.2). The state lives in an LDS ring of lds_words words
 *           (a power of two from 512 to 4096, at least N + 64; 0 = automatic),
 *           each word stored twice so that no read wraps. This is the
 *           automatic shape of a batch call with at least 8 requests (or
 *           jump-ahead segments) per compute unit whose generators all
 *           allow it (read-ahead 2 when all allow it); with fewer, the
 *           workgroup form gives each request more lanes.
 *   mode | MTGP_MODE_REC_BASIS: the recursion table rec[u & 0xf] is evaluated
 *           from its four F2 basis words in registers instead of read from
 *           LDS: more vector instructions per step, but no lookup on the
 *           chain of a round. Which form is faster depends on the workload;
 *           the autotuner tries both. (Modes 0 and 1; the chunked form
 *           always looks the table up.)
 * In modes 0 and 1 each generator uses the largest supported s <= spl with
 * lanes*s <= N - M (lanes = threads in mode 0, 64 in mode 1), so a round
 * computes W = min(N - M, lanes*s) steps (section 3.2); in mode 2 a round is
 * one chunk of 64 steps (split limits count chunks). lds_words is the LDS
 * window per generator (0 = automatic; must be >= 2N + lanes*s for every
 * generator served) and grid the number of workgroups (0 = automatic). mode < 0
 * restores the automatic choice. Returns MTGP_EINVAL for an unsupported
 * shape; a batch call whose requests do not fit the shape fails with
 * MTGP_EINVAL.
 * ------------------------------------------------------------------------- */
#define MTGP_MODE_REC_BASIS 4
int mtgp_batch_set_launch(mtgp_batch_t *b, int mode, int threads, int spl, int lds_words, int grid);
int mtgp_set_launch(mtgp_t *g, int mode, int threads, int spl, int lds_words);

/* Code of the last failing call on this thread, and a message for a code. */
int mtgp_last_error(void);
const char *mtgp_strerror(int code);

/* ---------------------------------------------------------------------------
 * Parameter search (section 5, MTGPDC's recursion-parameter search), on the
 * host; no device is used. Draws candidates (M, R) with sh1 = 13, sh2 = 4
 * (fixed as in section 5), M in 2 < M < N - floor2(N) (2 <= M <= N-1 when that
 * range is empty), the 32-bit `id` embedded in R -- its 16 MSBs in the 16
 * MSBs of the first row, its 16 LSBs in bits 19..4 of the second row (the
 * paper's "12th .. 28th MSB" names 17 positions for 16 bits; the 16 just
 * above the four LSBs are taken) -- the four LSBs of the rows drawn until
 * I + R44 is invertible, the remaining bits random. A candidate is accepted
 * when the minimal polynomial (Berlekamp-Massey) of bit 31 of its raw words
 * has degree mexp and is irreducible (no factor of degree <= 256, and
 * x^(2^mexp) = x modulo it): for a Mersenne exponent mexp that means period
 * 2^mexp - 1. The tempering table is a random F2-linear table (its
 * equidistribution search needs SIS and is not done). Candidate i uses a
 * random stream derived from (seed, id, i); the lowest accepted index wins,
 * so the result does not depend on `threads` (0 = the CPUs in the calling
 * process's affinity mask, at most 16).
 * Arguments: mexp prime in 67..65536 (a Mersenne exponent for the period
 * claim), max_draws > 0, out non-NULL; stats may be NULL. Returns MTGP_OK,
 * MTGP_EINVAL, or MTGP_ENOTFOUND when max_draws candidates fail.
 * ------------------------------------------------------------------------- */
typedef struct {
    uint64_t draws;          /* index of the accepted candidate + 1 (max_draws if none) */
    uint64_t evaluated;      /* candidates evaluated by all threads */
    uint64_t full_degree;    /* of those, linear complexity mexp */
    uint64_t sieve_passed;   /* of those, no factor of degree <= 256 */
    double seconds;          /* wall time */
} mtgp_search_stats;
int mtgp_search_params(uint32_t mexp, uint32_t id, uint64_t seed, uint64_t max_draws, uint32_t threads,
                       mtgp_param_set *out, mtgp_search_stats *stats);

/* ---------------------------------------------------------------------------
 * Dimension of equidistribution (section 3.4): k[v-1] = k(v) for v = 1 ..
 * vmax, the largest k such that the v MSBs of k consecutive outputs are
 * k-dimensionally equidistributed over the period, and *delta (may be NULL)
 * = sum over v <= vmax of floor(p/v) - k(v), the total dimension defect
 * (vmax = 32 gives the paper's Delta). `tempered` selects the uint32
 * outputs (the float [1,2) and [0,1) outputs carry their 23 MSBs, so k(v)
 * for v <= 23 is theirs too); 0 selects the untempered words x_{i+N}.
 * Computed on the host by lattice reduction over F2[t] (the dual form of
 * the lattice methods section 5 uses); no device is used. The definition
 * needs period 2^p - 1: the set must pass the library's checks, mexp must be
 * a prime in 67..65536 and the characteristic polynomial irreducible of
 * degree mexp (what mtgp_search_params returns), else MTGP_EINVAL.
 * Arguments: ps and k non-NULL (k holds vmax words), 1 <= vmax <= 32.
 * Returns MTGP_OK, MTGP_EINVAL or MTGP_ENOMEM. The time grows about as
 * vmax^2 mexp^2.
 * ------------------------------------------------------------------------- */
int mtgp_equidistribution(const mtgp_param_set *ps, uint32_t tempered, uint32_t vmax, uint32_t *k,
                          uint32_t *delta);

/* ---------------------------------------------------------------------------
 * Serving: a continuous-batching request loop over a batch's resident
 * generators, for callers that receive stream requests over time. Requests
 * are admitted in arrival order while their outputs (4n bytes, 256-byte
 * aligned) fit a caller-owned device arena (first fit; a request that does
 * not fit waits, and so do the ones behind it). Each mtgp_server_poll
 * retires ticks whose completion event has fired, admits what fits, and
 * launches ticks on `stream` while fewer than `depth` are in flight. A tick
 * advances every generator with admitted work by up to `chunk` outputs of
 * its oldest unfinished request, in one batched launch; requests of one
 * generator are served in arrival order, so each result is exactly the
 * stream segment it would get alone. A completed request's outputs stay in
 * the arena until mtgp_server_release. The batch and the arena must outlive
 * the server; other calls on the batch must not run concurrently with it.
 * Not thread-safe. Create returns NULL for a NULL batch or arena, an arena
 * below 256 bytes or not 256-byte aligned, chunk 0 or depth 0 (chunk is
 * rounded down to even).
 * ------------------------------------------------------------------------- */
typedef struct mtgp_server mtgp_server_t;
typedef struct {
    uint64_t rid;      /* the id given at submit */
    uint64_t offset;   /* byte offset of its n outputs in the arena */
    uint64_t n;
} mtgp_completion;
mtgp_server_t *mtgp_server_create(mtgp_batch_t *b, void *arena, uint64_t arena_bytes, uint64_t chunk,
                                  uint32_t depth, void *stream);
typedef struct {
    uint64_t rid;      /* caller's id; ids of unreleased requests must be distinct */
    uint32_t gen;
    uint32_t kind;
    uint64_t n;
} mtgp_server_request;
/* Queue `count` requests in arrival order. All-or-nothing: MTGP_EINVAL if
 * any has a bad generator or kind, n = 0, an odd n for normals, or outputs
 * larger than the arena. */
int mtgp_server_submit(mtgp_server_t *s, const mtgp_server_request *reqs, uint32_t count);
/* One scheduling step; writes up to max_done completions (oldest first; the
 * rest are returned by later polls) and their count. MTGP_EDEVICE on a HIP
 * error. */
int mtgp_server_poll(mtgp_server_t *s, mtgp_completion *done, uint32_t max_done, uint32_t *n_done);
/* Return completed requests' arena space; ids that are unknown or not yet
 * finished are skipped and make the call return MTGP_EINVAL. */
int mtgp_server_release(mtgp_server_t *s, const uint64_t *rids, uint32_t count);
int mtgp_server_pending(const mtgp_server_t *s, uint64_t *waiting, uint64_t *active, uint32_t *inflight);
void mtgp_server_destroy(mtgp_server_t *s);   /* NULL-safe; waits for in-flight ticks */

/*
 * Jump-ahead inside the request loop (the paper's section 7 discusses jumping
 * ahead). With min_outputs > 0, a request with at least min_outputs
 * outputs left, on a generator whose orbit annihilator is cached
 * (mtgp_batch_prepare_split), is split into up to max_segments segments of
 * seg_chunks * chunk outputs (the last one shorter) that advance together,
 * one chunk each per tick, instead of one chunk per tick in all: segment k
 * starts from the state F^{kJ} S of the request's current position S,
 * computed on the device in the tick that splits it (raw prefix and jump
 * kernels, as for split plans). The jump polynomials x^{kJ} mod psi are
 * computed by host worker threads; the request keeps advancing by plain
 * chunks until they are ready. Outputs are identical to the unsplit stream.
 * At most `slots` requests are split at a time (device state buffers of
 * slots * max_segments * N words). Call before the first poll; min_outputs 0
 * (the default) turns splitting off. MTGP_EINVAL for max_segments < 2 or
 * > 64, seg_chunks or slots 0 with min_outputs > 0; MTGP_ENOMEM.
 * Currently disabled: any min_outputs > 0 returns MTGP_EINVAL (its first
 * device run stopped answering; the tick logic is kept and checked on the
 * host only until the cause is found).
 */
int mtgp_server_set_split(mtgp_server_t *s, uint64_t min_outputs, uint32_t max_segments, uint32_t seg_chunks,
                          uint32_t slots);

/*
 * Find and cache the orbit annihilators that jump-ahead needs (what a split
 * plan computes on first use) for `count` generators: raw words on the
 * device from the current states (states and counters unchanged), then
 * Berlekamp-Massey on the host, threaded. Synchronous; generators already
 * prepared are skipped; mtgp_batch_set_state drops a generator's entry.
 * MTGP_EINVAL for a bad index or NULL gens with count > 0, MTGP_ENOMEM,
 * MTGP_EDEVICE.
 */
int mtgp_batch_prepare_split(mtgp_batch_t *b, const uint32_t *gens, uint32_t count);

#ifdef __cplusplus
}
#endif

#endif /* MTGP_H */
