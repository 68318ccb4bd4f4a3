// Internal records shared by the MTGP host library and its gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mtgp_impl {

// Per-generator parameters as the kernels read them (one 256-byte record,
// so a workgroup fetches it with a few scalar loads).
struct alignas(256) GenRecord {
    uint32_t N;          // state words, ceil(p / 32)
    uint32_t M;          // middle position
    uint32_t sh1, sh2;   // shifts of the recursion
    uint32_t mask;       // 32-r MSBs set (r = 32N - p)
    uint32_t pad0[3];
    uint64_t state_off;  // word offset of this generator's state in the state array
    uint64_t pad1;
    uint32_t rec[16];    // recursion table (u & 0xf) -> (u^4) R
    uint32_t tmp[16];    // tempering table (t & 0xf) -> (t^4) T
    uint32_t flt[16];    // tempering table for float output: 0x3f800000 | (tmp >> 9)
};
static_assert(sizeof(GenRecord) == 256, "GenRecord layout");

// Output kinds of a work item (low byte of WorkItem::kind).
constexpr uint16_t kKindU32 = 0;     // tempered uint32
constexpr uint16_t kKindF12 = 1;     // float [1,2)
constexpr uint16_t kKindF01 = 2;     // float [0,1)
constexpr uint16_t kKindNormal = 3;  // Gaussian float by Box-Muller on pairs of float [1,2) outputs
constexpr uint16_t kKindRaw = 4;     // untempered words: the N start words, then x_{c+N}, x_{c+N+1}, ...
constexpr uint16_t kKeepState = 0x100;   // flag: do not write the end state back to the generator
constexpr uint16_t kStateToSrc = 0x200;  // flag: write the end state back to src (a segment's own state
                                         // buffer), not to the generator

// One unit of work: n outputs of `kind` from generator `gen` into `out`,
// starting from the generator's resident state, or from `src` if non-zero.
struct alignas(32) WorkItem {
    uint64_t out;        // device address of the first output word
    uint64_t n;          // outputs to produce
    uint32_t gen;        // index into the GenRecord array
    uint16_t kind;       // kind in the low byte, kKeepState / kStateToSrc flags
    uint16_t spl;        // steps per lane per round for this item
    uint64_t src;        // device address of N start words, or 0 for the generator's state
};

// One jump: out[w] = XOR over the set bits i of h (D bits) of raw[i + w], for
// w < N. raw holds D + N - 1 consecutive words of a stream starting at the
// state to jump from. h is laid out for the kernel's geometry (JumpShape): in
// blocks of R bits, block k = bits [kR, kR + R) of h in the low bits of a
// 16-bit field, four blocks per 64-bit word (block k in bits 16 (k % 4) of
// word k / 4), ceil(D / 4R) words.
struct alignas(32) JumpItem {
    uint64_t raw;
    uint64_t poly;
    uint64_t out;
    uint32_t D;
    uint32_t N;
};
static_assert(sizeof(JumpItem) == 32, "JumpItem layout");

// Geometry of the jump kernel for a state of N words: a lane owns R
// consecutive words (6 <= R <= 16), a wavefront covers 64 R words, G
// wavefronts cover the N words and P wavefronts of each word group split the
// bits of h (P = 4 / G here, the least a launch uses; launch_jumps may double
// it). raw is staged through LDS CI iterations of 4R bits at a
// time. Per bit of h a wavefront does about R / 2 XORs and one cross-lane move
// per lane, so R is chosen for the least G (R + 2), then for all four
// wavefronts busy, then the smaller R.
struct JumpShape {
    uint32_t R, G, P, CI;
};
constexpr uint32_t kJumpStageBits = 8192;   // raw words per LDS stage, at most
constexpr uint32_t kJumpMinR = 6, kJumpMaxR = 16;

__host__ __device__ inline JumpShape jump_shape(uint32_t N)
{
    JumpShape best = {0, 0, 0, 0};
    uint32_t best_cost = 0;
    for (uint32_t R = kJumpMinR; R <= kJumpMaxR; R++) {
        const uint32_t G = (N + 64 * R - 1) / (64 * R);
        if (G > 4)
            continue;
        const uint32_t cost = G * (R + 2);
        const bool better = best.R == 0 || cost < best_cost ||
                            (cost == best_cost && (4 / G) * G > best.P * best.G);
        if (better) {
            best = {R, G, 4 / G, kJumpStageBits / (4 * R)};
            best_cost = cost;
        }
    }
    return best;
}

// 64-bit words of h in the jump kernel's layout for a D-bit h.
__host__ __device__ inline uint32_t jump_poly_words(uint32_t N, uint32_t D)
{
    const uint32_t step = 4 * jump_shape(N).R;
    return (D + step - 1) / step;
}

// LDS words the jump kernel uses for a state of N words: a stage of raw words,
// the N - 1 words past it rounded up to the word groups plus the window
// read-ahead, then CI 64-bit words of h.
__host__ __device__ inline uint32_t jump_lds_words(uint32_t N)
{
    const JumpShape s = jump_shape(N);
    const uint32_t raw = 4 * s.R * s.CI + s.G * 64 * s.R + 6 * s.R;
    return (raw + 1) / 2 * 2 + 2 * s.CI;
}

static_assert(sizeof(WorkItem) == 32, "WorkItem layout");

// Launch shape of the generation kernels.
constexpr int kModeGroup = 0;   // one workgroup per generator, a barrier per round
constexpr int kModeWave = 1;    // one wavefront per generator, no barriers
constexpr int kModeChunk = 2;   // one wavefront per generator, 64-step chunks pipelined three deep
constexpr int kModeRecBasis = 4; // flag in the public mode value: LaunchShape::rec_basis

// The chunked form issues the LDS reads of a chunk of 64 steps `depth`
// (1 or 2) iterations before it computes it, and computes it one iteration
// before finishing it: chunk q + depth + 1 must depend only on chunks up to
// q - 1, i.e. N - M >= 64 (depth + 2).
inline uint32_t chunk_min_gap(uint32_t depth) { return 64u * (depth + 2u); }

// Ring length of the chunked form for a state of N words: the least power of
// two L >= max(512, N + 64) (the ring holds the N live words plus a chunk;
// 512 keeps every block of eight chunks inside one turn of the ring).
__host__ __device__ inline uint32_t chunk_ring_words(uint32_t N)
{
    uint32_t L = 512;
    while (L < N + 64)
        L *= 2;
    return L;
}

struct LaunchShape {
    int mode;        // kModeGroup, kModeWave or kModeChunk
    int threads;     // workgroup size (multiple of 64, <= 1024)
    int spl;         // largest steps per lane per round an item may use
                     // (group: 1, 2, 4; wave: 1, 2, 4, 6, 8, 12, 16); chunk form: the
                     // read-ahead depth in chunks (1 or 2)
    int lds_words;   // group and wave forms: LDS window length in words per generator
                     // (>= 2N + lanes*spl of every item); chunk form: ring length L
                     // (a power of two >= chunk_ring_words(N) of every item)
    int grid;        // workgroups
    int rec_basis = 0;  // 1: recursion table from its F2 basis in registers, 0: LDS lookup
                        // (group and wave forms; the chunked form always looks it up)
};

inline uint32_t shape_lanes(const LaunchShape &s) { return s.mode == kModeGroup ? (uint32_t)s.threads : 64u; }

// Steps per lane per round for a generator under a launch shape: the largest
// supported value s <= shape.spl with lanes*s <= N - M (every slot of a round
// useful), or 1 when even one slot per lane exceeds N - M. The chunked form
// takes one step per lane per chunk (its "round" is a chunk of 64 steps).
inline uint16_t item_spl(uint32_t N, uint32_t M, const LaunchShape &s)
{
    if (s.mode == kModeChunk)
        return 1;
    static const uint16_t group_spl[] = {4, 2, 1};
    static const uint16_t wave_spl[] = {16, 12, 8, 6, 4, 2, 1};
    const uint16_t *cand = s.mode == kModeGroup ? group_spl : wave_spl;
    const int ncand = s.mode == kModeGroup ? 3 : 7;
    const uint32_t lanes = shape_lanes(s);
    for (int i = 0; i < ncand; i++)
        if (cand[i] <= s.spl && lanes * cand[i] <= N - M)
            return cand[i];
    return 1;
}

// W of a generator under a launch shape: min(N - M, lanes * item_spl); 64
// (one chunk) in the chunked form.
inline uint32_t round_width(uint32_t N, uint32_t M, const LaunchShape &s)
{
    if (s.mode == kModeChunk)
        return 64u;
    const uint32_t w = N - M;
    const uint32_t cap = shape_lanes(s) * item_spl(N, M, s);
    return w < cap ? w : cap;
}

// Step slots a round writes: lanes * item_spl. Every slot writes its word
// (slots beyond W write words that the next round overwrites), so the LDS
// window must hold 2N + this many words.
inline uint32_t round_span(uint32_t N, uint32_t M, const LaunchShape &s)
{
    return shape_lanes(s) * item_spl(N, M, s);
}

// Queue counters of the persistent form: [0] next item, [1] units done.
// The last unit to finish resets both, so a launch needs no memset.
hipError_t launch_generate(const GenRecord *recs, uint32_t *states, const WorkItem *items,
                           uint32_t nitems, uint32_t *counters, const WorkItem &single,
                           const LaunchShape &shape, hipStream_t stream);

// One workgroup of 64 G P lanes per jump item (geometry jump_shape(N), P
// chosen per launch); d_items on the device, h_items the same items on the
// host, grouped by lane width and word groups (one launch per run).
hipError_t launch_jumps(const JumpItem *d_items, const JumpItem *h_items, uint32_t nitems, hipStream_t stream);

// Allow every generation kernel to use up to `bytes` of dynamic LDS.
hipError_t opt_in_lds(size_t bytes);

// The allocation-free batch call's fixed device scratch: 256 bytes of queue
// counters, then up to kStaticMaxItems work items (128 KiB + 256 bytes).
constexpr uint32_t kStaticMaxItems = 4096;
constexpr size_t kStaticCounterBytes = 256;
constexpr size_t kStaticScratchBytes = kStaticCounterBytes + (size_t)kStaticMaxItems * sizeof(WorkItem);

// Device address of that scratch on the current device (looked up once per
// device, then cached).
hipError_t static_scratch(void **ptr);

// Zero n words at p with a one-wavefront kernel on `stream`.
hipError_t launch_zero_words(uint32_t *p, uint32_t n, hipStream_t stream);

}  // namespace mtgp_impl
