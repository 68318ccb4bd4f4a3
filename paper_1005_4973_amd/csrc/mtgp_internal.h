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

// One unit of work: n outputs of `kind` from generator `gen` into `out`.
struct alignas(32) WorkItem {
    uint64_t out;        // device address of the first output word
    uint64_t n;          // outputs to produce
    uint32_t gen;        // index into the GenRecord array
    uint16_t kind;       // 0 uint32, 1 float [1,2), 2 float [0,1)
    uint16_t spl;        // steps per lane per round for this item
    uint64_t reserved;   // 0
};
static_assert(sizeof(WorkItem) == 32, "WorkItem layout");

// Launch shape of the generation kernels.
constexpr int kModeGroup = 0;   // one workgroup per generator, a barrier per round
constexpr int kModeWave = 1;    // one wavefront per generator, no barriers

struct LaunchShape {
    int mode;        // kModeGroup or kModeWave
    int threads;     // workgroup size (multiple of 64, <= 1024)
    int spl;         // largest steps per lane per round an item may use
                     // (group: 1, 2, 4; wave: 1, 2, 4, 6, 8, 12, 16)
    int lds_words;   // LDS window length L in words per generator (>= 2N + lanes*spl of every item)
    int grid;        // workgroups
};

inline uint32_t shape_lanes(const LaunchShape &s) { return s.mode == kModeGroup ? (uint32_t)s.threads : 64u; }

// Steps per lane per round for a generator under a launch shape: the largest
// supported value s <= shape.spl with lanes*s <= N - M (every slot of a round
// useful), or 1 when even one slot per lane exceeds N - M.
inline uint16_t item_spl(uint32_t N, uint32_t M, const LaunchShape &s)
{
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

// W of a generator under a launch shape: min(N - M, lanes * item_spl).
inline uint32_t round_width(uint32_t N, uint32_t M, const LaunchShape &s)
{
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

// Allow every generation kernel to use up to `bytes` of dynamic LDS.
hipError_t opt_in_lds(size_t bytes);

}  // namespace mtgp_impl
