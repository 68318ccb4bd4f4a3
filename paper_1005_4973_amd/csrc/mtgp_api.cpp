// C ABI of the MTGP library (declared in include/mtgp.h): parameter
// validation, state seeding, device residency of states and parameters, and
// the launch paths (single generator, persistent batch, one launch per
// request, graph-captured plans).
#include "../../include/mtgp.h"
#include "mtgp_f2.h"
#include "mtgp_internal.h"
#include "mtgp_host.h"

static_assert(mtgp_impl::kModeRecBasis == MTGP_MODE_REC_BASIS, "launch mode flag");
static_assert(mtgp_impl::kStaticMaxItems == MTGP_STATIC_MAX_ITEMS, "allocation-free call: item limit");
static_assert(mtgp_impl::kStaticScratchBytes == MTGP_STATIC_SCRATCH_BYTES, "allocation-free call: scratch size");

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <thread>
#include <vector>

using namespace mtgp_impl;

namespace {

thread_local int g_last_error = MTGP_OK;

int fail(int code)
{
    g_last_error = code;
    return code;
}

constexpr uint32_t kMinMexp = 65;           // N >= 3
constexpr uint32_t kMaxMexp = 65536;        // N <= 2048
constexpr size_t kLdsPerCu = 160u * 1024u;  // gfx950 LDS per compute unit
constexpr size_t kUnitLdsExtra = 64;        // table words ahead of each window
constexpr uint32_t kWavesPerCu = 32;        // resident wavefront limit per CU used for sizing grids

uint32_t words_of(uint32_t mexp) { return (mexp + 31u) / 32u; }

bool table_is_linear(const uint32_t *tbl)
{
    if (tbl[0] != 0)
        return false;
    for (int a = 0; a < 16; a++)
        for (int b = 0; b < 16; b++)
            if (tbl[a ^ b] != (tbl[a] ^ tbl[b]))
                return false;
    return true;
}

bool params_valid(const mtgp_param_set *ps)
{
    if (!ps || ps->mexp < kMinMexp || ps->mexp > kMaxMexp)
        return false;
    const uint32_t N = words_of(ps->mexp);
    if (ps->pos < 2 || ps->pos > N - 1)
        return false;
    if (ps->sh1 > 31 || ps->sh2 > 31)
        return false;
    return table_is_linear(ps->param_tbl) && table_is_linear(ps->temper_tbl);
}

GenRecord make_record(const mtgp_param_set *ps, uint64_t state_off)
{
    GenRecord r;
    std::memset(&r, 0, sizeof(r));
    r.N = words_of(ps->mexp);
    r.M = ps->pos;
    r.sh1 = ps->sh1;
    r.sh2 = ps->sh2;
    const uint32_t rbits = 32u * r.N - ps->mexp;
    r.mask = 0xffffffffu << rbits;
    r.state_off = state_off;
    for (int i = 0; i < 16; i++) {
        r.rec[i] = ps->param_tbl[i];
        r.tmp[i] = ps->temper_tbl[i];
        // float output: exponent bits of 1.0 above the 23 MSBs of the tempering word
        r.flt[i] = 0x3f800000u | (ps->temper_tbl[i] >> 9);
    }
    return r;
}

// Seeding (the paper leaves it open): the MT19937 initialisation recurrence.
void seed_words(uint32_t seed, uint32_t n, uint32_t *x)
{
    uint32_t v = seed;
    x[0] = v;
    for (uint32_t i = 1; i < n; i++) {
        v = 1812433253u * (v ^ (v >> 30)) + i;
        x[i] = v;
    }
}

int check_out(const void *out, size_t n)
{
    if (n == 0)
        return MTGP_OK;
    if (out == nullptr || (reinterpret_cast<uintptr_t>(out) & 3u) != 0)
        return MTGP_EINVAL;
    return MTGP_OK;
}

// Largest dynamic LDS a workgroup may use on the current device; the kernels
// are opted in to it once per process.
size_t device_max_lds()
{
    static size_t cached = 0;
    if (cached)
        return cached;
    int dev = 0;
    int val = 0;
    size_t lim = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        if (hipDeviceGetAttribute(&val, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && val > 0)
            lim = (size_t)val;
        else if (hipDeviceGetAttribute(&val, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                 val > 0)
            lim = (size_t)val;
    }
    lim = std::min(lim, kLdsPerCu);
    if (lim > 65536 && opt_in_lds(lim) != hipSuccess)
        lim = 65536;
    cached = lim;
    return cached;
}

bool spl_supported(int mode, int spl)
{
    if (mode == kModeGroup)
        return spl == 1 || spl == 2 || spl == 4;
    if (mode == kModeChunk)
        return spl == 1 || spl == 2;
    return spl == 1 || spl == 2 || spl == 4 || spl == 6 || spl == 8 || spl == 12 || spl == 16;
}

uint32_t shape_units(const LaunchShape &s) { return s.mode == kModeGroup ? 1u : (uint32_t)(s.threads / 64); }

// LDS words per wavefront of the chunked form with ring length L: the ring
// and its copy, and the two 16-word tables.
size_t chunk_unit_words(uint32_t L) { return 2u * (size_t)L + 32u; }

// LDS bytes a launch shape asks for per workgroup.
size_t shape_lds_bytes(const LaunchShape &s)
{
    if (s.mode == kModeChunk)
        return (size_t)shape_units(s) * chunk_unit_words((uint32_t)s.lds_words) * 4u;
    return (size_t)shape_units(s) * (kUnitLdsExtra + (size_t)s.lds_words) * 4u;
}

constexpr uint32_t kChunkMaxRing = 4096;   // ring lengths the chunked kernel is built for: 512 .. 4096

uint32_t max_window_words(const LaunchShape &s, size_t max_lds)
{
    if (s.mode == kModeChunk) {
        uint32_t L = kChunkMaxRing;
        while (L > 512 && shape_units(s) * chunk_unit_words(L) * 4u > max_lds)
            L /= 2;
        return L;
    }
    return (uint32_t)(max_lds / 4u / shape_units(s) - kUnitLdsExtra);
}

// Whether the chunked form with read-ahead `depth` can run a generator
// (N - M >= 64 (depth + 2), and a ring it is built for).
// A generator's state words and M, kept beside the batch's records in a
// compact array: the per-item passes of every launch (shape, checks, order)
// read only these, and 8 bytes a generator stay in cache where the 256-byte
// records of tens of thousands of generators do not.
struct GenShape {
    uint32_t N, M;
};

template <class R>
bool chunk_ok(const R &r, uint32_t depth)
{
    return r.N - r.M >= chunk_min_gap(depth) && chunk_ring_words(r.N) <= kChunkMaxRing;
}

// Window a generator needs under a shape: 2N + lanes * item_spl words; the
// chunked form's ring length (no length serves a generator it cannot run).
template <class R>
uint32_t window_need(const R &r, const LaunchShape &s)
{
    if (s.mode == kModeChunk)
        return chunk_ok(r, (uint32_t)s.spl) ? chunk_ring_words(r.N) : UINT32_MAX;
    return 2 * r.N + round_span(r.N, r.M, s);
}

bool shape_valid(const LaunchShape &s, size_t max_lds)
{
    if (s.mode != kModeGroup && s.mode != kModeWave && s.mode != kModeChunk)
        return false;
    if (s.threads < 64 || s.threads > 1024 || s.threads % 64 != 0)
        return false;
    if (!spl_supported(s.mode, s.spl) || s.lds_words <= 0 || s.grid <= 0)
        return false;
    if (s.mode == kModeChunk && (s.lds_words < 512 || s.lds_words > (int)kChunkMaxRing ||
                                 (s.lds_words & (s.lds_words - 1)) != 0))
        return false;
    return shape_lds_bytes(s) <= max_lds;
}

// Workgroups that fit on the device at once for a shape (LDS and wave limits).
uint64_t resident_groups(const LaunchShape &s, int cu_count)
{
    const size_t by_lds = std::max<size_t>(1u, kLdsPerCu / shape_lds_bytes(s));
    const size_t by_waves = std::max<size_t>(1u, kWavesPerCu / (size_t)(s.threads / 64));
    return (uint64_t)cu_count * std::min(by_lds, by_waves);
}

// Launch shape for one generator alone on the GPU: one workgroup of 256
// lanes (fewer when N - M < 256), up to four steps per lane, and the largest
// LDS window (fewest compactions).
LaunchShape single_shape(const GenRecord &r, size_t max_lds)
{
    LaunchShape s;
    s.mode = kModeGroup;
    const uint32_t w = r.N - r.M;
    const uint32_t lanes = w >= 256 ? 256u : (w + 63u) / 64u * 64u;
    s.threads = (int)std::max<uint32_t>(64u, lanes);
    s.spl = 4;
    s.grid = 1;
    s.lds_words = 1;
    s.lds_words = (int)max_window_words(s, max_lds);
    return s;
}

}  // namespace

struct mtgp {
    mtgp_param_set ps;
    GenRecord rec;
    GenRecord *d_rec = nullptr;
    uint32_t *d_state = nullptr;
    uint64_t consumed = 0;
    hipStream_t last = nullptr;
    LaunchShape shape;
    size_t max_lds = 65536;
    int cu_count = 0;
    // jump-ahead for long calls
    uint32_t split_rounds = 0;                 // 0: never split a call
    f2::Poly psi;                              // annihilator of the orbit (deg < 1: not known)
    bool psi_known = false;
    uint64_t split_J = 0;                      // segment length the buffers below were made for
    uint32_t split_S = 0;
    char *d_split = nullptr;                   // [raw][polynomials][segment states][jump items][work items][counters]
    uint32_t *d_raw = nullptr, *d_seg = nullptr, *d_counters = nullptr;
    JumpItem *d_jumps = nullptr;
    WorkItem *d_items = nullptr;
    std::vector<JumpItem> jumps;               // host copy, for the launch grouping
    WorkItem *h_items = nullptr;               // pinned staging of the segment items
    hipEvent_t items_free = nullptr;           // the staging copy of the previous split call is done
    bool items_pending = false;
};

struct mtgp_batch {
    uint32_t count = 0;
    std::vector<GenRecord> recs;
    std::vector<GenShape> gs;       // N and M of each record, compact
    std::vector<uint64_t> consumed;
    GenRecord *d_recs = nullptr;
    uint32_t *d_states = nullptr;
    size_t state_words = 0;        // words of d_states
    uint32_t *d_counters = nullptr;
    WorkItem *d_items = nullptr;
    WorkItem *h_items = nullptr;   // pinned staging for the item list
    uint32_t item_cap = 0;
    hipEvent_t items_free = nullptr;
    bool items_pending = false;
    hipStream_t last = nullptr;
    int cu_count = 0;
    size_t max_lds = 65536;
    bool have_override = false;
    LaunchShape override_shape;
    // jump-ahead
    std::vector<uint32_t> mexp;
    uint32_t split_rounds = 0;                 // 0: never split a request
    std::vector<uint64_t> epoch;               // bumped by set_state
    std::vector<f2::Poly> psi;                 // annihilator of the generator's orbit (empty: none)
    std::vector<uint64_t> psi_epoch;           // epoch + 1 when psi was computed, 0 if never
    mtgp_plan *eager_plan = nullptr;           // the last eager call run as a one-off split plan
    // allocation-free calls (mtgp_batch_generate_static): pinned staging of
    // kStaticMaxItems items, made with the batch, and the event after which
    // the last such call's upload has read it
    WorkItem *h_static = nullptr;
    hipEvent_t static_free = nullptr;
    bool static_pending = false;
};

struct mtgp_plan {
    mtgp_batch *b = nullptr;
    std::vector<WorkItem> items;
    WorkItem *d_items = nullptr;
    uint32_t *d_counters = nullptr;
    hipStream_t capture = nullptr;
    // graphs: [0] both phases, [1] prepare only, [2] generate only
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    LaunchShape shape;
    // jump-ahead segments
    std::vector<uint32_t> split_gens;
    std::vector<uint64_t> split_epochs;
    void *d_jump_mem = nullptr;                // raw words, polynomials, segment states, prefix and jump items
    WorkItem *d_prefix = nullptr;              // raw-prefix items (in d_items' allocation)
    uint32_t nprefix = 0;
    LaunchShape pshape;                        // launch shape of the raw prefix
    JumpItem *d_jumps = nullptr;               // jump items (in d_items' allocation)
    std::vector<JumpItem> jumps;               // host copy, grouped by lane width
    // the jump launches (one per lane width and word-group count) as two
    // branches of the captured graph: the run with the most work (its jumps'
    // D N summed) on the capture stream, the other runs one after another on
    // a side stream; run k = items [runs[k], runs[k + 1])
    std::vector<uint32_t> runs;
    uint32_t heavy = 0;                        // the run on the capture stream
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

// Default persistent launch shape for a batch (when no override is set):
// 256-lane workgroups (one generator each, up to four steps per lane) and k
// workgroups per CU, k = ceil(requests / CUs) capped by the resident-wave
// limit. The LDS window is sized so that exactly k workgroups fit in a CU's
// LDS and the grid is k * CUs: the hardware then has to place k workgroups on
// every CU. (Left free, it packed several latency-bound generators onto one
// CU while others idled.) k = 1 gives each generator a whole CU.
// A read-only view of a work-item list (a vector, or the allocation-free
// call's staging array): shape choices take this so that no list is copied.
struct Items {
    const WorkItem *ptr = nullptr;
    size_t count = 0;
    Items(const std::vector<WorkItem> &v) : ptr(v.data()), count(v.size()) {}
    Items(const WorkItem *p, size_t n) : ptr(p), count(n) {}
    const WorkItem *begin() const { return ptr; }
    const WorkItem *end() const { return ptr + count; }
    size_t size() const { return count; }
    bool empty() const { return count == 0; }
};

// Chunked-form launch for a set of items whose generators it can all run:
// `threads` lanes per workgroup (one item per wavefront), the least ring
// that serves every item, and as many workgroups as the items fill, up to
// kChunkWavesPerCu wavefronts on every CU. Two wavefronts a SIMD measured
// fastest: with more, the output streams written at once multiply and the
// store throughput falls (16 a CU ran 24 % slower than 8 on uneven batches).
constexpr uint32_t kChunkWavesPerCu = 8;
// The automatic shape is the chunked form only with at least this many items
// per CU: one wavefront per item needs about eight per CU to keep a CU's
// issue, LDS and stores busy, while with fewer items the workgroup form (four
// wavefronts per item) both fills the GPU and gives each item a shorter
// latency (request-loop ticks, a few hundred generators).
constexpr uint32_t kChunkMinItemsPerCu = 8;

LaunchShape chunk_shape(const mtgp_batch *b, Items items, int threads = 256, int depth = 0)
{
    LaunchShape s;
    s.mode = kModeChunk;
    s.threads = threads;
    // read two chunks ahead where every item allows it (the deeper pipeline
    // measured 3-6 % faster), else one
    if (depth == 0) {
        depth = 2;
        for (const WorkItem &it : items)
            if (!chunk_ok(b->gs[it.gen], 2))
                depth = 1;
    }
    s.spl = depth;
    uint32_t L = 512;
    for (const WorkItem &it : items)
        L = std::max(L, chunk_ring_words(b->gs[it.gen].N));
    s.lds_words = (int)L;
    const uint32_t units = (uint32_t)threads / 64u;
    const uint32_t by_lds = (uint32_t)(kLdsPerCu / (chunk_unit_words(L) * 4u)) / units;
    const uint32_t per_cu = std::max(1u, std::min(by_lds, std::max(1u, kChunkWavesPerCu / units)));
    const uint64_t want = (items.size() + units - 1) / units;
    s.grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)per_cu * (uint64_t)b->cu_count));
    return s;
}

bool all_chunk_ok(const mtgp_batch *b, Items items, uint32_t depth = 1)
{
    for (const WorkItem &it : items)
        if (!chunk_ok(b->gs[it.gen], depth))
            return false;
    return !items.empty();
}

LaunchShape batch_default_shape(const mtgp_batch *b, Items items, int threads = 256,
                                int spl = 4)
{
    LaunchShape s;
    s.mode = kModeGroup;
    s.threads = threads;
    s.spl = spl;
    s.grid = 1;
    uint32_t need = 0;
    for (const WorkItem &it : items)
        need = std::max(need, window_need(b->gs[it.gen], s));
    s.lds_words = 1;
    const uint32_t cap = max_window_words(s, b->max_lds);
    const uint32_t by_waves = std::max(1u, kWavesPerCu / (uint32_t)(s.threads / 64));
    const uint64_t cus = (uint64_t)b->cu_count;
    uint32_t k = (uint32_t)std::min<uint64_t>(by_waves, (items.size() + cus - 1) / cus);
    k = std::max(k, 1u);
    // bytes per workgroup, kept 1 KiB below an even share (allocation granularity)
    const size_t share = (kLdsPerCu / k) / 1024u * 1024u - 1024u;
    const uint32_t fit = (uint32_t)(share / 4u - kUnitLdsExtra);
    s.lds_words = (int)std::min(cap, std::max(need, fit));
    s.grid = (int)std::min<uint64_t>(items.size(), (uint64_t)k * cus);
    return s;
}

// Resolve the launch shape for a set of items: override (with automatic
// window and grid filled in) or default; validated against every item.
int resolve_shape(const mtgp_batch *b, Items items, LaunchShape &out)
{
    LaunchShape s;
    if (b->have_override && b->override_shape.mode == kModeChunk && b->override_shape.lds_words == 0 &&
        b->override_shape.grid == 0) {
        // chunked form with automatic ring and grid
        s = chunk_shape(b, items, b->override_shape.threads, b->override_shape.spl);
    } else if (b->have_override && b->override_shape.mode == kModeGroup && b->override_shape.lds_words == 0 &&
        b->override_shape.grid == 0) {
        // workgroup form with automatic window and grid: placed like the default
        s = batch_default_shape(b, items, b->override_shape.threads, b->override_shape.spl);
        s.rec_basis = b->override_shape.rec_basis;
    } else if (b->have_override) {
        s = b->override_shape;
        if (s.lds_words == 0) {
            uint32_t need = 0;
            for (const WorkItem &it : items)
                need = std::max(need, window_need(b->gs[it.gen], s));
            s.lds_words = (int)need;
        }
        if (s.grid == 0) {
            const uint64_t units = shape_units(s);
            const uint64_t want = (items.size() + units - 1) / units;
            s.grid = (int)std::min<uint64_t>(want, resident_groups(s, b->cu_count));
        }
    } else if (all_chunk_ok(b, items) && items.size() >= (size_t)kChunkMinItemsPerCu * (size_t)b->cu_count) {
        s = chunk_shape(b, items);
    } else {
        s = batch_default_shape(b, items);
    }
    if (!shape_valid(s, b->max_lds))
        return MTGP_EINVAL;
    for (const WorkItem &it : items)
        if ((uint32_t)s.lds_words < window_need(b->gs[it.gen], s))
            return MTGP_EINVAL;
    out = s;
    return MTGP_OK;
}

// Normals come in pairs within a call, and a round must hold whole pairs.
bool normal_ok(const GenRecord &r, uint64_t n) { return n % 2 == 0 && r.N - r.M >= 2; }

int validate_requests(const mtgp_batch *b, const mtgp_request *reqs, uint32_t nreq, bool unique)
{
    if (!b || (nreq > 0 && !reqs))
        return MTGP_EINVAL;
    std::vector<uint8_t> seen(unique ? b->count : 0, 0);
    for (uint32_t i = 0; i < nreq; i++) {
        const mtgp_request &r = reqs[i];
        if (r.gen >= b->count || r.kind > MTGP_KIND_NORMAL_FLOAT32 || check_out(r.out, r.n) != MTGP_OK)
            return MTGP_EINVAL;
        if (r.kind == MTGP_KIND_NORMAL_FLOAT32 && !normal_ok(b->recs[r.gen], r.n))
            return MTGP_EINVAL;
        if (unique && r.n > 0) {
            if (seen[r.gen])
                return MTGP_EINVAL;
            seen[r.gen] = 1;
        }
    }
    return MTGP_OK;
}

std::vector<WorkItem> items_of(const mtgp_request *reqs, uint32_t nreq)
{
    std::vector<WorkItem> items;
    items.reserve(nreq);
    for (uint32_t i = 0; i < nreq; i++) {
        if (reqs[i].n == 0)
            continue;
        WorkItem it;
        std::memset(&it, 0, sizeof(it));
        it.out = reinterpret_cast<uint64_t>(reqs[i].out);
        it.n = reqs[i].n;
        it.gen = reqs[i].gen;
        it.kind = (uint16_t)reqs[i].kind;
        items.push_back(it);
    }
    return items;
}

// Fill in steps per lane and order the items longest critical path first
// (rounds = ceil(n / W), each round weighted by its slots per lane).
void finish_items(const mtgp_batch *b, std::vector<WorkItem> &items, const LaunchShape &s)
{
    // each item's cost once, then the items in decreasing cost, equal costs
    // in their given order
    std::vector<std::pair<uint64_t, uint32_t>> key(items.size());
    for (size_t i = 0; i < items.size(); i++) {
        WorkItem &it = items[i];
        const GenShape &r = b->gs[it.gen];
        it.spl = item_spl(r.N, r.M, s);
        const uint64_t w = round_width(r.N, r.M, s);
        key[i] = {(it.n + w - 1) / w * (uint64_t)it.spl, (uint32_t)i};
    }
    std::sort(key.begin(), key.end(), [](const std::pair<uint64_t, uint32_t> &x, const std::pair<uint64_t, uint32_t> &y) {
        return x.first != y.first ? x.first > y.first : x.second < y.second;
    });
    std::vector<WorkItem> sorted(items.size());
    for (size_t i = 0; i < key.size(); i++)
        sorted[i] = items[key[i].second];
    items.swap(sorted);
}

void batch_free(mtgp_batch *b)
{
    if (!b)
        return;
    (void)hipFree(b->d_recs);
    (void)hipFree(b->d_states);
    (void)hipFree(b->d_counters);
    (void)hipFree(b->d_items);
    if (b->h_items)
        (void)hipHostFree(b->h_items);
    if (b->items_free)
        (void)hipEventDestroy(b->items_free);
    if (b->h_static)
        (void)hipHostFree(b->h_static);
    if (b->static_free)
        (void)hipEventDestroy(b->static_free);
    delete b;
}

void plan_free(mtgp_plan *p)
{
    if (!p)
        return;
    for (int k = 0; k < 3; k++) {
        if (p->exec[k])
            (void)hipGraphExecDestroy(p->exec[k]);
        if (p->graph[k])
            (void)hipGraphDestroy(p->graph[k]);
    }
    if (p->capture)
        (void)hipStreamDestroy(p->capture);
    if (p->side)
        (void)hipStreamDestroy(p->side);
    if (p->ev_fork)
        (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join)
        (void)hipEventDestroy(p->ev_join);
    (void)hipFree(p->d_items);
    (void)hipFree(p->d_counters);
    (void)hipFree(p->d_jump_mem);
    delete p;
}

// Enqueue the kernels of a plan's phases (bit 0: raw prefix and jumps, bit 1:
// generation) on the plan's capture stream and instantiate them as a graph.
bool capture_phases(mtgp_plan *p, int mask, hipGraph_t &graph, hipGraphExec_t &exec)
{
    if (hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return false;
    WorkItem none;
    std::memset(&none, 0, sizeof(none));
    const mtgp_batch *b = p->b;
    hipError_t le = hipSuccess;
    if ((mask & 1) && p->nprefix > 0) {
        le = launch_generate(b->d_recs, b->d_states, p->d_prefix, p->nprefix, nullptr, none, p->pshape, p->capture);
        if (le == hipSuccess && !p->side) {
            le = launch_jumps(p->d_jumps, p->jumps.data(), (uint32_t)p->jumps.size(), p->capture);
        } else if (le == hipSuccess) {
            // fork after the raw prefix: the heaviest run here, the others on
            // the side stream; joined whatever happened, so the capture can end
            le = hipEventRecord(p->ev_fork, p->capture);
            if (le == hipSuccess)
                le = hipStreamWaitEvent(p->side, p->ev_fork, 0);
            for (size_t k = 0; k + 1 < p->runs.size() && le == hipSuccess; k++) {
                const uint32_t a = p->runs[k], n = p->runs[k + 1] - a;
                le = launch_jumps(p->d_jumps + a, p->jumps.data() + a, n, k == p->heavy ? p->capture : p->side);
            }
            const hipError_t je = hipEventRecord(p->ev_join, p->side);
            const hipError_t we = je == hipSuccess ? hipStreamWaitEvent(p->capture, p->ev_join, 0) : je;
            if (le == hipSuccess)
                le = we;
        }
    }
    if ((mask & 2) && le == hipSuccess)
        le = launch_generate(b->d_recs, b->d_states, p->d_items, (uint32_t)p->items.size(), p->d_counters, none,
                             p->shape, p->capture);
    const hipError_t ce = hipStreamEndCapture(p->capture, &graph);
    if (le != hipSuccess || ce != hipSuccess || graph == nullptr)
        return false;
    return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
}

// ---------------------------------------------------------------------------
// Jump-ahead (section 7): a request whose rounds exceed the batch's split
// limit becomes S segments of J outputs; segment k starts from F^{kJ} S,
// computed on the GPU as h_k(F) S with h_k = x^{kJ} mod psi, where psi
// annihilates the generator's orbit.
// ---------------------------------------------------------------------------

void parallel_for(size_t n, const std::function<void(size_t)> &fn)
{
    size_t nt = std::max<size_t>(1u, std::min<size_t>(std::thread::hardware_concurrency(), 16u));
    nt = std::min(nt, n);
    std::atomic<size_t> next{0};
    std::vector<std::thread> th;
    for (size_t t = 0; t < nt; t++)
        th.emplace_back([&] {
            for (;;) {
                const size_t i = next++;
                if (i >= n)
                    break;
                fn(i);
            }
        });
    for (auto &x : th)
        x.join();
}

// True if sum_{i: phi_i = 1} X[i + w] = 0 for every w < N.
bool annihilates(const f2::Poly &phi, const uint32_t *X, size_t len, uint32_t N)
{
    if (phi.deg < 0 || (size_t)phi.deg + N > len)
        return false;
    std::vector<uint32_t> acc(N, 0);
    for (int64_t i = 0; i <= phi.deg; i++)
        if (phi.bit(i))
            for (uint32_t w = 0; w < N; w++)
                acc[w] ^= X[i + w];
    for (uint32_t w = 0; w < N; w++)
        if (acc[w])
            return false;
    return true;
}

// Raw words needed to find an annihilator for exponent p: the N state words
// and 2p + 65 new ones (Berlekamp-Massey needs twice the linear complexity,
// which is at most p + 1 here).
uint64_t raw_steps_for(uint32_t p) { return 2ull * p + 65; }

// Annihilating polynomial of the orbit of the state X[0..N) (X continues with
// the raw words that follow): the LCM of the minimal polynomials of the bit
// planes of x_{c+1}, x_{c+2}, ... -- a polynomial annihilates the word
// sequence exactly when it annihilates every bit plane -- taken until it
// annihilates the state at c+1 (checked on all N words), then multiplied by x
// so that it annihilates the state at c too (the transition may be singular).
// Returns the zero polynomial if no annihilator is found.
f2::Poly orbit_annihilator(const uint32_t *X, size_t len, uint32_t N, uint32_t p)
{
    const int64_t nbits = 2 * (int64_t)p + 64;
    if ((size_t)nbits + 1 > len)
        return f2::Poly();
    static const int order[32] = {0, 16, 8, 24, 4, 12, 20, 28, 2, 6, 10, 14, 18, 22, 26, 30,
                                  1, 3, 5, 7, 9, 11, 13, 15, 17, 19, 21, 23, 25, 27, 29, 31};
    std::vector<uint64_t> packed((size_t)(nbits / 64 + 1));
    f2::Poly phi = f2::Poly::one();
    for (int bi = 0; bi < 32; bi++) {
        const int b = order[bi];
        std::fill(packed.begin(), packed.end(), 0);
        for (int64_t j = 0; j < nbits; j++)
            if ((X[1 + j] >> b) & 1u)
                packed[(size_t)(j >> 6)] |= 1ull << (j & 63);
        phi = f2::lcm(phi, f2::minpoly(packed.data(), nbits));
        if (phi.deg > (int64_t)p + 1)
            return f2::Poly();
        if (annihilates(phi, X + 1, len - 1, N)) {
            f2::Poly psi = f2::mul(phi, f2::Poly::from_words(std::vector<uint64_t>{2}.data(), 1));
            return psi;
        }
    }
    return f2::Poly();
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Shape of the prefix launch that writes raw words: 256 lanes per generator.
LaunchShape raw_shape(const mtgp_batch *b, const std::vector<uint32_t> &gens)
{
    LaunchShape s;
    s.mode = kModeGroup;
    s.threads = 256;
    s.spl = 4;
    s.grid = (int)gens.size();
    uint32_t need = 0;
    for (uint32_t g : gens)
        need = std::max(need, window_need(b->recs[g], s));
    s.lds_words = (int)std::max(need, 4096u);
    return s;
}

// Make sure every generator in `gens` has an annihilator for its current
// orbit: raw words are generated on the GPU from the current states (the
// states are not advanced) and reduced on the host.
int ensure_annihilators(mtgp_batch *b, const std::vector<uint32_t> &gens)
{
    std::vector<uint32_t> todo;
    for (uint32_t g : gens)
        if (b->psi_epoch[g] != b->epoch[g] + 1)
            todo.push_back(g);
    if (todo.empty())
        return MTGP_OK;
    std::vector<WorkItem> items(todo.size());
    std::vector<size_t> off(todo.size());
    size_t total = 0;
    for (size_t i = 0; i < todo.size(); i++) {
        const GenRecord &r = b->recs[todo[i]];
        off[i] = total;
        total += r.N + raw_steps_for(b->mexp[todo[i]]);
    }
    const LaunchShape s = raw_shape(b, todo);
    uint32_t *d_raw = nullptr;
    WorkItem *d_items = nullptr;
    hipStream_t st = nullptr;
    int rc = MTGP_OK;
    if (hipStreamSynchronize(b->last) != hipSuccess)
        return MTGP_EDEVICE;
    if (hipMalloc(&d_raw, total * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&d_items, items.size() * sizeof(WorkItem)) != hipSuccess) {
        (void)hipFree(d_raw);
        return MTGP_ENOMEM;
    }
    for (size_t i = 0; i < todo.size(); i++) {
        const GenRecord &r = b->recs[todo[i]];
        std::memset(&items[i], 0, sizeof(WorkItem));
        items[i].out = reinterpret_cast<uint64_t>(d_raw + off[i]);
        items[i].n = raw_steps_for(b->mexp[todo[i]]);
        items[i].gen = todo[i];
        items[i].kind = kKindRaw | kKeepState;
        items[i].spl = item_spl(r.N, r.M, s);
    }
    std::vector<uint32_t> raw(total);
    WorkItem none;
    std::memset(&none, 0, sizeof(none));
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        launch_generate(b->d_recs, b->d_states, d_items, (uint32_t)items.size(), nullptr, none, s, st) != hipSuccess ||
        hipMemcpyAsync(raw.data(), d_raw, total * sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        rc = MTGP_EDEVICE;
    if (st)
        (void)hipStreamDestroy(st);
    (void)hipFree(d_items);
    (void)hipFree(d_raw);
    if (rc != MTGP_OK)
        return rc;
    parallel_for(todo.size(), [&](size_t i) {
        const uint32_t g = todo[i];
        const uint32_t N = b->recs[g].N;
        b->psi[g] = orbit_annihilator(raw.data() + off[i], N + raw_steps_for(b->mexp[g]), N, b->mexp[g]);
    });
    for (uint32_t g : todo)
        b->psi_epoch[g] = b->epoch[g] + 1;
    return MTGP_OK;
}

// Segments for a request of n outputs needing `rounds` rounds: S segments of
// J outputs (the last takes the rest), J even so normals keep their pairs.
// At most kMaxSegments per request: more would not run at once, and each
// costs a jump and a host polynomial product.
constexpr uint64_t kMaxSegments = 1024;

void split_count(uint64_t n, uint64_t rounds, uint32_t split_rounds, uint32_t &S, uint64_t &J)
{
    S = (uint32_t)std::min<uint64_t>((rounds + split_rounds - 1) / split_rounds, kMaxSegments);
    auto seg_len = [&](uint32_t s) { return ((n + s - 1) / s + 1) & ~(uint64_t)1; };
    J = seg_len(S);
    while (S > 1 && (uint64_t)(S - 1) * J >= n) {
        S--;
        J = seg_len(S);
    }
}

// Jump polynomials h_k = x^{kJ} mod psi, k = 1 .. S-1.
std::vector<f2::Poly> jump_polys(const f2::Poly &psi, uint64_t J, uint32_t S)
{
    std::vector<f2::Poly> h;
    if (S < 2)
        return h;
    const f2::Poly g = f2::powmod_x(J, psi);
    h.push_back(g);
    if (psi.deg < 8) {
        for (uint32_t k = 2; k < S; k++)
            h.push_back(f2::mulmod(h.back(), g, psi));
        return h;
    }
    // h_k = h_{k-1} g in the ring of psi (table reduction)
    f2::SquareMod ring(psi);
    const size_t nw = ring.words();
    std::vector<uint64_t> gw(nw, 0), cur(nw, 0), next(nw, 0);
    std::copy(g.w.begin(), g.w.end(), gw.begin());
    cur = gw;
    for (uint32_t k = 2; k < S; k++) {
        ring.mul(cur.data(), gw.data(), next.data());
        cur.swap(next);
        h.push_back(f2::Poly::from_words(cur.data(), (int64_t)nw * 64 - 1));
    }
    return h;
}

// h in the jump kernel's layout (JumpItem): bit e of h is bit e % R of block
// e / R, four 16-bit blocks per word; dst has jump_poly_words(N, deg psi)
// zeroed words.
void layout_poly(const f2::Poly &h, uint32_t N, uint64_t *dst)
{
    const uint32_t R = jump_shape(N).R;
    for (int64_t e = 0; e <= h.deg; e++)
        if (h.bit(e)) {
            const uint64_t blk = (uint64_t)e / R;
            dst[blk / 4] |= 1ull << (16 * (blk % 4) + (uint64_t)e % R);
        }
}

struct SplitSpec {
    size_t item;        // index in the request's item list
    uint32_t gen;
    uint32_t S;         // segments
    uint64_t J;         // outputs per segment (the last one takes the rest)
};

// Split the plan's long requests into segments. Builds the prefix (raw words)
// and jump work, lays out their device memory, and returns the new item list.
int plan_split(mtgp_plan *p, std::vector<WorkItem> &items, std::vector<WorkItem> &prefix,
               std::vector<JumpItem> &jumps)
{
    mtgp_batch *b = p->b;
    std::vector<SplitSpec> specs;
    for (size_t i = 0; i < items.size(); i++) {
        const GenRecord &r = b->recs[items[i].gen];
        const uint64_t w = round_width(r.N, r.M, p->shape);
        const uint64_t rounds = (items[i].n + w - 1) / w;
        if (rounds <= b->split_rounds)
            continue;
        uint32_t S;
        uint64_t J;
        split_count(items[i].n, rounds, b->split_rounds, S, J);
        if (S > 1)
            specs.push_back({i, items[i].gen, S, J});
    }
    if (specs.empty())
        return MTGP_OK;
    std::vector<uint32_t> gens;
    for (const SplitSpec &sp : specs)
        gens.push_back(sp.gen);
    int rc = ensure_annihilators(b, gens);
    if (rc != MTGP_OK)
        return rc;
    std::vector<SplitSpec> ok;
    for (const SplitSpec &sp : specs)
        if (b->psi[sp.gen].deg >= 1)
            ok.push_back(sp);
    if (ok.empty())
        return MTGP_OK;
    // jump polynomials h_k = x^{kJ} mod psi, k = 1 .. S-1
    std::vector<std::vector<f2::Poly>> polys(ok.size());
    parallel_for(ok.size(), [&](size_t i) { polys[i] = jump_polys(b->psi[ok[i].gen], ok[i].J, ok[i].S); });
    // device layout: [raw words][polynomials][segment states]
    std::vector<size_t> raw_off(ok.size()), poly_off(ok.size()), seg_off(ok.size());
    size_t bytes = 0;
    for (size_t i = 0; i < ok.size(); i++) {
        const uint32_t N = b->recs[ok[i].gen].N;
        const uint32_t D = (uint32_t)b->psi[ok[i].gen].deg;
        raw_off[i] = bytes;
        bytes = align256(bytes + (size_t)(N + D) * 4u);
        poly_off[i] = bytes;
        bytes = align256(bytes + (size_t)(ok[i].S - 1) * jump_poly_words(N, D) * 8u);
        seg_off[i] = bytes;
        bytes = align256(bytes + (size_t)(ok[i].S - 1) * N * 4u);
    }
    char *mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess)
        return MTGP_ENOMEM;
    p->d_jump_mem = mem;
    std::vector<uint64_t> hpoly(bytes / 8, 0);   // staging of the polynomial region (same offsets)
    std::vector<WorkItem> out;
    std::vector<bool> replaced(items.size(), false);
    for (size_t i = 0; i < ok.size(); i++) {
        const SplitSpec &sp = ok[i];
        const WorkItem base = items[sp.item];
        replaced[sp.item] = true;
        const GenRecord &r = b->recs[sp.gen];
        const uint32_t N = r.N;
        const uint32_t D = (uint32_t)b->psi[sp.gen].deg;
        const uint32_t pw = jump_poly_words(N, D);
        uint32_t *raw = reinterpret_cast<uint32_t *>(mem + raw_off[i]);
        uint32_t *seg = reinterpret_cast<uint32_t *>(mem + seg_off[i]);
        // prefix: the state and D - 1 new raw words (states stay put)
        WorkItem pre;
        std::memset(&pre, 0, sizeof(pre));
        pre.out = reinterpret_cast<uint64_t>(raw);
        pre.n = D - 1;
        pre.gen = sp.gen;
        pre.kind = kKindRaw | kKeepState;
        prefix.push_back(pre);
        for (uint32_t k = 1; k < sp.S; k++) {
            layout_poly(polys[i][k - 1], N, hpoly.data() + (poly_off[i] / 8) + (size_t)(k - 1) * pw);
            JumpItem j;
            std::memset(&j, 0, sizeof(j));
            j.raw = reinterpret_cast<uint64_t>(raw);
            j.poly = reinterpret_cast<uint64_t>(mem + poly_off[i] + (size_t)(k - 1) * pw * 8u);
            j.out = reinterpret_cast<uint64_t>(seg + (size_t)(k - 1) * N);
            j.D = D;
            j.N = N;
            jumps.push_back(j);
        }
        for (uint32_t k = 0; k < sp.S; k++) {
            WorkItem it = base;
            const uint64_t start = (uint64_t)k * sp.J;
            it.n = k + 1 < sp.S ? sp.J : base.n - start;
            it.out = base.out + 4u * start;
            it.src = k == 0 ? reinterpret_cast<uint64_t>(raw)
                            : reinterpret_cast<uint64_t>(seg + (size_t)(k - 1) * N);
            it.kind = (uint16_t)(base.kind | (k + 1 < sp.S ? kKeepState : 0));
            out.push_back(it);
        }
        p->split_gens.push_back(sp.gen);
        p->split_epochs.push_back(b->epoch[sp.gen]);
    }
    for (size_t i = 0; i < items.size(); i++)
        if (!replaced[i])
            out.push_back(items[i]);
    items.swap(out);
    // the jump kernel is launched once per lane width and word-group count
    group_jumps_by_shape(jumps);
    // upload the polynomials (only their regions are meaningful)
    for (size_t i = 0; i < ok.size(); i++) {
        const uint32_t D = (uint32_t)b->psi[ok[i].gen].deg;
        const size_t len = (size_t)(ok[i].S - 1) * jump_poly_words(b->recs[ok[i].gen].N, D) * 8u;
        if (hipMemcpy(mem + poly_off[i], hpoly.data() + poly_off[i] / 8, len, hipMemcpyHostToDevice) != hipSuccess)
            return MTGP_EDEVICE;
    }
    return MTGP_OK;
}

}  // namespace

extern "C" {

uint32_t mtgp_state_words(uint32_t mexp)
{
    if (mexp < kMinMexp || mexp > kMaxMexp)
        return 0;
    return words_of(mexp);
}

int mtgp_last_error(void) { return g_last_error; }

const char *mtgp_strerror(int code)
{
    switch (code) {
    case MTGP_OK: return "ok";
    case MTGP_EINVAL: return "invalid argument or parameter set";
    case MTGP_ENOMEM: return "out of memory";
    case MTGP_EDEVICE: return "HIP device error";
    case MTGP_ENOTFOUND: return "no parameter set found within the draw limit";
    default: return "unknown error";
    }
}

mtgp_t *mtgp_create(const mtgp_param_set *ps, uint32_t seed)
{
    if (!params_valid(ps)) {
        fail(MTGP_EINVAL);
        return nullptr;
    }
    mtgp *g = new (std::nothrow) mtgp();
    if (!g) {
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    g->ps = *ps;
    g->rec = make_record(ps, 0);
    const uint32_t N = g->rec.N;
    std::vector<uint32_t> words(N);
    seed_words(seed, N, words.data());
    if (hipMalloc(&g->d_rec, sizeof(GenRecord)) != hipSuccess ||
        hipMalloc(&g->d_state, N * sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(g->d_rec);
        (void)hipFree(g->d_state);
        delete g;
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    if (hipMemcpy(g->d_rec, &g->rec, sizeof(GenRecord), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_state, words.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(g->d_rec);
        (void)hipFree(g->d_state);
        delete g;
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    g->max_lds = device_max_lds();
    g->shape = single_shape(g->rec, g->max_lds);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        g->cu_count = prop.multiProcessorCount;
    return g;
}

// A long call as S segments (section 7): the raw prefix of the current
// state, the S-1 jump correlations, then one persistent launch over the
// segments, all on `s`. The orbit's annihilator is found on the first split
// call (and after set_state); the jump polynomials and device buffers are
// kept for the last segment length used. Returns MTGP_ENOTFOUND when no
// annihilator exists (the caller runs the call unsplit).
static int generate_split(mtgp_t *g, uint64_t n, void *out, hipStream_t s, uint32_t kind)
{
    const GenRecord &r = g->rec;
    const uint32_t N = r.N;
    WorkItem none;
    std::memset(&none, 0, sizeof(none));
    if (!g->psi_known) {
        // raw words of the current state: the N state words and 2p + 65 more
        const uint64_t steps = raw_steps_for(g->ps.mexp);
        std::vector<uint32_t> raw(N + steps);
        uint32_t *d_raw = nullptr;
        if (hipMalloc(&d_raw, raw.size() * sizeof(uint32_t)) != hipSuccess)
            return MTGP_ENOMEM;
        WorkItem it = none;
        it.out = reinterpret_cast<uint64_t>(d_raw);
        it.n = steps;
        it.kind = kKindRaw | kKeepState;
        it.spl = item_spl(N, r.M, g->shape);
        const bool ok = launch_generate(g->d_rec, g->d_state, nullptr, 1, nullptr, it, g->shape, s) == hipSuccess &&
                        hipMemcpyAsync(raw.data(), d_raw, raw.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s) ==
                            hipSuccess &&
                        hipStreamSynchronize(s) == hipSuccess;
        (void)hipFree(d_raw);
        if (!ok)
            return MTGP_EDEVICE;
        g->psi = orbit_annihilator(raw.data(), raw.size(), N, g->ps.mexp);
        g->psi_known = true;
    }
    if (g->psi.deg < 1)
        return MTGP_ENOTFOUND;
    const uint32_t D = (uint32_t)g->psi.deg;
    const uint64_t w = round_width(N, r.M, g->shape);
    uint32_t S;
    uint64_t J;
    split_count(n, (n + w - 1) / w, g->split_rounds, S, J);
    if (S < 2)
        return MTGP_ENOTFOUND;
    if (J != g->split_J || S != g->split_S) {
        // buffers and jump polynomials for this segment length
        if (hipStreamSynchronize(g->last) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return MTGP_EDEVICE;
        (void)hipFree(g->d_split);
        g->d_split = nullptr;
        g->split_J = 0;
        g->split_S = 0;
        const uint32_t pw = jump_poly_words(N, D);
        size_t off = 0;
        const size_t raw_off = off;
        off = align256(off + (size_t)(N + D) * 4u);
        const size_t poly_off = off;
        off = align256(off + (size_t)(S - 1) * pw * 8u);
        const size_t seg_off = off;
        off = align256(off + (size_t)(S - 1) * N * 4u);
        const size_t jump_off = off;
        off = align256(off + (size_t)(S - 1) * sizeof(JumpItem));
        const size_t item_off = off;
        off = align256(off + (size_t)S * sizeof(WorkItem));
        const size_t ctr_off = off;
        off += 2 * sizeof(uint32_t);
        char *mem = nullptr;
        if (hipMalloc(&mem, off) != hipSuccess)
            return MTGP_ENOMEM;
        g->d_split = mem;
        g->d_raw = reinterpret_cast<uint32_t *>(mem + raw_off);
        g->d_seg = reinterpret_cast<uint32_t *>(mem + seg_off);
        g->d_jumps = reinterpret_cast<JumpItem *>(mem + jump_off);
        g->d_items = reinterpret_cast<WorkItem *>(mem + item_off);
        g->d_counters = reinterpret_cast<uint32_t *>(mem + ctr_off);
        const std::vector<f2::Poly> h = jump_polys(g->psi, J, S);
        std::vector<uint64_t> hpoly((size_t)(S - 1) * pw, 0);
        g->jumps.assign(S - 1, JumpItem{});
        for (uint32_t k = 1; k < S; k++) {
            layout_poly(h[k - 1], N, hpoly.data() + (size_t)(k - 1) * pw);
            JumpItem &j = g->jumps[k - 1];
            std::memset(&j, 0, sizeof(j));
            j.raw = reinterpret_cast<uint64_t>(g->d_raw);
            j.poly = reinterpret_cast<uint64_t>(mem + poly_off + (size_t)(k - 1) * pw * 8u);
            j.out = reinterpret_cast<uint64_t>(g->d_seg + (size_t)(k - 1) * N);
            j.D = D;
            j.N = N;
        }
        if (hipMemcpy(mem + poly_off, hpoly.data(), hpoly.size() * 8u, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g->d_jumps, g->jumps.data(), g->jumps.size() * sizeof(JumpItem), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemset(g->d_counters, 0, 2 * sizeof(uint32_t)) != hipSuccess)
            return MTGP_EDEVICE;
        if (g->h_items)
            (void)hipHostFree(g->h_items);
        g->h_items = nullptr;
        if (hipHostMalloc(reinterpret_cast<void **>(&g->h_items), (size_t)S * sizeof(WorkItem)) != hipSuccess)
            return MTGP_ENOMEM;
        if (!g->items_free && hipEventCreateWithFlags(&g->items_free, hipEventDisableTiming) != hipSuccess)
            return MTGP_EDEVICE;
        g->items_pending = false;
        g->split_J = J;
        g->split_S = S;
    }
    // segment items: segment k writes outputs [kJ, kJ + J) from its start state
    if (g->items_pending && hipEventSynchronize(g->items_free) != hipSuccess)
        return MTGP_EDEVICE;
    LaunchShape sh;
    {
        std::vector<WorkItem> items(S);
        for (uint32_t k = 0; k < S; k++) {
            WorkItem &it = items[k];
            std::memset(&it, 0, sizeof(it));
            it.out = reinterpret_cast<uint64_t>(out) + 4u * (uint64_t)k * J;
            it.n = k + 1 < S ? J : n - (uint64_t)k * J;
            it.kind = (uint16_t)(kind | (k + 1 < S ? kKeepState : 0));
            it.src = k == 0 ? reinterpret_cast<uint64_t>(g->d_raw)
                            : reinterpret_cast<uint64_t>(g->d_seg + (size_t)(k - 1) * N);
        }
        // the launch shape of the segments: 256-lane workgroups, as many per
        // CU as the segments need (up to 8), each with an even share of LDS,
        // and the generator's recursion-table form
        sh.mode = kModeGroup;
        sh.threads = 256;
        sh.spl = 4;
        sh.rec_basis = g->shape.rec_basis;
        sh.grid = 1;
        sh.lds_words = 1;
        const uint32_t cus = (uint32_t)std::max(1, g->cu_count);
        const uint32_t kpc = std::max(1u, std::min(8u, (S + cus - 1) / cus));
        const size_t share = (kLdsPerCu / kpc) / 1024u * 1024u - 1024u;
        const uint32_t need = window_need(r, sh);
        const uint32_t cap = max_window_words(sh, g->max_lds);
        sh.lds_words = (int)std::min(cap, std::max(need, (uint32_t)(share / 4u - kUnitLdsExtra)));
        sh.grid = (int)std::min<uint64_t>(S, (uint64_t)kpc * cus);
        if (!shape_valid(sh, g->max_lds) || (uint32_t)sh.lds_words < need)
            return MTGP_EINVAL;
        for (WorkItem &it : items)
            it.spl = item_spl(N, r.M, sh);
        std::memcpy(g->h_items, items.data(), items.size() * sizeof(WorkItem));
    }
    WorkItem pre = none;
    pre.out = reinterpret_cast<uint64_t>(g->d_raw);
    pre.n = D - 1;
    pre.kind = kKindRaw | kKeepState;
    pre.spl = item_spl(N, r.M, g->shape);
    if (hipMemcpyAsync(g->d_items, g->h_items, (size_t)S * sizeof(WorkItem), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(g->items_free, s) != hipSuccess)
        return MTGP_EDEVICE;
    g->items_pending = true;
    if (launch_generate(g->d_rec, g->d_state, nullptr, 1, nullptr, pre, g->shape, s) != hipSuccess ||
        launch_jumps(g->d_jumps, g->jumps.data(), (uint32_t)g->jumps.size(), s) != hipSuccess ||
        launch_generate(g->d_rec, g->d_state, g->d_items, S, g->d_counters, none, sh, s) != hipSuccess)
        return MTGP_EDEVICE;
    g->consumed += n;
    g->last = s;
    return MTGP_OK;
}

static int generate_kind(mtgp_t *g, size_t n, void *out, void *stream, uint32_t kind)
{
    if (!g)
        return fail(MTGP_EINVAL);
    if (check_out(out, n) != MTGP_OK)
        return fail(MTGP_EINVAL);
    if (kind == MTGP_KIND_NORMAL_FLOAT32 && !normal_ok(g->rec, n))
        return fail(MTGP_EINVAL);
    if (n == 0)
        return MTGP_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->split_rounds > 0) {
        const uint64_t w = round_width(g->rec.N, g->rec.M, g->shape);
        if ((n + w - 1) / w > g->split_rounds) {
            const int rc = generate_split(g, n, out, s, kind);
            if (rc != MTGP_ENOTFOUND)   // no annihilator: run the call unsplit
                return rc == MTGP_OK ? MTGP_OK : fail(rc);
        }
    }
    WorkItem it;
    std::memset(&it, 0, sizeof(it));
    it.out = reinterpret_cast<uint64_t>(out);
    it.n = n;
    it.gen = 0;
    it.kind = (uint16_t)kind;
    it.spl = item_spl(g->rec.N, g->rec.M, g->shape);
    if (launch_generate(g->d_rec, g->d_state, nullptr, 1, nullptr, it, g->shape, s) != hipSuccess)
        return fail(MTGP_EDEVICE);
    g->consumed += n;
    g->last = s;
    return MTGP_OK;
}

int mtgp_generate_uint32(mtgp_t *g, size_t n, uint32_t *out, void *stream)
{
    return generate_kind(g, n, out, stream, MTGP_KIND_UINT32);
}

int mtgp_generate_float32_1to2(mtgp_t *g, size_t n, float *out, void *stream)
{
    return generate_kind(g, n, out, stream, MTGP_KIND_FLOAT32_1TO2);
}

int mtgp_generate_float32_0to1(mtgp_t *g, size_t n, float *out, void *stream)
{
    return generate_kind(g, n, out, stream, MTGP_KIND_FLOAT32_0TO1);
}

int mtgp_generate_normal_float32(mtgp_t *g, size_t n, float *out, void *stream)
{
    return generate_kind(g, n, out, stream, MTGP_KIND_NORMAL_FLOAT32);
}

void mtgp_destroy(mtgp_t *g)
{
    if (!g)
        return;
    (void)hipStreamSynchronize(g->last);
    (void)hipFree(g->d_rec);
    (void)hipFree(g->d_state);
    (void)hipFree(g->d_split);
    if (g->h_items)
        (void)hipHostFree(g->h_items);
    if (g->items_free)
        (void)hipEventDestroy(g->items_free);
    delete g;
}

int mtgp_get_state(mtgp_t *g, uint32_t *host_words, uint64_t *consumed)
{
    if (!g || !host_words)
        return fail(MTGP_EINVAL);
    if (hipStreamSynchronize(g->last) != hipSuccess ||
        hipMemcpy(host_words, g->d_state, g->rec.N * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(MTGP_EDEVICE);
    if (consumed)
        *consumed = g->consumed;
    return MTGP_OK;
}

int mtgp_set_state(mtgp_t *g, const uint32_t *host_words, uint64_t consumed)
{
    if (!g || !host_words)
        return fail(MTGP_EINVAL);
    if (hipStreamSynchronize(g->last) != hipSuccess ||
        hipMemcpy(g->d_state, host_words, g->rec.N * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
        return fail(MTGP_EDEVICE);
    g->consumed = consumed;
    g->psi_known = false;   // the orbit may have changed: annihilator and jump polynomials are stale
    g->split_J = 0;
    g->split_S = 0;
    return MTGP_OK;
}

int mtgp_set_split(mtgp_t *g, uint32_t max_rounds)
{
    if (!g)
        return fail(MTGP_EINVAL);
    g->split_rounds = max_rounds;
    return MTGP_OK;
}

int mtgp_set_launch(mtgp_t *g, int mode, int threads, int spl, int lds_words)
{
    if (!g)
        return fail(MTGP_EINVAL);
    if (mode < 0) {
        g->shape = single_shape(g->rec, g->max_lds);
        return MTGP_OK;
    }
    LaunchShape s;
    s.rec_basis = (mode & kModeRecBasis) ? 1 : 0;
    mode &= ~kModeRecBasis;
    s.mode = mode;
    s.threads = mode == kModeGroup ? threads : 64;
    s.spl = spl;
    s.grid = 1;
    s.lds_words = mode == kModeChunk ? 512 : 1;
    if (!shape_valid(s, g->max_lds) || lds_words < 0)
        return fail(MTGP_EINVAL);
    s.lds_words = lds_words > 0 ? lds_words : (int)max_window_words(s, g->max_lds);
    if (!shape_valid(s, g->max_lds) || (uint32_t)s.lds_words < window_need(g->rec, s))
        return fail(MTGP_EINVAL);
    g->shape = s;
    return MTGP_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

mtgp_batch_t *mtgp_batch_create(const mtgp_param_set *ps, const uint32_t *seeds, uint32_t count)
{
    if (!ps || !seeds || count == 0) {
        fail(MTGP_EINVAL);
        return nullptr;
    }
    for (uint32_t i = 0; i < count; i++)
        if (!params_valid(&ps[i])) {
            fail(MTGP_EINVAL);
            return nullptr;
        }
    mtgp_batch *b = new (std::nothrow) mtgp_batch();
    if (!b) {
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    b->count = count;
    b->recs.resize(count);
    b->gs.resize(count);
    b->consumed.assign(count, 0);
    b->mexp.resize(count);
    for (uint32_t i = 0; i < count; i++)
        b->mexp[i] = ps[i].mexp;
    b->epoch.assign(count, 0);
    b->psi.assign(count, f2::Poly());
    b->psi_epoch.assign(count, 0);
    uint64_t off = 0;
    for (uint32_t i = 0; i < count; i++) {
        b->recs[i] = make_record(&ps[i], off);
        b->gs[i] = GenShape{b->recs[i].N, b->recs[i].M};
        off += b->recs[i].N;
    }
    std::vector<uint32_t> words(off);
    for (uint32_t i = 0; i < count; i++)
        seed_words(seeds[i], b->recs[i].N, words.data() + b->recs[i].state_off);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        batch_free(b);
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    b->cu_count = prop.multiProcessorCount;
    b->max_lds = device_max_lds();
    if (hipMalloc(&b->d_recs, count * sizeof(GenRecord)) != hipSuccess ||
        (b->state_words = off, hipMalloc(&b->d_states, off * sizeof(uint32_t)) != hipSuccess) ||
        hipMalloc(&b->d_counters, 2 * sizeof(uint32_t)) != hipSuccess) {
        batch_free(b);
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    if (hipMemcpy(b->d_recs, b->recs.data(), count * sizeof(GenRecord), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_states, words.data(), off * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->d_counters, 0, 2 * sizeof(uint32_t)) != hipSuccess ||
        hipEventCreateWithFlags(&b->items_free, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->static_free, hipEventDisableTiming) != hipSuccess) {
        batch_free(b);
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&b->h_static), kStaticMaxItems * sizeof(WorkItem),
                      hipHostMallocDefault) != hipSuccess) {
        batch_free(b);
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    return b;
}

uint32_t mtgp_batch_size(const mtgp_batch_t *b) { return b ? b->count : 0; }

void mtgp_batch_destroy(mtgp_batch_t *b)
{
    if (!b)
        return;
    mtgp_plan_destroy(b->eager_plan);   // waits for the batch's last stream
    b->eager_plan = nullptr;
    (void)hipStreamSynchronize(b->last);
    batch_free(b);
}

int mtgp_batch_generate(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream)
{
    return mtgp_impl::batch_generate(b, reqs, nreq, stream, true);
}

// The eager batch call without jump-ahead and without any allocation: the
// work items are built in the batch's pinned staging array, checked and
// ordered in place (std::sort, which needs no buffer), uploaded to this
// GPU's fixed scratch array, whose queue counters a one-wavefront kernel
// zeroes first; the generation kernels are the ones mtgp_batch_generate uses.
int mtgp_batch_generate_static(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream)
{
    if (!b || (nreq > 0 && !reqs) || nreq > kStaticMaxItems)
        return fail(MTGP_EINVAL);
    if (validate_requests(b, reqs, nreq, false) != MTGP_OK)
        return fail(MTGP_EINVAL);
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *scr = nullptr;
    if (static_scratch(&scr) != hipSuccess)
        return fail(MTGP_EDEVICE);
    // the previous call's upload must have read the staging array
    if (b->static_pending) {
        if (hipEventSynchronize(b->static_free) != hipSuccess)
            return fail(MTGP_EDEVICE);
        b->static_pending = false;
    }
    WorkItem *h = b->h_static;
    uint32_t k = 0;
    for (uint32_t i = 0; i < nreq; i++) {
        if (reqs[i].n == 0)
            continue;
        WorkItem &it = h[k++];
        std::memset(&it, 0, sizeof(it));
        it.out = reinterpret_cast<uint64_t>(reqs[i].out);
        it.n = reqs[i].n;
        it.gen = reqs[i].gen;
        it.kind = (uint16_t)reqs[i].kind;
    }
    if (k == 0)
        return MTGP_OK;
    // one request per generator
    std::sort(h, h + k, [](const WorkItem &x, const WorkItem &y) { return x.gen < y.gen; });
    for (uint32_t j = 1; j < k; j++)
        if (h[j].gen == h[j - 1].gen)
            return fail(MTGP_EINVAL);
    LaunchShape shape;
    if (resolve_shape(b, Items(h, k), shape) != MTGP_OK)
        return fail(MTGP_EINVAL);
    // steps per lane, then longest critical path first (ties by generator)
    for (uint32_t j = 0; j < k; j++)
        h[j].spl = item_spl(b->recs[h[j].gen].N, b->recs[h[j].gen].M, shape);
    auto cost = [&](const WorkItem &it) {
        const GenRecord &r = b->recs[it.gen];
        const uint64_t w = round_width(r.N, r.M, shape);
        return (it.n + w - 1) / w * (uint64_t)it.spl;
    };
    std::sort(h, h + k, [&](const WorkItem &x, const WorkItem &y) {
        const uint64_t cx = cost(x), cy = cost(y);
        return cx != cy ? cx > cy : x.gen < y.gen;
    });
    uint32_t *counters = static_cast<uint32_t *>(scr);
    WorkItem *d_items = reinterpret_cast<WorkItem *>(static_cast<char *>(scr) + kStaticCounterBytes);
    WorkItem none;
    std::memset(&none, 0, sizeof(none));
    if (launch_zero_words(counters, 2, s) != hipSuccess ||
        hipMemcpyAsync(d_items, h, (size_t)k * sizeof(WorkItem), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(b->static_free, s) != hipSuccess)
        return fail(MTGP_EDEVICE);
    b->static_pending = true;
    if (launch_generate(b->d_recs, b->d_states, d_items, k, counters, none, shape, s) != hipSuccess)
        return fail(MTGP_EDEVICE);
    for (uint32_t j = 0; j < k; j++)
        b->consumed[h[j].gen] += h[j].n;
    b->last = s;
    return MTGP_OK;
}

}  // extern "C"

namespace mtgp_impl {

int batch_generate(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream, bool allow_split)
{
    if (validate_requests(b, reqs, nreq, true) != MTGP_OK)
        return fail(MTGP_EINVAL);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<WorkItem> items = items_of(reqs, nreq);
    if (items.empty())
        return MTGP_OK;
    LaunchShape shape;
    if (resolve_shape(b, items, shape) != MTGP_OK)
        return fail(MTGP_EINVAL);
    if (allow_split && b->split_rounds > 0) {
        bool long_request = false;
        for (const WorkItem &it : items) {
            const GenRecord &r = b->recs[it.gen];
            const uint32_t W = round_width(r.N, r.M, shape);
            long_request = long_request || (it.n + W - 1) / W > b->split_rounds;
        }
        if (long_request) {
            // the call as a one-off plan of jump-ahead segments, kept until the
            // next such call or the batch's destruction (each waits for the
            // batch's last stream before freeing it)
            mtgp_plan_destroy(b->eager_plan);
            b->eager_plan = nullptr;
            mtgp_plan_t *p = mtgp_batch_plan_create(b, reqs, nreq);
            if (!p) {
                const int e = mtgp_last_error();
                return e != MTGP_OK ? e : fail(MTGP_EDEVICE);
            }
            b->eager_plan = p;
            return mtgp_plan_launch(p, stream);
        }
    }
    return launch_work_items(b, items, s);
}

// The persistent generation over prepared work items on stream s: launch
// shape (override or automatic), queue order, upload through the batch's
// pinned staging, launch, consumed counters.
int launch_work_items(mtgp_batch_t *b, std::vector<WorkItem> &items, hipStream_t s)
{
    if (items.empty())
        return MTGP_OK;
    LaunchShape shape;
    if (resolve_shape(b, items, shape) != MTGP_OK)
        return fail(MTGP_EINVAL);
    finish_items(b, items, shape);
    const uint32_t nitems = (uint32_t)items.size();
    if (b->items_pending) {
        if (hipEventSynchronize(b->items_free) != hipSuccess)
            return fail(MTGP_EDEVICE);
        b->items_pending = false;
    }
    if (nitems > b->item_cap) {
        (void)hipFree(b->d_items);
        if (b->h_items)
            (void)hipHostFree(b->h_items);
        b->d_items = nullptr;
        b->h_items = nullptr;
        b->item_cap = 0;
        const uint32_t cap = std::max<uint32_t>(nitems, 1024u);
        if (hipMalloc(&b->d_items, cap * sizeof(WorkItem)) != hipSuccess ||
            hipHostMalloc(&b->h_items, cap * sizeof(WorkItem), hipHostMallocDefault) != hipSuccess)
            return fail(MTGP_ENOMEM);
        b->item_cap = cap;
    }
    std::memcpy(b->h_items, items.data(), nitems * sizeof(WorkItem));
    if (hipMemcpyAsync(b->d_items, b->h_items, nitems * sizeof(WorkItem), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(MTGP_EDEVICE);
    if (hipEventRecord(b->items_free, s) != hipSuccess)
        return fail(MTGP_EDEVICE);
    b->items_pending = true;
    WorkItem none;
    std::memset(&none, 0, sizeof(none));
    if (launch_generate(b->d_recs, b->d_states, b->d_items, nitems, b->d_counters, none, shape, s) != hipSuccess)
        return fail(MTGP_EDEVICE);
    for (const WorkItem &it : items)
        b->consumed[it.gen] += it.n;
    b->last = s;
    return MTGP_OK;
}

// ---------------------------------------------------------------------------
// Request-loop support (jump-ahead segments inside ticks)
// ---------------------------------------------------------------------------

bool split_ready(const mtgp_batch_t *b, uint32_t g)
{
    return g < b->count && b->psi_epoch[g] == b->epoch[g] + 1 && b->psi[g].deg >= 1;
}

const f2::Poly &split_psi(const mtgp_batch_t *b, uint32_t g) { return b->psi[g]; }

uint32_t gen_words(const mtgp_batch_t *b, uint32_t g) { return b->recs[g].N; }

uint32_t max_gen_words(const mtgp_batch_t *b)
{
    uint32_t m = 0;
    for (uint32_t g = 0; g < b->count; g++)
        m = std::max(m, b->recs[g].N);
    return m;
}

int prepare_annihilators(mtgp_batch_t *b, const std::vector<uint32_t> &gens) { return ensure_annihilators(b, gens); }

uint32_t poly_words(uint32_t N, uint32_t D) { return jump_poly_words(N, D); }

void poly_layout(const f2::Poly &h, uint32_t N, uint64_t *dst) { layout_poly(h, N, dst); }

std::vector<f2::Poly> segment_polys(const f2::Poly &psi, uint64_t J, uint32_t S) { return jump_polys(psi, J, S); }

LaunchShape prefix_shape(const mtgp_batch_t *b, const std::vector<uint32_t> &gens) { return raw_shape(b, gens); }

uint16_t prefix_spl(const mtgp_batch_t *b, uint32_t g, const LaunchShape &shape)
{
    return item_spl(b->recs[g].N, b->recs[g].M, shape);
}

hipError_t launch_prefix(mtgp_batch_t *b, const WorkItem *d_items, uint32_t n, const LaunchShape &shape,
                         hipStream_t s)
{
    WorkItem none;
    std::memset(&none, 0, sizeof(none));
    return launch_generate(b->d_recs, b->d_states, d_items, n, nullptr, none, shape, s);
}

}  // namespace mtgp_impl

extern "C" {

int mtgp_batch_generate_plain(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream)
{
    if (validate_requests(b, reqs, nreq, false) != MTGP_OK)
        return fail(MTGP_EINVAL);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (uint32_t i = 0; i < nreq; i++) {
        const mtgp_request &r = reqs[i];
        if (r.n == 0)
            continue;
        const GenRecord &rec = b->recs[r.gen];
        const LaunchShape shape = single_shape(rec, b->max_lds);
        WorkItem it;
        std::memset(&it, 0, sizeof(it));
        it.out = reinterpret_cast<uint64_t>(r.out);
        it.n = r.n;
        it.gen = r.gen;
        it.kind = (uint16_t)r.kind;
        it.spl = item_spl(rec.N, rec.M, shape);
        if (launch_generate(b->d_recs, b->d_states, nullptr, 1, nullptr, it, shape, s) != hipSuccess)
            return fail(MTGP_EDEVICE);
        b->consumed[r.gen] += r.n;
        b->last = s;
    }
    return MTGP_OK;
}

int mtgp_batch_set_launch(mtgp_batch_t *b, int mode, int threads, int spl, int lds_words, int grid)
{
    if (!b)
        return fail(MTGP_EINVAL);
    if (mode < 0) {
        b->have_override = false;
        return MTGP_OK;
    }
    LaunchShape s;
    s.rec_basis = (mode & kModeRecBasis) ? 1 : 0;
    s.mode = mode & ~kModeRecBasis;
    s.threads = threads;
    s.spl = spl;
    s.lds_words = lds_words > 0 ? lds_words : (s.mode == kModeChunk ? 512 : 1);
    s.grid = grid > 0 ? grid : 1;
    if (lds_words < 0 || grid < 0 || !shape_valid(s, b->max_lds))
        return fail(MTGP_EINVAL);
    s.lds_words = lds_words;
    s.grid = grid;
    b->override_shape = s;
    b->have_override = true;
    return MTGP_OK;
}

int mtgp_batch_set_split(mtgp_batch_t *b, uint32_t max_rounds)
{
    if (!b)
        return fail(MTGP_EINVAL);
    b->split_rounds = max_rounds;
    return MTGP_OK;
}

int mtgp_batch_get_state(mtgp_batch_t *b, uint32_t gen, uint32_t *host_words, uint64_t *consumed)
{
    if (!b || gen >= b->count || !host_words)
        return fail(MTGP_EINVAL);
    const GenRecord &r = b->recs[gen];
    if (hipStreamSynchronize(b->last) != hipSuccess ||
        hipMemcpy(host_words, b->d_states + r.state_off, r.N * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(MTGP_EDEVICE);
    if (consumed)
        *consumed = b->consumed[gen];
    return MTGP_OK;
}

int mtgp_batch_set_state(mtgp_batch_t *b, uint32_t gen, const uint32_t *host_words, uint64_t consumed)
{
    if (!b || gen >= b->count || !host_words)
        return fail(MTGP_EINVAL);
    const GenRecord &r = b->recs[gen];
    if (hipStreamSynchronize(b->last) != hipSuccess ||
        hipMemcpy(b->d_states + r.state_off, host_words, r.N * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
        return fail(MTGP_EDEVICE);
    b->consumed[gen] = consumed;
    b->epoch[gen]++;           // the orbit may have changed: annihilator and plans are stale
    return MTGP_OK;
}

// ---------------------------------------------------------------------------
// Plans: a fixed request list, uploaded once, its persistent launch captured
// in a HIP graph and replayed.
// ---------------------------------------------------------------------------

mtgp_plan_t *mtgp_batch_plan_create(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq)
{
    if (validate_requests(b, reqs, nreq, true) != MTGP_OK) {
        fail(MTGP_EINVAL);
        return nullptr;
    }
    mtgp_plan *p = new (std::nothrow) mtgp_plan();
    if (!p) {
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    p->b = b;
    p->items = items_of(reqs, nreq);
    if (p->items.empty() || resolve_shape(b, p->items, p->shape) != MTGP_OK) {
        delete p;
        fail(MTGP_EINVAL);
        return nullptr;
    }
    std::vector<WorkItem> prefix;
    std::vector<JumpItem> jumps;
    if (b->split_rounds > 0) {
        int rc = plan_split(p, p->items, prefix, jumps);
        // the segments change the item count: size the launch for them
        if (rc == MTGP_OK && !prefix.empty() && resolve_shape(b, p->items, p->shape) != MTGP_OK)
            rc = MTGP_EINVAL;
        if (rc != MTGP_OK) {
            plan_free(p);
            fail(rc);
            return nullptr;
        }
    }
    finish_items(b, p->items, p->shape);
    const uint32_t nitems = (uint32_t)p->items.size();
    const size_t extra = prefix.size() * sizeof(WorkItem) + jumps.size() * sizeof(JumpItem);
    char *d_extra = nullptr;
    if (hipMalloc(&p->d_items, nitems * sizeof(WorkItem) + extra) != hipSuccess ||
        hipMalloc(&p->d_counters, 2 * sizeof(uint32_t)) != hipSuccess) {
        plan_free(p);
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    d_extra = reinterpret_cast<char *>(p->d_items + nitems);
    p->d_prefix = reinterpret_cast<WorkItem *>(d_extra);
    p->nprefix = (uint32_t)prefix.size();
    p->d_jumps = reinterpret_cast<JumpItem *>(d_extra + prefix.size() * sizeof(WorkItem));
    p->jumps = jumps;
    std::vector<uint32_t> pgens;
    for (const WorkItem &it : prefix)
        pgens.push_back(it.gen);
    if (!prefix.empty()) {
        p->pshape = raw_shape(b, pgens);
        for (WorkItem &it : prefix)
            it.spl = item_spl(b->recs[it.gen].N, b->recs[it.gen].M, p->pshape);
    }
    if (hipMemcpy(p->d_items, p->items.data(), nitems * sizeof(WorkItem), hipMemcpyHostToDevice) != hipSuccess ||
        (!prefix.empty() &&
         hipMemcpy(p->d_prefix, prefix.data(), prefix.size() * sizeof(WorkItem), hipMemcpyHostToDevice) != hipSuccess) ||
        (!jumps.empty() &&
         hipMemcpy(p->d_jumps, jumps.data(), jumps.size() * sizeof(JumpItem), hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemset(p->d_counters, 0, 2 * sizeof(uint32_t)) != hipSuccess ||
        hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess) {
        plan_free(p);
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    // runs of jump items with one launch shape (the items are grouped so)
    for (uint32_t i = 0; i < (uint32_t)p->jumps.size(); i++) {
        const JumpShape a = jump_shape(p->jumps[i].N);
        if (i == 0 || a.R != jump_shape(p->jumps[i - 1].N).R || a.G != jump_shape(p->jumps[i - 1].N).G)
            p->runs.push_back(i);
    }
    p->runs.push_back((uint32_t)p->jumps.size());
    if (p->runs.size() > 2) {
        uint64_t most = 0;
        for (size_t k = 0; k + 1 < p->runs.size(); k++) {
            uint64_t work = 0;
            for (uint32_t i = p->runs[k]; i < p->runs[k + 1]; i++)
                work += (uint64_t)p->jumps[i].D * p->jumps[i].N;
            if (work > most) {
                most = work;
                p->heavy = (uint32_t)k;
            }
        }
        if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess) {
            plan_free(p);
            fail(MTGP_EDEVICE);
            return nullptr;
        }
    }
    bool ok = true;
    for (int k = 0; k < 3 && ok; k++)
        if (k != MTGP_PHASE_PREPARE || p->nprefix > 0)   // an unsplit plan has nothing to prepare
            ok = capture_phases(p, k == MTGP_PHASE_ALL ? 3 : k, p->graph[k], p->exec[k]);
    if (!ok) {
        plan_free(p);
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    return p;
}

int mtgp_plan_launch(mtgp_plan_t *p, void *stream)
{
    return mtgp_plan_launch_phase(p, MTGP_PHASE_ALL, stream);
}

int mtgp_plan_launch_phase(mtgp_plan_t *p, int phase, void *stream)
{
    if (!p || phase < MTGP_PHASE_ALL || phase > MTGP_PHASE_GENERATE)
        return fail(MTGP_EINVAL);
    for (size_t i = 0; i < p->split_gens.size(); i++)
        if (p->b->epoch[p->split_gens[i]] != p->split_epochs[i])
            return fail(MTGP_EINVAL);   // a split generator's state was replaced: the plan is stale
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->exec[phase] && hipGraphLaunch(p->exec[phase], s) != hipSuccess)
        return fail(MTGP_EDEVICE);
    if (phase != MTGP_PHASE_PREPARE)
        for (const WorkItem &it : p->items)
            p->b->consumed[it.gen] += it.n;
    p->b->last = s;
    return MTGP_OK;
}

int mtgp_batch_prepare_split(mtgp_batch_t *b, const uint32_t *gens, uint32_t count)
{
    if (!b || (count > 0 && !gens))
        return fail(MTGP_EINVAL);
    std::vector<uint32_t> g(gens, gens + count);
    for (uint32_t x : g)
        if (x >= b->count)
            return fail(MTGP_EINVAL);
    std::sort(g.begin(), g.end());
    g.erase(std::unique(g.begin(), g.end()), g.end());
    const int rc = ensure_annihilators(b, g);
    return rc == MTGP_OK ? MTGP_OK : fail(rc);
}

int mtgp_plan_describe(const mtgp_plan_t *p, mtgp_plan_info *info)
{
    if (!p || !info)
        return fail(MTGP_EINVAL);
    info->mode = p->shape.mode | (p->shape.rec_basis ? kModeRecBasis : 0);
    info->threads = (uint32_t)p->shape.threads;
    info->spl = (uint32_t)p->shape.spl;
    info->lds_words = (uint32_t)p->shape.lds_words;
    info->grid = (uint32_t)p->shape.grid;
    info->items = (uint32_t)p->items.size();
    info->jumps = (uint32_t)p->jumps.size();
    return MTGP_OK;
}

int mtgp_plan_items(const mtgp_plan_t *p, uint64_t *outs, uint64_t *ns, uint32_t cap)
{
    if (!p || (cap > 0 && (!outs || !ns)))
        return fail(MTGP_EINVAL);
    const uint32_t k = (uint32_t)std::min<size_t>(cap, p->items.size());
    for (uint32_t i = 0; i < k; i++) {
        outs[i] = p->items[i].out;
        ns[i] = p->items[i].n;
    }
    return (int)k;
}

void mtgp_plan_destroy(mtgp_plan_t *p)
{
    if (!p)
        return;
    if (p->b)
        (void)hipStreamSynchronize(p->b->last);
    plan_free(p);
}

int mtgp_batch_autotune(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream, uint32_t reps,
                        mtgp_tuning *best)
{
    if (!b || nreq == 0 || reps == 0 || validate_requests(b, reqs, nreq, true) != MTGP_OK)
        return fail(MTGP_EINVAL);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the generators' states and counters, restored after every trial
    uint32_t *d_save = nullptr;
    if (hipStreamSynchronize(b->last) != hipSuccess)
        return fail(MTGP_EDEVICE);
    if (hipMalloc(&d_save, b->state_words * sizeof(uint32_t)) != hipSuccess)
        return fail(MTGP_ENOMEM);
    if (hipMemcpy(d_save, b->d_states, b->state_words * sizeof(uint32_t), hipMemcpyDeviceToDevice) != hipSuccess) {
        (void)hipFree(d_save);
        return fail(MTGP_EDEVICE);
    }
    const std::vector<uint64_t> consumed = b->consumed;
    const bool had_override = b->have_override;
    const LaunchShape had_shape = b->override_shape;
    const uint32_t had_split = b->split_rounds;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(d_save);
        return fail(MTGP_EDEVICE);
    }

    struct Cand {
        bool automatic;
        LaunchShape shape;
        uint32_t split;
        float ms;
    };
    // mean launch time of one configuration, or a negative value if its plan
    // cannot be built
    bool device_ok = true;
    auto trial = [&](Cand &c) {
        b->have_override = !c.automatic;
        b->override_shape = c.shape;
        b->split_rounds = c.split;
        c.ms = -1.0f;
        mtgp_plan *p = mtgp_batch_plan_create(b, reqs, nreq);
        if (!p)
            return;
        bool ok = mtgp_plan_launch(p, s) == MTGP_OK && hipEventRecord(e0, s) == hipSuccess;
        for (uint32_t r = 0; ok && r < reps; r++)
            ok = mtgp_plan_launch(p, s) == MTGP_OK;
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            c.ms = ms / (float)reps;
        device_ok = device_ok && ok;
        mtgp_plan_destroy(p);
        device_ok = device_ok &&
                    hipMemcpyAsync(b->d_states, d_save, b->state_words * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                   s) == hipSuccess &&
                    hipStreamSynchronize(s) == hipSuccess;
        b->consumed = consumed;
    };

    // split limits: none, then halving from the longest request's rounds
    // (rounds of the automatic shape, in which the split limits are tried)
    std::vector<WorkItem> items = items_of(reqs, nreq);
    b->have_override = false;
    LaunchShape ds;
    if (resolve_shape(b, items, ds) != MTGP_OK)
        ds = batch_default_shape(b, items);
    b->have_override = had_override;
    uint64_t rmax = 0, rsum = 0;
    for (const WorkItem &it : items) {
        const GenRecord &r = b->recs[it.gen];
        const uint32_t W = round_width(r.N, r.M, ds);
        rmax = std::max<uint64_t>(rmax, (it.n + W - 1) / W);
        rsum += (it.n + W - 1) / W;
    }
    std::vector<Cand> tried;
    Cand c0{true, had_shape, 0, 0.0f};
    trial(c0);
    tried.push_back(c0);
    // the fair share of one unit of the automatic launch (all rounds over its
    // units), and three quarters of it: with segments about that long the
    // queue can balance the units with few jumps, where halvings of the
    // longest request can land far from it
    const uint64_t units = (uint64_t)std::max(1, ds.grid) * shape_units(ds);
    const uint64_t share = rsum / std::max<uint64_t>(1, units);
    for (const uint64_t sr : {share, share * 3 / 4}) {
        if (!device_ok || sr < 128 || sr >= rmax)
            continue;
        Cand c{true, had_shape, (uint32_t)std::min<uint64_t>(sr, UINT32_MAX), 0.0f};
        trial(c);
        tried.push_back(c);
    }
    // then seven halvings of the longest request's rounds; beyond them
    // (requests with millions of rounds) the sweep goes on while each halving
    // is the fastest configuration so far
    for (uint64_t sr = rmax / 2; sr >= 128 && tried.size() < 20 && device_ok; sr /= 2) {
        if (tried.size() >= 10) {
            const float last = tried.back().ms;
            bool fastest = last > 0;
            for (const Cand &t : tried)
                fastest = fastest && !(t.ms > 0 && t.ms < last);
            if (!fastest)
                break;
        }
        Cand c{true, had_shape, (uint32_t)sr, 0.0f};
        trial(c);
        tried.push_back(c);
    }
    // the first configuration tried wins unless a later one is at least 2 %
    // faster: timing noise then does not flip the choice between runs
    auto best_of = [&]() {
        size_t k = 0;
        for (size_t i = 0; i < tried.size(); i++)
            if (tried[i].ms > 0 && (tried[k].ms <= 0 || tried[i].ms < 0.98f * tried[k].ms))
                k = i;
        return tried[k];
    };
    // launch shapes, each at the split limit that cuts the same segment
    // lengths in steps as the best one so far (a split limit counts rounds,
    // and a round's width depends on the shape), and at half of it
    const uint32_t split = best_of().split;
    // mean round width of the request list under a shape, weighted by rounds
    auto mean_width = [&](const LaunchShape &s) {
        uint64_t steps = 0, rounds = 0;
        for (const WorkItem &it : items) {
            const GenRecord &r = b->recs[it.gen];
            const uint64_t w = round_width(r.N, r.M, s);
            steps += it.n;
            rounds += (it.n + w - 1) / w;
        }
        return rounds ? (double)steps / (double)rounds : 1.0;
    };
    const double w_auto = mean_width(ds);
    const int shapes[][3] = {{kModeChunk, 64, 2},  {kModeChunk, 256, 2}, {kModeChunk, 1024, 2},
                             {kModeChunk, 256, 1},
                             {kModeGroup, 256, 1}, {kModeGroup, 256, 2}, {kModeGroup, 512, 1},
                             {kModeGroup, 512, 2}, {kModeGroup, 1024, 1}, {kModeGroup, 128, 4},
                             {kModeWave, 256, 8}};
    for (const auto &sh : shapes) {
        if (!device_ok)
            break;
        Cand c{false, LaunchShape{}, split, 0.0f};
        c.shape.mode = sh[0];
        c.shape.threads = sh[1];
        c.shape.spl = sh[2];
        c.shape.lds_words = 0;
        c.shape.grid = 0;
        LaunchShape probe = c.shape;
        probe.lds_words = sh[0] == kModeChunk ? 512 : 1;
        probe.grid = 1;
        if (!shape_valid(probe, b->max_lds))
            continue;
        if (sh[0] == kModeChunk && !all_chunk_ok(b, items, (uint32_t)sh[2]))
            continue;
        const uint32_t eq = split == 0 ? 0u
                                       : (uint32_t)std::max(128.0, (double)split * w_auto / mean_width(c.shape));
        for (uint32_t sp : {eq, eq / 2}) {
            if (!device_ok || (sp == eq / 2 && (eq == 0 || sp < 128)))
                continue;
            c.split = sp;
            trial(c);
            tried.push_back(c);
        }
    }
    // the best so far with the other recursion-table form (the automatic
    // shape is the 256-lane workgroup form with up to 4 steps per lane)
    if (device_ok) {
        Cand c = best_of();
        if (c.automatic) {
            c.automatic = false;
            c.shape = LaunchShape{};
            c.shape.mode = kModeGroup;
            c.shape.threads = 256;
            c.shape.spl = 4;
            c.shape.lds_words = 0;
            c.shape.grid = 0;
        }
        c.shape.rec_basis = 1 - c.shape.rec_basis;
        trial(c);
        tried.push_back(c);
    }
    // a local step around the best split limit: the candidates above are a
    // factor of two apart (or fixed fractions of the fair share), and the
    // best limit often lies between them
    if (device_ok && best_of().split > 0) {
        const Cand base = best_of();
        for (const double f : {1.3, 1.0 / 1.3}) {
            Cand c = base;
            c.split = (uint32_t)std::max(128.0, std::round((double)base.split * f));
            if (!device_ok || c.split == base.split)
                continue;
            trial(c);
            tried.push_back(c);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_save);
    const Cand win = best_of();
    if (!device_ok || win.ms <= 0) {
        b->have_override = had_override;
        b->override_shape = had_shape;
        b->split_rounds = had_split;
        return fail(device_ok ? MTGP_EINVAL : MTGP_EDEVICE);
    }
    b->have_override = !win.automatic;
    b->override_shape = win.shape;
    b->split_rounds = win.split;
    if (best) {
        best->mode = win.automatic ? -1 : (win.shape.mode | (win.shape.rec_basis ? kModeRecBasis : 0));
        best->threads = win.automatic ? 0 : win.shape.threads;
        best->spl = win.automatic ? 0 : win.shape.spl;
        best->split_rounds = win.split;
        best->ms = win.ms;
        best->trials = (uint32_t)tried.size();
    }
    return MTGP_OK;
}

}  // extern "C"
