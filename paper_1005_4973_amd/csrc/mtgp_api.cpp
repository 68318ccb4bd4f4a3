// C ABI of the MTGP library (declared in include/mtgp.h): parameter
// validation, state seeding, device residency of states and parameters, and
// the launch paths (single generator, persistent batch, one launch per
// request, graph-captured plans).
#include "../../include/mtgp.h"
#include "mtgp_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
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
// A window this large (in words) takes more than half of a CU's LDS, so the
// hardware places at most one such workgroup per CU.
constexpr uint32_t kExclusiveWindow = 24000;

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
    return spl == 1 || spl == 2 || spl == 4 || spl == 6 || spl == 8 || spl == 12 || spl == 16;
}

uint32_t shape_units(const LaunchShape &s) { return s.mode == kModeGroup ? 1u : (uint32_t)(s.threads / 64); }

// LDS bytes a launch shape asks for per workgroup.
size_t shape_lds_bytes(const LaunchShape &s)
{
    return (size_t)shape_units(s) * (kUnitLdsExtra + (size_t)s.lds_words) * 4u;
}

uint32_t max_window_words(const LaunchShape &s, size_t max_lds)
{
    return (uint32_t)(max_lds / 4u / shape_units(s) - kUnitLdsExtra);
}

// Window a generator needs under a shape: 2N + lanes * item_spl words.
uint32_t window_need(const GenRecord &r, const LaunchShape &s) { return 2 * r.N + round_span(r.N, r.M, s); }

bool shape_valid(const LaunchShape &s, size_t max_lds)
{
    if (s.mode != kModeGroup && s.mode != kModeWave)
        return false;
    if (s.threads < 64 || s.threads > 1024 || s.threads % 64 != 0)
        return false;
    if (!spl_supported(s.mode, s.spl) || s.lds_words <= 0 || s.grid <= 0)
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
};

struct mtgp_batch {
    uint32_t count = 0;
    std::vector<GenRecord> recs;
    std::vector<uint64_t> consumed;
    GenRecord *d_recs = nullptr;
    uint32_t *d_states = nullptr;
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
};

struct mtgp_plan {
    mtgp_batch *b = nullptr;
    std::vector<WorkItem> items;
    WorkItem *d_items = nullptr;
    uint32_t *d_counters = nullptr;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    LaunchShape shape;
};

namespace {

// Default persistent launch shape for a batch (when no override is set):
// - at most as many requests as CUs: one 256-lane workgroup per generator
//   and one workgroup per CU (an exclusive LDS window), because each
//   generator's rounds are latency-bound and two workgroups on one CU would
//   share its issue slots;
// - more requests: 256-lane workgroups with the smallest window that fits
//   every request, so several generators share each CU.
LaunchShape batch_default_shape(const mtgp_batch *b, const std::vector<WorkItem> &items)
{
    LaunchShape s;
    s.mode = kModeGroup;
    s.threads = 256;
    s.spl = 4;
    s.grid = 1;
    uint32_t need = 0;
    for (const WorkItem &it : items)
        need = std::max(need, window_need(b->recs[it.gen], s));
    s.lds_words = 1;
    const uint32_t cap = max_window_words(s, b->max_lds);
    if (items.size() <= (size_t)b->cu_count)
        s.lds_words = (int)std::min(cap, std::max(need, kExclusiveWindow));
    else
        s.lds_words = (int)std::min(cap, std::max(need, 4096u));
    s.grid = (int)std::min<uint64_t>(items.size(), resident_groups(s, b->cu_count));
    return s;
}

// Resolve the launch shape for a set of items: override (with automatic
// window and grid filled in) or default; validated against every item.
int resolve_shape(const mtgp_batch *b, const std::vector<WorkItem> &items, LaunchShape &out)
{
    LaunchShape s;
    if (b->have_override) {
        s = b->override_shape;
        if (s.lds_words == 0) {
            uint32_t need = 0;
            for (const WorkItem &it : items)
                need = std::max(need, window_need(b->recs[it.gen], s));
            s.lds_words = (int)need;
        }
        if (s.grid == 0) {
            const uint64_t units = shape_units(s);
            const uint64_t want = (items.size() + units - 1) / units;
            s.grid = (int)std::min<uint64_t>(want, resident_groups(s, b->cu_count));
        }
    } else {
        s = batch_default_shape(b, items);
    }
    if (!shape_valid(s, b->max_lds))
        return MTGP_EINVAL;
    for (const WorkItem &it : items)
        if ((uint32_t)s.lds_words < window_need(b->recs[it.gen], s))
            return MTGP_EINVAL;
    out = s;
    return MTGP_OK;
}

int validate_requests(const mtgp_batch *b, const mtgp_request *reqs, uint32_t nreq, bool unique)
{
    if (!b || (nreq > 0 && !reqs))
        return MTGP_EINVAL;
    std::vector<uint8_t> seen(unique ? b->count : 0, 0);
    for (uint32_t i = 0; i < nreq; i++) {
        const mtgp_request &r = reqs[i];
        if (r.gen >= b->count || r.kind > 2 || check_out(r.out, r.n) != MTGP_OK)
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
    for (WorkItem &it : items)
        it.spl = item_spl(b->recs[it.gen].N, b->recs[it.gen].M, s);
    auto cost = [&](const WorkItem &it) {
        const GenRecord &r = b->recs[it.gen];
        const uint64_t w = round_width(r.N, r.M, s);
        return (it.n + w - 1) / w * (uint64_t)it.spl;
    };
    std::stable_sort(items.begin(), items.end(),
                     [&](const WorkItem &x, const WorkItem &y) { return cost(x) > cost(y); });
}

void batch_free(mtgp_batch *b)
{
    if (!b)
        return;
    hipFree(b->d_recs);
    hipFree(b->d_states);
    hipFree(b->d_counters);
    hipFree(b->d_items);
    if (b->h_items)
        hipHostFree(b->h_items);
    if (b->items_free)
        hipEventDestroy(b->items_free);
    delete b;
}

void plan_free(mtgp_plan *p)
{
    if (!p)
        return;
    if (p->exec)
        hipGraphExecDestroy(p->exec);
    if (p->graph)
        hipGraphDestroy(p->graph);
    if (p->capture)
        hipStreamDestroy(p->capture);
    hipFree(p->d_items);
    hipFree(p->d_counters);
    delete p;
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
        hipFree(g->d_rec);
        hipFree(g->d_state);
        delete g;
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    if (hipMemcpy(g->d_rec, &g->rec, sizeof(GenRecord), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_state, words.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(g->d_rec);
        hipFree(g->d_state);
        delete g;
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    g->max_lds = device_max_lds();
    g->shape = single_shape(g->rec, g->max_lds);
    return g;
}

static int generate_kind(mtgp_t *g, size_t n, void *out, void *stream, uint32_t kind)
{
    if (!g)
        return fail(MTGP_EINVAL);
    if (check_out(out, n) != MTGP_OK)
        return fail(MTGP_EINVAL);
    if (n == 0)
        return MTGP_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
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

void mtgp_destroy(mtgp_t *g)
{
    if (!g)
        return;
    hipStreamSynchronize(g->last);
    hipFree(g->d_rec);
    hipFree(g->d_state);
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
    s.mode = mode;
    s.threads = mode == kModeGroup ? threads : 64;
    s.spl = spl;
    s.grid = 1;
    s.lds_words = 1;
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
    b->consumed.assign(count, 0);
    uint64_t off = 0;
    for (uint32_t i = 0; i < count; i++) {
        b->recs[i] = make_record(&ps[i], off);
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
        hipMalloc(&b->d_states, off * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&b->d_counters, 2 * sizeof(uint32_t)) != hipSuccess) {
        batch_free(b);
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    if (hipMemcpy(b->d_recs, b->recs.data(), count * sizeof(GenRecord), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_states, words.data(), off * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->d_counters, 0, 2 * sizeof(uint32_t)) != hipSuccess ||
        hipEventCreateWithFlags(&b->items_free, hipEventDisableTiming) != hipSuccess) {
        batch_free(b);
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    return b;
}

uint32_t mtgp_batch_size(const mtgp_batch_t *b) { return b ? b->count : 0; }

void mtgp_batch_destroy(mtgp_batch_t *b)
{
    if (!b)
        return;
    hipStreamSynchronize(b->last);
    batch_free(b);
}

int mtgp_batch_generate(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream)
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
    finish_items(b, items, shape);
    const uint32_t nitems = (uint32_t)items.size();
    if (b->items_pending) {
        if (hipEventSynchronize(b->items_free) != hipSuccess)
            return fail(MTGP_EDEVICE);
        b->items_pending = false;
    }
    if (nitems > b->item_cap) {
        hipFree(b->d_items);
        if (b->h_items)
            hipHostFree(b->h_items);
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
    s.mode = mode;
    s.threads = threads;
    s.spl = spl;
    s.lds_words = lds_words > 0 ? lds_words : 1;
    s.grid = grid > 0 ? grid : 1;
    if (lds_words < 0 || grid < 0 || !shape_valid(s, b->max_lds))
        return fail(MTGP_EINVAL);
    s.lds_words = lds_words;
    s.grid = grid;
    b->override_shape = s;
    b->have_override = true;
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
    finish_items(b, p->items, p->shape);
    const uint32_t nitems = (uint32_t)p->items.size();
    if (hipMalloc(&p->d_items, nitems * sizeof(WorkItem)) != hipSuccess ||
        hipMalloc(&p->d_counters, 2 * sizeof(uint32_t)) != hipSuccess) {
        plan_free(p);
        fail(MTGP_ENOMEM);
        return nullptr;
    }
    if (hipMemcpy(p->d_items, p->items.data(), nitems * sizeof(WorkItem), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(p->d_counters, 0, 2 * sizeof(uint32_t)) != hipSuccess ||
        hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess) {
        plan_free(p);
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    WorkItem none;
    std::memset(&none, 0, sizeof(none));
    bool ok = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const hipError_t le = launch_generate(b->d_recs, b->d_states, p->d_items, nitems, p->d_counters, none,
                                              p->shape, p->capture);
        const hipError_t ce = hipStreamEndCapture(p->capture, &p->graph);
        ok = le == hipSuccess && ce == hipSuccess && p->graph != nullptr;
    }
    if (ok)
        ok = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        plan_free(p);
        fail(MTGP_EDEVICE);
        return nullptr;
    }
    return p;
}

int mtgp_plan_launch(mtgp_plan_t *p, void *stream)
{
    if (!p)
        return fail(MTGP_EINVAL);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipGraphLaunch(p->exec, s) != hipSuccess)
        return fail(MTGP_EDEVICE);
    for (const WorkItem &it : p->items)
        p->b->consumed[it.gen] += it.n;
    p->b->last = s;
    return MTGP_OK;
}

void mtgp_plan_destroy(mtgp_plan_t *p)
{
    if (!p)
        return;
    if (p->b)
        hipStreamSynchronize(p->b->last);
    plan_free(p);
}

}  // extern "C"
