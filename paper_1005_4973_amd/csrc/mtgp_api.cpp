// C ABI of the MTGP library (declared in include/mtgp.h): parameter
// validation, state seeding, device residency of states and parameters, and
// the launch paths (single generator, persistent batch, one launch per
// request).
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

constexpr uint32_t kMinMexp = 65;       // N >= 3
constexpr uint32_t kMaxMexp = 65536;    // N <= 2048
constexpr int kMaxLdsWords = 16384 - 64;  // default window: 64 KiB per workgroup incl. tables
constexpr size_t kLdsPerCu = 160u * 1024u;  // gfx950 LDS per compute unit

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

// Launch shape for one generator alone on the GPU: one workgroup with as
// many lanes as the round width N - M allows (up to 1024, two steps per lane
// beyond that) and the largest LDS window.
LaunchShape single_shape(uint32_t N, uint32_t M)
{
    LaunchShape s;
    s.mode = kModeGroup;
    const uint32_t wfull = N - M;
    s.spl = wfull <= 1024 ? 1 : 2;
    uint32_t lanes = (wfull + s.spl - 1) / s.spl;
    lanes = (lanes + 63u) / 64u * 64u;
    s.threads = (int)std::min<uint32_t>(1024u, std::max<uint32_t>(64u, lanes));
    s.lds_words = kMaxLdsWords;
    s.grid = 1;
    return s;
}

bool spl_supported(int mode, int spl)
{
    if (mode == kModeGroup)
        return spl == 1 || spl == 2 || spl == 4;
    return spl == 1 || spl == 2 || spl == 4 || spl == 6 || spl == 8 || spl == 12 || spl == 16;
}

// LDS bytes a launch shape asks for per workgroup.
size_t shape_lds_bytes(const LaunchShape &s)
{
    const size_t per = (size_t)(64 + s.lds_words) * 4;
    return s.mode == kModeGroup ? per : per * (size_t)(s.threads / 64);
}

// Largest LDS window the items of a launch need: 2N + lanes*spl words each.
uint32_t window_need(const std::vector<GenRecord> &recs, const std::vector<uint32_t> &gens, const LaunchShape &s)
{
    uint32_t need = 0;
    for (uint32_t g : gens)
        need = std::max<uint32_t>(need, 2 * recs[g].N + round_span(s));
    return need;
}

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

int check_out(const void *out, size_t n)
{
    if (n == 0)
        return MTGP_OK;
    if (out == nullptr || (reinterpret_cast<uintptr_t>(out) & 3u) != 0)
        return MTGP_EINVAL;
    return MTGP_OK;
}

// Largest dynamic LDS a workgroup may use on the current device; kernels are
// opted in to it once per process.
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
    if (lim > kLdsPerCu)
        lim = kLdsPerCu;
    if (lim > 65536 && opt_in_lds(lim) != hipSuccess)
        lim = 65536;
    cached = lim;
    return cached;
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
    g->shape = single_shape(N, g->rec.M);
    g->max_lds = device_max_lds();
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
    it.kind = kind;
    hipError_t e = launch_generate(g->d_rec, g->d_state, nullptr, 1, nullptr, it, g->shape, s);
    if (e != hipSuccess)
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

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

static void batch_free(mtgp_batch *b)
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

static int validate_requests(mtgp_batch *b, const mtgp_request *reqs, uint32_t nreq, bool unique)
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

// Default persistent launch shape for a batch: 256-lane workgroups, up to two
// steps per lane (round width up to 512), an LDS window that holds the
// largest state twice plus a round, and as many resident workgroups as fit.
static LaunchShape batch_shape(mtgp_batch *b, const std::vector<uint32_t> &gens)
{
    LaunchShape s;
    s.mode = kModeGroup;
    s.threads = 256;
    s.spl = 2;
    s.grid = 1;
    const uint32_t need = window_need(b->recs, gens, s);
    uint32_t L = std::max<uint32_t>(need, 4096u);
    s.lds_words = (int)L;
    const size_t lds_bytes = shape_lds_bytes(s);
    const size_t by_lds = std::max<size_t>(1u, kLdsPerCu / lds_bytes);
    const size_t by_waves = 32u / (size_t)(s.threads / 64);
    const size_t per_cu = std::min(by_lds, by_waves);
    s.grid = (int)std::min<uint64_t>(gens.size(), (uint64_t)b->cu_count * per_cu);
    return s;
}

int mtgp_batch_generate(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream)
{
    if (validate_requests(b, reqs, nreq, true) != MTGP_OK)
        return fail(MTGP_EINVAL);
    hipStream_t s = static_cast<hipStream_t>(stream);
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
        it.kind = reqs[i].kind;
        items.push_back(it);
    }
    if (items.empty())
        return MTGP_OK;
    std::vector<uint32_t> gens;
    gens.reserve(items.size());
    for (const WorkItem &it : items)
        gens.push_back(it.gen);
    LaunchShape shape = b->have_override ? b->override_shape : batch_shape(b, gens);
    if (b->have_override) {
        if (shape.lds_words == 0)
            shape.lds_words = (int)window_need(b->recs, gens, shape);
        if (shape.grid == 0) {
            const size_t by_lds = std::max<size_t>(1u, kLdsPerCu / shape_lds_bytes(shape));
            const size_t by_waves = 32u / (size_t)(shape.threads / 64);
            const size_t units = shape.mode == kModeGroup ? 1 : (size_t)(shape.threads / 64);
            const uint64_t want = (items.size() + units - 1) / units;
            shape.grid = (int)std::min<uint64_t>(want, (uint64_t)b->cu_count * std::min(by_lds, by_waves));
        }
    }
    if (!shape_valid(shape, b->max_lds) || (uint32_t)shape.lds_words < window_need(b->recs, gens, shape))
        return fail(MTGP_EINVAL);
    // longest critical path first: rounds = ceil(n / W)
    std::stable_sort(items.begin(), items.end(), [&](const WorkItem &x, const WorkItem &y) {
        const uint64_t wx = round_width(b->recs[x.gen].N, b->recs[x.gen].M, shape);
        const uint64_t wy = round_width(b->recs[y.gen].N, b->recs[y.gen].M, shape);
        return (x.n + wx - 1) / wx > (y.n + wy - 1) / wy;
    });
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
        WorkItem it;
        std::memset(&it, 0, sizeof(it));
        it.out = reinterpret_cast<uint64_t>(r.out);
        it.n = r.n;
        it.gen = r.gen;
        it.kind = r.kind;
        const LaunchShape shape = single_shape(rec.N, rec.M);
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

int mtgp_set_launch(mtgp_t *g, int mode, int threads, int spl, int lds_words)
{
    if (!g)
        return fail(MTGP_EINVAL);
    if (mode < 0) {
        g->shape = single_shape(g->rec.N, g->rec.M);
        return MTGP_OK;
    }
    LaunchShape s;
    s.mode = mode;
    s.threads = mode == kModeGroup ? threads : 64;
    s.spl = spl;
    s.grid = 1;
    s.lds_words = lds_words > 0 ? lds_words : kMaxLdsWords;
    const uint32_t need = 2 * g->rec.N + round_span(s);
    if (!shape_valid(s, g->max_lds) || (uint32_t)s.lds_words < need)
        return fail(MTGP_EINVAL);
    g->shape = s;
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

}  // extern "C"
