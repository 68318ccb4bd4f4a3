// Continuous-batching request loop over a batch's resident generators.
//
// Requests (generator, kind, n) are queued by the caller and admitted in
// arrival order while their outputs fit the output arena (a free range from
// a two-level segregated-fit index, mtgp_arena.h: constant time, and it fails
// only when no free range can hold the request; a request that does not fit
// waits, and so do the ones behind it). Every
// scheduling step retires ticks whose completion event has fired, admits
// what fits, and launches ticks while fewer than `depth` are in flight. A
// tick advances every generator that has admitted work by up to `chunk`
// outputs of its oldest unfinished request, in one persistent batched launch
// (mtgp_batch_generate); consecutive chunks of one generator stay in stream
// order, so each request gets exactly the stream segment it would get alone,
// and requests that arrive while others run join at the next tick.
//
// Jump-ahead (mtgp_server_set_split; refused for now, see kSplitTicksEnabled):
// a long request on a generator whose orbit annihilator psi is cached becomes
// S segments of J outputs that advance together, one chunk each per tick, each
// from its own state buffer (a work item reading its start state from that
// buffer and writing its end state back there). The tick that splits a request
// first runs the raw prefix of the generator's current state and the jump
// correlations that give the segments' start states (segment 0's by the
// polynomial 1, a copy); the last segment's final chunk writes the generator's
// state. The jump polynomials x^{kJ} mod psi depend only on psi, J and k, so
// host worker threads compute them while the request still advances by plain
// chunks. Their words and the tick's prefix and jump items go up through a
// ring of pinned and device memory whose blocks are released as ticks retire,
// in order; nothing in the loop allocates device memory or waits for the
// device.
#include "../../include/mtgp.h"
#include "mtgp_arena.h"
#include "mtgp_ridmap.h"
#include "mtgp_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

using mtgp_impl::JumpItem;
using mtgp_impl::LaunchShape;
using mtgp_impl::WorkItem;
namespace f2 = mtgp_impl::f2;

namespace {

// Jump-ahead inside ticks is refused (mtgp_server_set_split); the CPU
// self-test of the tick logic over a stand-in device builds this file with
// MTGP_SERVE_SPLIT_TICKS=1. The library build never sets it.
#ifndef MTGP_SERVE_SPLIT_TICKS
#define MTGP_SERVE_SPLIT_TICKS 0
#endif
constexpr bool kSplitTicksEnabled = MTGP_SERVE_SPLIT_TICKS != 0;

// Jump polynomials of one generator for segments of J outputs, laid out for
// the jump kernel: entry 0 is the polynomial 1 (segment 0's copy), entry k
// is x^{kJ} mod psi, each pw words.
struct PolyJob {
    uint32_t gen = 0, N = 0, S = 0, D = 0, pw = 0;
    uint64_t J = 0;
    f2::Poly psi;
    std::vector<uint64_t> words;
    bool done = false;   // guarded by the server's job mutex
};

struct Req {
    Req(uint64_t rid_, uint32_t gen_, uint32_t kind_, uint64_t n_) : rid(rid_), gen(gen_), kind(kind_), n(n_) {}
    // a pooled request for a new submission: every field as the constructor
    // leaves it (the segment vectors keep their capacity)
    void reset(uint64_t rid_, uint32_t gen_, uint32_t kind_, uint64_t n_)
    {
        rid = rid_;
        gen = gen_;
        kind = kind_;
        n = n_;
        next = nullptr;
        offset = 0;
        blk = 0;
        scheduled = 0;
        finished = 0;
        job.reset();
        split = false;
        S = 0;
        slot = 0;
        base = 0;
        J = 0;
        seg_len.clear();
        seg_sched.clear();
    }
    uint64_t rid;
    uint32_t gen;
    uint32_t kind;
    uint64_t n;
    Req *next = nullptr;     // the generator's next admitted request
    uint64_t offset = 0;     // byte offset of its outputs in the arena
    uint32_t blk = 0;        // its block in the arena index
    uint64_t scheduled = 0;  // outputs put in ticks
    uint64_t finished = 0;   // outputs whose tick completed
    // jump-ahead
    std::shared_ptr<PolyJob> job;   // polynomials requested (null: none)
    bool split = false;
    uint32_t S = 0, slot = 0;
    uint64_t base = 0;              // request position where segment 0 starts
    uint64_t J = 0;
    std::vector<uint64_t> seg_len, seg_sched;
};

// A generator's admitted, unfinished requests in arrival order (an intrusive
// list), and the oldest of them with outputs not yet put in a tick.
struct GenQ {
    Req *head = nullptr, *tail = nullptr;
    Req *sched = nullptr;
    bool ready = false;   // listed in the server's ready generators
};

struct Tick {
    hipEvent_t done;
    std::vector<std::pair<Req *, uint64_t>> chunks;
    int64_t ring_off = -1;   // staging block of this tick (-1: none)
    uint64_t ring_len = 0;
};

}  // namespace

struct mtgp_server {
    mtgp_batch_t *b = nullptr;
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    uint64_t chunk = 0;
    uint32_t depth = 0;
    hipStream_t stream = nullptr;
    std::unique_ptr<mtgp_impl::ArenaIndex> index;         // free ranges of the arena, in kAlign units
    std::deque<Req *> waiting;                             // submitted, not admitted
    std::vector<GenQ> gq;                                  // per generator: admitted, unfinished
    std::vector<uint32_t> ready, ready_next;               // generators with outputs to put in ticks
    uint64_t active = 0;                                   // admitted, unfinished requests
    std::vector<Req *> req_pool;                           // released requests, for reuse
    std::deque<Tick> inflight;
    std::vector<hipEvent_t> spare_events;
    mtgp_impl::RidMap<Req> completed;                      // rid -> finished, not released
    std::deque<mtgp_completion> unreported;                // finished, not yet returned by poll
    std::vector<WorkItem> items;
    // jump-ahead
    uint64_t split_min = 0;
    uint32_t split_max = 0, seg_chunks = 0, slots = 0, nmax = 0;
    uint32_t *d_pool = nullptr;                // slots x split_max x nmax state words
    std::vector<uint32_t> free_slots;
    char *d_ring = nullptr, *h_ring = nullptr; // staging ring (device, pinned host), same offsets
    uint64_t ring_bytes = 0, ring_head = 0;
    std::mutex job_mu;
    std::condition_variable job_cv;
    std::deque<std::shared_ptr<PolyJob>> jobs;
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace {

constexpr uint64_t kAlign = 256;   // output regions start on 256-byte boundaries

uint64_t round_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

uint64_t align256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

void job_worker(mtgp_server *s)
{
    for (;;) {
        std::shared_ptr<PolyJob> job;
        {
            std::unique_lock<std::mutex> lk(s->job_mu);
            s->job_cv.wait(lk, [&] { return s->stop || !s->jobs.empty(); });
            if (s->stop)
                return;
            job = s->jobs.front();
            s->jobs.pop_front();
        }
        std::vector<uint64_t> w((size_t)job->S * job->pw, 0);
        mtgp_impl::poly_layout(f2::Poly::one(), job->N, w.data());
        const std::vector<f2::Poly> h = mtgp_impl::segment_polys(job->psi, job->J, job->S);
        for (uint32_t k = 1; k < job->S; k++)
            mtgp_impl::poly_layout(h[k - 1], job->N, w.data() + (size_t)k * job->pw);
        std::lock_guard<std::mutex> lk(s->job_mu);
        job->words.swap(w);
        job->done = true;
    }
}

bool job_done(mtgp_server *s, const std::shared_ptr<PolyJob> &job)
{
    std::lock_guard<std::mutex> lk(s->job_mu);
    return job->done;
}

// A block of `bytes` in the staging ring behind the blocks of the ticks still
// in flight, which retire in order: the live blocks run from the oldest
// one's start (tail) to ring_head, wrapping at the end. False when it does
// not fit now.
bool ring_take(mtgp_server *s, uint64_t bytes, uint64_t *off)
{
    bytes = align256(bytes);
    if (bytes > s->ring_bytes)
        return false;
    int64_t tail = -1;
    for (const Tick &t : s->inflight)
        if (t.ring_off >= 0) {
            tail = t.ring_off;
            break;
        }
    uint64_t at;
    if (tail < 0)
        at = 0;   // nothing live
    else if (s->ring_head > (uint64_t)tail)
        // live blocks in [tail, head): room after head, else from 0 to tail
        at = s->ring_head + bytes <= s->ring_bytes ? s->ring_head : (bytes <= (uint64_t)tail ? 0 : UINT64_MAX);
    else
        // wrapped: live blocks in [tail, end) and [0, head), room in [head, tail)
        at = s->ring_head + bytes <= (uint64_t)tail ? s->ring_head : UINT64_MAX;
    if (at == UINT64_MAX)
        return false;
    *off = at;
    s->ring_head = at + bytes;
    return true;
}

// Queue the jump polynomials for r's generator when r qualifies for a split.
void maybe_request_polys(mtgp_server *s, Req *r)
{
    if (s->split_min == 0 || r->job || r->split || r->n - r->scheduled < s->split_min ||
        !mtgp_impl::split_ready(s->b, r->gen))
        return;
    auto job = std::make_shared<PolyJob>();
    job->gen = r->gen;
    job->N = mtgp_impl::gen_words(s->b, r->gen);
    job->psi = mtgp_impl::split_psi(s->b, r->gen);
    job->D = (uint32_t)job->psi.deg;
    job->pw = mtgp_impl::poly_words(job->N, job->D);
    job->J = (uint64_t)s->seg_chunks * s->chunk;
    // as many segments as the request has left now (fewer later)
    job->S = (uint32_t)std::min<uint64_t>(s->split_max, (r->n - r->scheduled + job->J - 1) / job->J);
    if (job->S < 2)
        return;
    r->job = job;
    {
        std::lock_guard<std::mutex> lk(s->job_mu);
        s->jobs.push_back(job);
    }
    s->job_cv.notify_one();
}

struct SplitStart {
    Req *r;
    uint32_t S;
    uint64_t raw_off, poly_off;   // device ring offsets of its raw words and polynomials
};

int launch_tick(mtgp_server *s)
{
    Tick t;
    s->items.clear();
    std::vector<SplitStart> starts;
    auto add_item = [&](Req *r, uint64_t pos, uint64_t k, uint64_t src, uint16_t flags) {
        WorkItem it;
        std::memset(&it, 0, sizeof(it));
        it.out = reinterpret_cast<uint64_t>(s->arena + r->offset + 4u * pos);
        it.n = k;
        it.gen = r->gen;
        it.kind = (uint16_t)(r->kind | flags);
        it.src = src;
        s->items.push_back(it);
        t.chunks.emplace_back(r, k);
    };
    // requests to split in this tick: polynomials ready, a state slot free,
    // two or more segments' worth left (a generator's oldest request with
    // outputs left to schedule only)
    if (s->split_min > 0)
        for (uint32_t g : s->ready) {
            Req *r = s->gq[g].sched;
            if (!r->split && r->job && s->free_slots.size() > starts.size() && job_done(s, r->job)) {
                const uint64_t left = r->n - r->scheduled;
                const uint64_t S = std::min<uint64_t>(r->job->S, (left + r->job->J - 1) / r->job->J);
                if (left >= s->split_min && S >= 2)
                    starts.push_back(SplitStart{r, (uint32_t)S, 0, 0});
                else
                    r->job.reset();
            }
        }
    uint64_t ring_off = 0, ring_len = 0;
    if (!starts.empty()) {
        // staging block: polynomials, prefix items and jump items (uploaded),
        // then each start's raw words (device only)
        uint64_t bytes = 0;
        for (SplitStart &st : starts) {
            st.poly_off = bytes;
            bytes += (uint64_t)st.S * st.r->job->pw * 8u;
        }
        const uint64_t prefix_off = align256(bytes);
        const uint64_t jump_off = align256(prefix_off + starts.size() * sizeof(WorkItem));
        uint64_t nj = 0;
        for (const SplitStart &st : starts)
            nj += st.S;
        const uint64_t upload = jump_off + nj * sizeof(JumpItem);
        bytes = align256(upload);
        for (SplitStart &st : starts) {
            st.raw_off = bytes;
            bytes = align256(bytes + (uint64_t)(st.r->job->D + st.r->job->N) * 4u);
        }
        if (!ring_take(s, bytes, &ring_off)) {
            starts.clear();   // no room now: these requests go on by plain chunks
        } else {
            ring_len = bytes;
            char *h = s->h_ring + ring_off;
            char *d = s->d_ring + ring_off;
            std::vector<uint32_t> pgens;
            WorkItem *pre = reinterpret_cast<WorkItem *>(h + prefix_off);
            std::vector<JumpItem> jumps;
            for (size_t i = 0; i < starts.size(); i++) {
                SplitStart &st = starts[i];
                Req *r = st.r;
                const PolyJob &job = *r->job;
                std::memcpy(h + st.poly_off, job.words.data(), (size_t)st.S * job.pw * 8u);
                std::memset(&pre[i], 0, sizeof(WorkItem));
                pre[i].out = reinterpret_cast<uint64_t>(d + st.raw_off);
                pre[i].n = job.D - 1;
                pre[i].gen = r->gen;
                pre[i].kind = mtgp_impl::kKindRaw | mtgp_impl::kKeepState;
                pgens.push_back(r->gen);
                r->slot = s->free_slots.back();
                s->free_slots.pop_back();
                uint32_t *pool = s->d_pool + (size_t)r->slot * s->split_max * s->nmax;
                for (uint32_t k = 0; k < st.S; k++) {
                    JumpItem ji;
                    std::memset(&ji, 0, sizeof(ji));
                    ji.raw = reinterpret_cast<uint64_t>(d + st.raw_off);
                    ji.poly = reinterpret_cast<uint64_t>(d + st.poly_off + (size_t)k * job.pw * 8u);
                    ji.out = reinterpret_cast<uint64_t>(pool + (size_t)k * s->nmax);
                    ji.D = k == 0 ? 1u : job.D;
                    ji.N = job.N;
                    jumps.push_back(ji);
                }
                r->split = true;
                r->S = st.S;
                r->J = job.J;
                r->base = r->scheduled;
                const uint64_t left = r->n - r->scheduled;
                r->seg_len.assign(st.S, 0);
                r->seg_sched.assign(st.S, 0);
                // S - 1 segments of J outputs and the rest in the last one (longer
                // than J when the polynomials were made for fewer segments)
                for (uint32_t k = 0; k < st.S; k++)
                    r->seg_len[k] = k + 1 < st.S ? r->J : left - (uint64_t)(st.S - 1) * r->J;
                r->job.reset();
            }
            // the jump kernel is launched once per lane width and word-group count
            mtgp_impl::group_jumps_by_shape(jumps);
            std::memcpy(h + jump_off, jumps.data(), jumps.size() * sizeof(JumpItem));
            const LaunchShape pshape = mtgp_impl::prefix_shape(s->b, pgens);
            for (size_t i = 0; i < starts.size(); i++)
                pre[i].spl = mtgp_impl::prefix_spl(s->b, pre[i].gen, pshape);
            if (hipMemcpyAsync(d, h, upload, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
                mtgp_impl::launch_prefix(s->b, reinterpret_cast<const WorkItem *>(d + prefix_off),
                                         (uint32_t)starts.size(), pshape, s->stream) != hipSuccess ||
                mtgp_impl::launch_jumps(reinterpret_cast<const JumpItem *>(d + jump_off), jumps.data(),
                                        (uint32_t)jumps.size(), s->stream) != hipSuccess)
                return MTGP_EDEVICE;
        }
    }
    // one chunk per ready generator from its oldest request with outputs left
    // (or one chunk of every segment of a split one); a request fully put in
    // ticks passes the turn to the next one from the following tick on
    s->ready_next.clear();
    for (uint32_t g : s->ready) {
        GenQ &q = s->gq[g];
        Req *r = q.sched;
        if (r->split) {
            uint32_t *pool = s->d_pool + (size_t)r->slot * s->split_max * s->nmax;
            for (uint32_t k = 0; k < r->S; k++) {
                const uint64_t left = r->seg_len[k] - r->seg_sched[k];
                if (left == 0)
                    continue;
                const uint64_t c = std::min(s->chunk, left);
                const bool last = r->seg_sched[k] + c == r->seg_len[k];
                // a segment's end state goes back to its buffer; at its end it is
                // dropped, except the last segment's, which is the generator's
                const uint16_t flags = !last ? mtgp_impl::kStateToSrc
                                             : (k + 1 == r->S ? (uint16_t)0 : mtgp_impl::kKeepState);
                add_item(r, r->base + (uint64_t)k * r->J + r->seg_sched[k], c,
                         reinterpret_cast<uint64_t>(pool + (size_t)k * s->nmax), flags);
                r->seg_sched[k] += c;
                r->scheduled += c;
            }
        } else {
            const uint64_t k = std::min(s->chunk, r->n - r->scheduled);
            add_item(r, r->scheduled, k, 0, 0);
            r->scheduled += k;
            maybe_request_polys(s, r);
        }
        if (r->scheduled == r->n)
            q.sched = r->next;   // admitted later, so nothing of it is scheduled yet
        if (q.sched)
            s->ready_next.push_back(g);
        else
            q.ready = false;
    }
    s->ready.swap(s->ready_next);
    if (t.chunks.empty())
        return MTGP_OK;
    if (s->spare_events.empty()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return MTGP_EDEVICE;
        s->spare_events.push_back(e);
    }
    t.done = s->spare_events.back();
    const int rc = mtgp_impl::launch_work_items(s->b, s->items, s->stream);
    if (rc != MTGP_OK)
        return rc;
    if (hipEventRecord(t.done, s->stream) != hipSuccess)
        return MTGP_EDEVICE;
    s->spare_events.pop_back();
    if (ring_len) {
        t.ring_off = (int64_t)ring_off;
        t.ring_len = ring_len;
    }
    s->inflight.push_back(std::move(t));
    return MTGP_OK;
}

bool has_unscheduled(const mtgp_server *s) { return !s->ready.empty(); }

Req *new_req(mtgp_server *s, const mtgp_server_request &q)
{
    Req *r;
    if (!s->req_pool.empty()) {
        r = s->req_pool.back();
        s->req_pool.pop_back();
        r->reset(q.rid, q.gen, q.kind, q.n);
    } else {
        r = new (std::nothrow) Req{q.rid, q.gen, q.kind, q.n};
    }
    return r;
}

// Put r at the end of its generator's queue (admission).
void gq_push(mtgp_server *s, Req *r)
{
    GenQ &q = s->gq[r->gen];
    r->next = nullptr;
    if (q.tail)
        q.tail->next = r;
    else
        q.head = r;
    q.tail = r;
    if (!q.sched)
        q.sched = r;
    if (!q.ready) {
        q.ready = true;
        s->ready.push_back(r->gen);
    }
    s->active++;
}

// Take finished r out of its generator's queue (it is the head whenever
// requests finish in arrival order, which one chunk per generator per tick
// keeps; the walk covers any other case).
void gq_remove(mtgp_server *s, Req *r)
{
    GenQ &q = s->gq[r->gen];
    Req *prev = nullptr, *x = q.head;
    for (; x && x != r; x = x->next)
        prev = x;
    if (!x)
        return;   // not queued (cannot happen: admitted requests stay queued until they finish)
    (prev ? prev->next : q.head) = r->next;
    if (q.tail == r)
        q.tail = prev;
    r->next = nullptr;
    s->active--;
}

}  // namespace

extern "C" {

mtgp_server_t *mtgp_server_create(mtgp_batch_t *b, void *arena, uint64_t arena_bytes, uint64_t chunk,
                                  uint32_t depth, void *stream)
{
    if (!b || !arena || arena_bytes < kAlign || chunk == 0 || depth == 0 ||
        (reinterpret_cast<uintptr_t>(arena) % kAlign) != 0)
        return nullptr;
    mtgp_server *s = new (std::nothrow) mtgp_server();
    if (!s)
        return nullptr;
    s->b = b;
    s->arena = static_cast<char *>(arena);
    s->arena_bytes = arena_bytes / kAlign * kAlign;
    s->chunk = chunk & ~(uint64_t)1;   // even, so chunks of normal requests hold whole pairs
    if (s->chunk == 0)
        s->chunk = 2;
    s->depth = depth;
    s->stream = static_cast<hipStream_t>(stream);
    s->index.reset(new (std::nothrow) mtgp_impl::ArenaIndex(s->arena_bytes / kAlign));
    if (!s->index) {
        delete s;
        return nullptr;
    }
    s->gq.resize(mtgp_batch_size(b));
    return s;
}

int mtgp_server_submit(mtgp_server_t *s, const mtgp_server_request *reqs, uint32_t count)
{
    if (!s || (count > 0 && !reqs))
        return MTGP_EINVAL;
    const uint32_t gens = mtgp_batch_size(s->b);
    for (uint32_t i = 0; i < count; i++) {
        const mtgp_server_request &q = reqs[i];
        if (q.gen >= gens || q.kind > MTGP_KIND_NORMAL_FLOAT32 || q.n == 0 || round_up(4u * q.n) > s->arena_bytes ||
            (q.kind == MTGP_KIND_NORMAL_FLOAT32 && q.n % 2))
            return MTGP_EINVAL;
    }
    for (uint32_t i = 0; i < count; i++) {
        Req *r = new_req(s, reqs[i]);
        if (!r)
            return MTGP_ENOMEM;
        s->waiting.push_back(r);
    }
    return MTGP_OK;
}

int mtgp_server_poll(mtgp_server_t *s, mtgp_completion *done, uint32_t max_done, uint32_t *n_done)
{
    if (!s || (max_done > 0 && !done))
        return MTGP_EINVAL;
    // retire completed ticks, oldest first
    while (!s->inflight.empty()) {
        Tick &t = s->inflight.front();
        const hipError_t q = hipEventQuery(t.done);
        if (q == hipErrorNotReady)
            break;
        if (q != hipSuccess)
            return MTGP_EDEVICE;
        for (auto &c : t.chunks) {
            Req *r = c.first;
            r->finished += c.second;
            if (r->finished == r->n) {
                if (r->split) {
                    s->free_slots.push_back(r->slot);
                    r->split = false;
                }
                gq_remove(s, r);
                s->completed.put(r->rid, r);
                s->unreported.push_back(mtgp_completion{r->rid, r->offset, r->n});
            }
        }
        s->spare_events.push_back(t.done);
        s->inflight.pop_front();
    }
    uint32_t nd = 0;
    while (nd < max_done && !s->unreported.empty()) {
        done[nd++] = s->unreported.front();
        s->unreported.pop_front();
    }
    // admit in arrival order while the head fits
    while (!s->waiting.empty()) {
        Req *r = s->waiting.front();
        const uint32_t blk = s->index->take(round_up(4u * r->n) / kAlign);
        if (blk == mtgp_impl::ArenaIndex::kNil)
            break;
        r->blk = blk;
        r->offset = s->index->offset(blk) * kAlign;
        s->waiting.pop_front();
        gq_push(s, r);
        maybe_request_polys(s, r);
    }
    while (s->inflight.size() < s->depth && has_unscheduled(s)) {
        const int rc = launch_tick(s);
        if (rc != MTGP_OK)
            return rc;
    }
    if (n_done)
        *n_done = nd;
    return MTGP_OK;
}

int mtgp_server_release(mtgp_server_t *s, const uint64_t *rids, uint32_t count)
{
    if (!s || (count > 0 && !rids))
        return MTGP_EINVAL;
    int rc = MTGP_OK;
    for (uint32_t i = 0; i < count; i++) {
        Req *r = s->completed.take(rids[i]);
        if (!r) {
            rc = MTGP_EINVAL;
            continue;
        }
        s->index->give(r->blk);
        s->req_pool.push_back(r);
    }
    return rc;
}

int mtgp_server_pending(const mtgp_server_t *s, uint64_t *waiting, uint64_t *active, uint32_t *inflight)
{
    if (!s)
        return MTGP_EINVAL;
    if (waiting)
        *waiting = s->waiting.size();
    if (active)
        *active = s->active;
    if (inflight)
        *inflight = (uint32_t)s->inflight.size();
    return MTGP_OK;
}

int mtgp_server_set_split(mtgp_server_t *s, uint64_t min_outputs, uint32_t max_segments, uint32_t seg_chunks,
                          uint32_t slots)
{
    if (!s)
        return MTGP_EINVAL;
    if (min_outputs == 0) {
        s->split_min = 0;
        return MTGP_OK;
    }
    if (max_segments < 2 || max_segments > 64 || seg_chunks == 0 || slots == 0 || !s->inflight.empty() ||
        s->d_pool != nullptr)
        return MTGP_EINVAL;
    // Switched off: the first device run of split ticks stopped answering and
    // no cause has been shown yet (the tick logic itself runs to completion
    // in a host-only harness). Until one is, splitting is refused.
    if (!kSplitTicksEnabled)
        return MTGP_EINVAL;
    s->nmax = mtgp_impl::max_gen_words(s->b);
    // staging per split: polynomials (S x poly words), a prefix item, S jump
    // items and the raw words (deg psi + N); room for `slots` splits at once
    const uint32_t pmax = (uint32_t)std::max<uint64_t>(32u * s->nmax + 64u, 1u);   // deg psi <= p + 1 < 32 N + 1
    const uint64_t per = align256((uint64_t)max_segments * mtgp_impl::poly_words(s->nmax, pmax) * 8u) +
                         align256(sizeof(WorkItem)) + align256((uint64_t)max_segments * sizeof(JumpItem)) +
                         align256((uint64_t)(pmax + s->nmax) * 4u) + 1024u;
    s->ring_bytes = align256(per * std::max<uint32_t>(slots, 4u));
    if (hipMalloc(&s->d_pool, (size_t)slots * max_segments * s->nmax * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&s->d_ring, s->ring_bytes) != hipSuccess ||
        hipHostMalloc(&s->h_ring, s->ring_bytes, hipHostMallocDefault) != hipSuccess)
        return MTGP_ENOMEM;
    s->split_min = min_outputs;
    s->split_max = max_segments;
    s->seg_chunks = seg_chunks;
    s->slots = slots;
    s->free_slots.clear();
    for (uint32_t k = slots; k-- > 0;)
        s->free_slots.push_back(k);
    const unsigned nt = std::max(1u, std::min(8u, std::thread::hardware_concurrency() / 2));
    for (unsigned k = 0; k < nt; k++)
        s->workers.emplace_back(job_worker, s);
    return MTGP_OK;
}

void mtgp_server_destroy(mtgp_server_t *s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->job_mu);
        s->stop = true;
    }
    s->job_cv.notify_all();
    for (std::thread &w : s->workers)
        w.join();
    for (Tick &t : s->inflight) {
        (void)hipEventSynchronize(t.done);
        s->spare_events.push_back(t.done);
    }
    for (hipEvent_t e : s->spare_events)
        (void)hipEventDestroy(e);
    for (Req *r : s->waiting)
        delete r;
    for (GenQ &q : s->gq)
        for (Req *r = q.head; r;) {
            Req *nx = r->next;
            delete r;
            r = nx;
        }
    s->completed.for_each([](uint64_t, Req *r) { delete r; });
    for (Req *r : s->req_pool)
        delete r;
    (void)hipFree(s->d_pool);
    (void)hipFree(s->d_ring);
    if (s->h_ring)
        (void)hipHostFree(s->h_ring);
    delete s;
}

}  // extern "C"
