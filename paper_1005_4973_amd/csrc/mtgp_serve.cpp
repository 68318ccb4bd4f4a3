// Continuous-batching request loop over a batch's resident generators.
//
// Requests (generator, kind, n) are queued by the caller and admitted in
// arrival order while their outputs fit the output arena (first fit; a
// request that does not fit waits, and so do the ones behind it). Every
// scheduling step retires ticks whose completion event has fired, admits
// what fits, and launches ticks while fewer than `depth` are in flight. A
// tick advances every generator that has admitted work by up to `chunk`
// outputs of its oldest unfinished request, in one persistent batched launch
// (mtgp_batch_generate); consecutive chunks of one generator stay in stream
// order, so each request gets exactly the stream segment it would get alone,
// and requests that arrive while others run join at the next tick.
#include "../../include/mtgp.h"
#include "mtgp_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

namespace {

struct Req {
    uint64_t rid;
    uint32_t gen;
    uint32_t kind;
    uint64_t n;
    uint64_t offset = 0;     // byte offset of its outputs in the arena
    uint64_t scheduled = 0;  // outputs put in ticks
    uint64_t finished = 0;   // outputs whose tick completed
};

struct Tick {
    hipEvent_t done;
    std::vector<std::pair<Req *, uint64_t>> chunks;
};

}  // namespace

struct mtgp_server {
    mtgp_batch_t *b = nullptr;
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    uint64_t chunk = 0;
    uint32_t depth = 0;
    hipStream_t stream = nullptr;
    std::map<uint64_t, uint64_t> free_ranges;              // offset -> length, disjoint and coalesced
    std::deque<Req *> waiting;                             // submitted, not admitted
    std::unordered_map<uint32_t, std::deque<Req *>> active;    // generator -> admitted, unfinished
    std::deque<Tick> inflight;
    std::vector<hipEvent_t> spare_events;
    std::unordered_map<uint64_t, Req *> completed;         // rid -> finished, not released
    std::deque<mtgp_completion> unreported;                // finished, not yet returned by poll
    std::vector<mtgp_request> scratch;
};

namespace {

constexpr uint64_t kAlign = 256;   // output regions start on 256-byte boundaries

uint64_t round_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool take_range(mtgp_server *s, uint64_t bytes, uint64_t *offset)
{
    for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it)
        if (it->second >= bytes) {
            *offset = it->first;
            const uint64_t rest = it->second - bytes;
            const uint64_t at = it->first + bytes;
            s->free_ranges.erase(it);
            if (rest)
                s->free_ranges.emplace(at, rest);
            return true;
        }
    return false;
}

void give_range(mtgp_server *s, uint64_t offset, uint64_t bytes)
{
    auto it = s->free_ranges.emplace(offset, bytes).first;
    // merge with the following and the preceding range
    auto next = std::next(it);
    if (next != s->free_ranges.end() && it->first + it->second == next->first) {
        it->second += next->second;
        s->free_ranges.erase(next);
    }
    if (it != s->free_ranges.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            s->free_ranges.erase(it);
        }
    }
}

int launch_tick(mtgp_server *s)
{
    Tick t;
    s->scratch.clear();
    for (auto &kv : s->active) {
        for (Req *r : kv.second)
            if (r->scheduled < r->n) {
                const uint64_t k = std::min(s->chunk, r->n - r->scheduled);
                mtgp_request q;
                q.gen = r->gen;
                q.kind = r->kind;
                q.n = k;
                q.out = s->arena + r->offset + 4u * r->scheduled;
                s->scratch.push_back(q);
                t.chunks.emplace_back(r, k);
                break;   // one chunk per generator per tick, from its oldest request
            }
    }
    if (t.chunks.empty())
        return MTGP_OK;
    if (s->spare_events.empty()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return MTGP_EDEVICE;
        s->spare_events.push_back(e);
    }
    t.done = s->spare_events.back();
    const int rc = mtgp_impl::batch_generate(s->b, s->scratch.data(), (uint32_t)s->scratch.size(), s->stream, false);
    if (rc != MTGP_OK)
        return rc;
    if (hipEventRecord(t.done, s->stream) != hipSuccess)
        return MTGP_EDEVICE;
    s->spare_events.pop_back();
    for (auto &c : t.chunks)
        c.first->scheduled += c.second;
    s->inflight.push_back(std::move(t));
    return MTGP_OK;
}

bool has_unscheduled(const mtgp_server *s)
{
    for (const auto &kv : s->active)
        for (const Req *r : kv.second)
            if (r->scheduled < r->n)
                return true;
    return false;
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
    s->free_ranges.emplace(0, s->arena_bytes);
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
        Req *r = new (std::nothrow) Req{reqs[i].rid, reqs[i].gen, reqs[i].kind, reqs[i].n};
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
                auto &q2 = s->active[r->gen];
                for (auto it = q2.begin(); it != q2.end(); ++it)
                    if (*it == r) {
                        q2.erase(it);
                        break;
                    }
                if (q2.empty())
                    s->active.erase(r->gen);
                s->completed[r->rid] = r;
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
        uint64_t off;
        if (!take_range(s, round_up(4u * r->n), &off))
            break;
        r->offset = off;
        s->waiting.pop_front();
        s->active[r->gen].push_back(r);
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
        auto it = s->completed.find(rids[i]);
        if (it == s->completed.end()) {
            rc = MTGP_EINVAL;
            continue;
        }
        Req *r = it->second;
        give_range(s, r->offset, round_up(4u * r->n));
        s->completed.erase(it);
        delete r;
    }
    return rc;
}

int mtgp_server_pending(const mtgp_server_t *s, uint64_t *waiting, uint64_t *active, uint32_t *inflight)
{
    if (!s)
        return MTGP_EINVAL;
    uint64_t a = 0;
    for (const auto &kv : s->active)
        a += kv.second.size();
    if (waiting)
        *waiting = s->waiting.size();
    if (active)
        *active = a;
    if (inflight)
        *inflight = (uint32_t)s->inflight.size();
    return MTGP_OK;
}

void mtgp_server_destroy(mtgp_server_t *s)
{
    if (!s)
        return;
    for (Tick &t : s->inflight) {
        (void)hipEventSynchronize(t.done);
        s->spare_events.push_back(t.done);
    }
    for (hipEvent_t e : s->spare_events)
        (void)hipEventDestroy(e);
    for (Req *r : s->waiting)
        delete r;
    for (auto &kv : s->active)
        for (Req *r : kv.second)
            delete r;
    for (auto &kv : s->completed)
        delete kv.second;
    delete s;
}

}  // extern "C"
