// CPU self-test of the request loop (csrc/mtgp_serve.cpp) over a stand-in
// device: the batch launch records its work items instead of running them,
// and events complete after a few polls (tests/host/mockhip). For random
// request streams it checks that every request completes exactly once with
// its size, that no generator gets two chunks in one tick, and that each
// generator's chunks, in launch order, cover its requests in arrival order,
// each one contiguously from its first output to its last. Built and run
// under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.
#include "mtgp.h"
#include "mtgp_arena.h"
#include "mtgp_host.h"
#include "mtgp_ridmap.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <unordered_map>
#include <vector>

struct mtgp_batch {
    uint32_t count;
};

static std::vector<std::vector<mtgp_impl::WorkItem>> g_launches;

extern "C" uint32_t mtgp_batch_size(const mtgp_batch_t *b) { return b->count; }

namespace mtgp_impl {
int launch_work_items(mtgp_batch_t *, std::vector<WorkItem> &items, hipStream_t)
{
    g_launches.push_back(items);
    return MTGP_OK;
}
// no generator is prepared for jump-ahead: these are never reached
bool split_ready(const mtgp_batch_t *, uint32_t) { return false; }
const f2::Poly &split_psi(const mtgp_batch_t *, uint32_t)
{
    static f2::Poly p;
    return p;
}
uint32_t gen_words(const mtgp_batch_t *, uint32_t) { return 351; }
uint32_t max_gen_words(const mtgp_batch_t *) { return 351; }
uint32_t poly_words(uint32_t, uint32_t) { return 1; }
void poly_layout(const f2::Poly &, uint32_t, uint64_t *) {}
std::vector<f2::Poly> segment_polys(const f2::Poly &, uint64_t, uint32_t) { return {}; }
LaunchShape prefix_shape(const mtgp_batch_t *, const std::vector<uint32_t> &) { return LaunchShape{}; }
uint16_t prefix_spl(const mtgp_batch_t *, uint32_t, const LaunchShape &) { return 1; }
hipError_t launch_prefix(mtgp_batch_t *, const WorkItem *, uint32_t, const LaunchShape &, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_jumps(const JumpItem *, const JumpItem *, uint32_t, hipStream_t) { return hipSuccess; }
}  // namespace mtgp_impl

static uint64_t g_rng = 88172645463325252ull;
static uint64_t rnd()
{
    g_rng ^= g_rng << 13;
    g_rng ^= g_rng >> 7;
    g_rng ^= g_rng << 17;
    return g_rng;
}

static int failures = 0;
#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            if (failures++ < 10) {                \
                std::printf("FAIL: " __VA_ARGS__); \
                std::printf("\n");                \
            }                                     \
        }                                         \
    } while (0)

// One request stream: G generators, nreq requests (a fifth of them up to
// `big` outputs), submitted a few at a time between polls.
static void run_stream(uint32_t G, uint32_t nreq, uint64_t big, uint64_t chunk, uint32_t depth, uint64_t arena_bytes)
{
    mtgp_batch b{G};
    void *arena = std::aligned_alloc(256, arena_bytes);
    mtgp_server_t *s = mtgp_server_create(&b, arena, arena_bytes, chunk, depth, nullptr);
    CHECK(s != nullptr, "create");
    if (!s)
        return;
    CHECK(mtgp_server_set_split(s, 1 << 16, 8, 2, 4) == MTGP_EINVAL, "split ticks are refused");
    std::vector<mtgp_server_request> reqs(nreq);
    for (uint32_t i = 0; i < nreq; i++) {
        reqs[i].rid = 1000 + i;
        reqs[i].gen = (uint32_t)(rnd() % G);
        reqs[i].kind = (uint32_t)(rnd() % 4);
        reqs[i].n = 1 + rnd() % (i % 5 == 0 ? big : 20000);
        if (reqs[i].kind == 3)
            reqs[i].n += reqs[i].n & 1;
    }
    g_launches.clear();
    std::vector<mtgp_completion> done(4096);
    std::vector<int> seen(nreq, 0);
    size_t next = 0, finished = 0;
    long polls = 0;
    while (finished < nreq && polls < 5000000) {
        if (next < nreq) {
            const size_t k = std::min<size_t>(1 + rnd() % 16, nreq - next);
            CHECK(mtgp_server_submit(s, &reqs[next], (uint32_t)k) == MTGP_OK, "submit");
            next += k;
        }
        uint32_t nd = 0;
        CHECK(mtgp_server_poll(s, done.data(), (uint32_t)done.size(), &nd) == MTGP_OK, "poll");
        std::vector<uint64_t> rel;
        for (uint32_t i = 0; i < nd; i++) {
            const uint64_t k = done[i].rid - 1000;
            CHECK(k < nreq && done[i].n == reqs[k].n, "completion %llu", (unsigned long long)done[i].rid);
            if (k < nreq)
                seen[k]++;
            rel.push_back(done[i].rid);
        }
        if (!rel.empty())
            CHECK(mtgp_server_release(s, rel.data(), (uint32_t)rel.size()) == MTGP_OK, "release");
        finished += nd;
        polls++;
    }
    for (uint32_t i = 0; i < nreq; i++)
        CHECK(seen[i] == 1, "request %u completed %d times", i, seen[i]);
    // per generator, the chunks in launch order against its requests in arrival order
    std::vector<std::vector<uint32_t>> order(G);
    for (uint32_t i = 0; i < nreq; i++)
        order[reqs[i].gen].push_back(i);
    std::vector<size_t> cur(G, 0);
    std::vector<uint64_t> left(G, 0), next_out(G, 0);
    for (uint32_t g = 0; g < G; g++)
        if (!order[g].empty())
            left[g] = reqs[order[g][0]].n;
    for (const auto &L : g_launches) {
        std::vector<int> per(G, 0);
        for (const auto &it : L) {
            const uint32_t g = it.gen;
            CHECK(g < G && per[g]++ == 0, "generator %u twice in a tick", g);
            if (g >= G || cur[g] >= order[g].size()) {
                CHECK(false, "chunk beyond the requests of generator %u", g);
                continue;
            }
            const mtgp_server_request &q = reqs[order[g][cur[g]]];
            CHECK((it.kind & 0xff) == q.kind && it.n > 0 && it.n <= chunk && it.n <= left[g] && it.src == 0,
                  "chunk of generator %u", g);
            CHECK(left[g] == q.n || it.out == next_out[g], "chunks of a request not contiguous (generator %u)", g);
            const uint64_t off = it.out - reinterpret_cast<uint64_t>(arena);
            CHECK(off % 4 == 0 && off + 4 * it.n <= arena_bytes, "chunk outside the arena");
            next_out[g] = it.out + 4 * it.n;
            left[g] -= std::min(left[g], it.n);
            if (left[g] == 0 && ++cur[g] < order[g].size())
                left[g] = reqs[order[g][cur[g]]].n;
        }
    }
    for (uint32_t g = 0; g < G; g++)
        CHECK(cur[g] == order[g].size(), "generator %u: %zu of %zu requests covered", g, cur[g], order[g].size());
    uint64_t waiting = 1, active = 1;
    uint32_t inflight = 1;
    mtgp_server_pending(s, &waiting, &active, &inflight);
    CHECK(waiting == 0 && active == 0 && inflight == 0, "pending after the stream");
    std::printf("stream G=%u requests=%u chunk=%llu depth=%u: %ld polls, %zu ticks\n", G, nreq,
                (unsigned long long)chunk, depth, polls, g_launches.size());
    mtgp_server_destroy(s);
    std::free(arena);
}

// The arena index against a plain model: after every take and give, the free
// blocks are exactly the units not taken (disjoint, merged with free
// neighbours), a take fails only when no free block holds the request, and
// taken blocks never overlap.
static void test_arena_index()
{
    for (uint64_t units : {1ull, 15ull, 16ull, 17ull, 1000ull, 1ull << 20, (1ull << 25) + 3}) {
        mtgp_impl::ArenaIndex ix(units);
        std::vector<std::pair<uint32_t, uint64_t>> live;   // (id, length)
        std::vector<uint8_t> used((size_t)std::min<uint64_t>(units, 1 << 20) , 0);
        const bool model = units <= (1u << 20);
        for (int step = 0; step < 4000; step++) {
            if (live.empty() || rnd() % 3) {
                const uint64_t want = 1 + (rnd() % 4 == 0 ? rnd() % units : rnd() % std::min<uint64_t>(units, 64));
                uint64_t largest = 0;
                for (auto &fb : ix.free_blocks())
                    largest = std::max(largest, fb.second);
                const uint32_t id = ix.take(want);
                CHECK((id == mtgp_impl::ArenaIndex::kNil) == (largest < want), "take %llu of %llu: largest free %llu",
                      (unsigned long long)want, (unsigned long long)units, (unsigned long long)largest);
                if (id == mtgp_impl::ArenaIndex::kNil)
                    continue;
                CHECK(ix.length(id) == want && ix.offset(id) + want <= units, "taken block");
                if (model)
                    for (uint64_t u = ix.offset(id); u < ix.offset(id) + want; u++) {
                        CHECK(!used[u], "overlap at unit %llu", (unsigned long long)u);
                        used[u] = 1;
                    }
                live.emplace_back(id, want);
            } else {
                const size_t k = rnd() % live.size();
                const uint32_t id = live[k].first;
                if (model)
                    for (uint64_t u = ix.offset(id); u < ix.offset(id) + live[k].second; u++)
                        used[u] = 0;
                ix.give(id);
                live[k] = live.back();
                live.pop_back();
            }
            if (model && step % 97 == 0) {
                // free blocks = maximal runs of unused units
                std::vector<std::pair<uint64_t, uint64_t>> runs;
                for (uint64_t u = 0; u < units;) {
                    if (used[u]) {
                        u++;
                        continue;
                    }
                    uint64_t e = u;
                    while (e < units && !used[e])
                        e++;
                    runs.emplace_back(u, e - u);
                    u = e;
                }
                auto fb = ix.free_blocks();
                std::sort(fb.begin(), fb.end());
                CHECK(fb == runs, "free blocks differ from the model (%zu against %zu runs)", fb.size(), runs.size());
            }
        }
        for (auto &l : live)
            ix.give(l.first);
        const auto fb = ix.free_blocks();
        CHECK(fb.size() == 1 && fb[0].first == 0 && fb[0].second == units, "everything given back: one block");
    }
    std::printf("arena index checked\n");
}

// The id map against std::unordered_map: random puts (new ids and
// replacements) and takes (present and absent ids), over sequential ids,
// ids in one residue class (equal low bits) and random ids, through several
// table growths; after each phase every entry is checked and the map drained.
static void test_rid_map()
{
    static int objs[1 << 16];
    for (int pattern = 0; pattern < 3; pattern++) {
        mtgp_impl::RidMap<int> m;
        std::unordered_map<uint64_t, int *> model;
        auto id_of = [&](uint64_t k) -> uint64_t {
            return pattern == 0 ? k : pattern == 1 ? (k << 20) : (k * 0x9e3779b97f4a7c15ull) ^ 0x5555;
        };
        for (int step = 0; step < 200000; step++) {
            const uint64_t k = rnd() % 40000;
            const uint64_t rid = id_of(k);
            if (rnd() % 2) {
                int *p = &objs[rnd() % (1 << 16)];
                m.put(rid, p);
                model[rid] = p;
            } else {
                auto it = model.find(rid);
                int *want = it == model.end() ? nullptr : it->second;
                CHECK(m.take(rid) == want, "take of id %llu (pattern %d)", (unsigned long long)rid, pattern);
                if (it != model.end())
                    model.erase(it);
            }
            CHECK(m.size() == model.size(), "size %zu against %zu", m.size(), model.size());
        }
        size_t seen = 0;
        m.for_each([&](uint64_t rid, int *p) {
            seen++;
            auto it = model.find(rid);
            CHECK(it != model.end() && it->second == p, "entry %llu", (unsigned long long)rid);
        });
        CHECK(seen == model.size(), "for_each visits %zu of %zu", seen, model.size());
        for (auto &kv : model)
            CHECK(m.take(kv.first) == kv.second, "drain %llu", (unsigned long long)kv.first);
        CHECK(m.size() == 0, "drained map not empty");
    }
    std::printf("rid map checked\n");
}

int main()
{
    test_rid_map();
    test_arena_index();
    run_stream(64, 3000, 300000, 1 << 14, 2, 64ull << 20);
    run_stream(8, 2000, 300000, 1 << 12, 3, 64ull << 20);
    run_stream(1000, 20000, 300000, 1 << 16, 1, 64ull << 20);
    // an arena smaller than the load: admission waits for releases
    run_stream(32, 4000, 100000, 1 << 13, 2, 2ull << 20);
    if (failures)
        std::printf("%d failures\n", failures);
    else
        std::printf("serve selftest ok\n");
    return failures ? 1 : 0;
}
