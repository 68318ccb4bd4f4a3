// CPU self-test of the request loop's split ticks (jump-ahead inside ticks,
// csrc/mtgp_serve.cpp built with MTGP_SERVE_SPLIT_TICKS=1) over a stand-in
// device (tests/host/mockhip): the launches record their work items, jump
// items and prefix items instead of running them. For random request streams
// on generators of which some are prepared for jump-ahead, it checks that
// every request completes and is covered exactly once by its chunks; that
// plain chunks come in order and before a request's split; that a split tick
// holds one raw-prefix item per split generator (state kept, deg psi - 1
// outputs) and one jump per segment from that prefix's words (the first an
// identity jump), each into its own state buffer; that segments start in the
// split tick, follow each other in output position, advance one chunk per
// tick, and carry the state flags (state to the segment buffer until its last
// chunk; the last segment alone writes the generator's state back); that a
// generator's requests run in arrival order; and that the staging blocks of
// ticks in flight at the same time never overlap. Built and run under
// AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.
#include "mtgp.h"
#include "mtgp_host.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

using mtgp_impl::JumpItem;
using mtgp_impl::WorkItem;

struct mtgp_batch {
    uint32_t count;
    uint32_t ready;
};

struct Tick {
    std::vector<WorkItem> prefix;
    std::vector<JumpItem> jumps;
    std::vector<WorkItem> gen;
    long launch_seq = 0, retire_seq = -1;
};
static std::vector<Tick> g_ticks;
static Tick g_cur;
static long g_seq = 0;   // order of launches and retirements (tick completions)
static size_t g_retired = 0;
static const uint32_t kN = 351, kD = 11214;

extern "C" uint32_t mtgp_batch_size(const mtgp_batch_t *b) { return b->count; }

namespace mtgp_impl {
int launch_work_items(mtgp_batch_t *, std::vector<WorkItem> &items, hipStream_t)
{
    g_cur.gen = items;
    g_cur.launch_seq = g_seq++;
    g_ticks.push_back(g_cur);
    g_cur = Tick{};
    return MTGP_OK;
}
bool split_ready(const mtgp_batch_t *b, uint32_t g) { return g < b->ready; }
const f2::Poly &split_psi(const mtgp_batch_t *, uint32_t)
{
    static f2::Poly p = [] {
        f2::Poly q;
        q.w.assign(kD / 64 + 1, 0);
        q.w[0] = 1;
        q.w[kD / 64] |= 1ull << (kD % 64);
        q.trim();
        return q;
    }();
    return p;
}
uint32_t gen_words(const mtgp_batch_t *, uint32_t) { return kN; }
uint32_t max_gen_words(const mtgp_batch_t *) { return kN; }
uint32_t poly_words(uint32_t N, uint32_t D) { return jump_poly_words(N, D); }
void poly_layout(const f2::Poly &, uint32_t, uint64_t *) {}
std::vector<f2::Poly> segment_polys(const f2::Poly &, uint64_t, uint32_t S)
{
    return std::vector<f2::Poly>(S > 1 ? S - 1 : 0, f2::Poly::one());
}
LaunchShape prefix_shape(const mtgp_batch_t *, const std::vector<uint32_t> &) { return LaunchShape{}; }
uint16_t prefix_spl(const mtgp_batch_t *, uint32_t, const LaunchShape &) { return 1; }
hipError_t launch_prefix(mtgp_batch_t *, const WorkItem *d, uint32_t n, const LaunchShape &, hipStream_t)
{
    g_cur.prefix.assign(d, d + n);
    return hipSuccess;
}
hipError_t launch_jumps(const JumpItem *d, const JumpItem *h, uint32_t n, hipStream_t)
{
    for (uint32_t i = 0; i < n; i++)
        if (std::memcmp(&d[i], &h[i], sizeof(JumpItem)) != 0)
            std::printf("FAIL: jump item %u uploaded differs from the host copy\n", i);
    g_cur.jumps.assign(d, d + n);
    return hipSuccess;
}
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
#define CHECK(cond, ...)                           \
    do {                                           \
        if (!(cond)) {                             \
            if (failures++ < 20) {                 \
                std::printf("FAIL: " __VA_ARGS__); \
                std::printf("\n");                 \
            }                                      \
        }                                          \
    } while (0)

struct Chunk {
    size_t tick;
    uint64_t pos, n, src;
    uint16_t kind;
};

static void run(uint32_t G, uint32_t ready, uint32_t nreq, uint64_t chunk, uint32_t depth, uint32_t maxseg,
                uint32_t segchunks, uint32_t slots, uint64_t min_out)
{
    mtgp_batch b{G, ready};
    const uint64_t arena_bytes = 1ull << 30;
    char *arena = (char *)std::aligned_alloc(256, arena_bytes);
    mtgp_server_t *s = mtgp_server_create(&b, arena, arena_bytes, chunk, depth, nullptr);
    CHECK(mtgp_server_set_split(s, min_out, maxseg, segchunks, slots) == MTGP_OK, "set_split");
    std::vector<mtgp_server_request> reqs(nreq);
    for (uint32_t i = 0; i < nreq; i++) {
        reqs[i].rid = i;
        reqs[i].gen = (uint32_t)(rnd() % G);
        reqs[i].kind = (uint32_t)(rnd() % 4);
        reqs[i].n = (i % 4 == 0) ? 100000 + rnd() % 500000 : 1 + rnd() % 30000;
        if (reqs[i].kind == 3)
            reqs[i].n += reqs[i].n & 1;
    }
    g_ticks.clear();
    g_retired = 0;
    mock_on_event_done = [] { g_ticks[g_retired++].retire_seq = g_seq++; };
    std::vector<mtgp_completion> done(4096);
    std::vector<uint64_t> offset(nreq, UINT64_MAX);
    size_t next = 0, fin = 0;
    long polls = 0;
    while (fin < nreq && polls < 20000000) {
        if (next < nreq) {
            const size_t k = std::min<size_t>(1 + rnd() % 8, nreq - next);
            CHECK(mtgp_server_submit(s, &reqs[next], (uint32_t)k) == MTGP_OK, "submit");
            next += k;
        }
        uint32_t nd = 0;
        CHECK(mtgp_server_poll(s, done.data(), (uint32_t)done.size(), &nd) == MTGP_OK, "poll");
        for (uint32_t i = 0; i < nd; i++)
            offset[done[i].rid] = done[i].offset;   // outputs kept (no release) so ranges stay unique
        fin += nd;
        polls++;
        if (nd == 0)
            std::this_thread::yield();
    }
    CHECK(fin == nreq, "completed %zu of %u", fin, nreq);
    // map generation items to requests
    std::map<uint64_t, uint32_t> by_off;
    for (uint32_t i = 0; i < nreq; i++)
        if (offset[i] != UINT64_MAX)
            by_off[offset[i]] = i;
    std::vector<std::vector<Chunk>> ch(nreq);
    for (size_t t = 0; t < g_ticks.size(); t++)
        for (const WorkItem &it : g_ticks[t].gen) {
            const uint64_t off = it.out - (uint64_t)arena;
            auto u = by_off.upper_bound(off);
            if (u == by_off.begin()) {
                CHECK(false, "item outside every request");
                continue;
            }
            --u;
            const uint32_t r = u->second;
            const uint64_t pos = (off - u->first) / 4;
            CHECK(it.gen == reqs[r].gen && pos + it.n <= reqs[r].n, "item of request %u", r);
            ch[r].push_back(Chunk{t, pos, it.n, it.src, it.kind});
        }
    int nsplit = 0;
    struct Slot {
        uint64_t base;   // the request's first segment state buffer
        uint32_t r;
        size_t from, to; // split tick and last tick
    };
    std::vector<Slot> live_slots;
    std::vector<std::vector<uint32_t>> order(G);
    for (uint32_t i = 0; i < nreq; i++)
        order[reqs[i].gen].push_back(i);
    std::vector<size_t> first_tick(nreq, SIZE_MAX), last_tick(nreq, 0);
    for (uint32_t r = 0; r < nreq; r++) {
        const auto &c = ch[r];
        // coverage
        std::vector<std::pair<uint64_t, uint64_t>> iv;
        for (const Chunk &x : c)
            iv.emplace_back(x.pos, x.pos + x.n);
        std::sort(iv.begin(), iv.end());
        uint64_t at = 0;
        for (auto &p : iv) {
            CHECK(p.first == at, "request %u: gap or overlap at %llu", r, (unsigned long long)at);
            at = p.second;
        }
        CHECK(at == reqs[r].n, "request %u covered to %llu of %llu", r, (unsigned long long)at,
              (unsigned long long)reqs[r].n);
        for (const Chunk &x : c) {
            first_tick[r] = std::min(first_tick[r], x.tick);
            last_tick[r] = std::max(last_tick[r], x.tick);
            CHECK((x.kind & 0xff) == reqs[r].kind, "kind");
        }
        // plain chunks: contiguous from 0, before any segment chunk
        size_t split_tick = SIZE_MAX;
        uint64_t plain_end = 0;
        for (const Chunk &x : c) {
            if (x.src == 0) {
                CHECK(x.pos == plain_end, "request %u plain chunk out of order", r);
                plain_end += x.n;
                CHECK(x.kind <= 0xff, "plain chunk flags");
            } else {
                split_tick = std::min(split_tick, x.tick);
            }
        }
        for (const Chunk &x : c)
            if (x.src == 0 && split_tick != SIZE_MAX)
                CHECK(x.tick < split_tick, "request %u plain chunk at or after its split", r);
        if (split_tick == SIZE_MAX)
            continue;
        nsplit++;
        // the split tick: one prefix item for the generator, S jumps from its raw words
        const Tick &T = g_ticks[split_tick];
        const WorkItem *pre = nullptr;
        for (const WorkItem &p : T.prefix)
            if (p.gen == reqs[r].gen) {
                CHECK(pre == nullptr, "two prefixes for one generator in a tick");
                pre = &p;
            }
        CHECK(pre != nullptr, "request %u: no prefix in its split tick", r);
        if (!pre)
            continue;
        CHECK((pre->kind & 0xff) == mtgp_impl::kKindRaw && (pre->kind & mtgp_impl::kKeepState) && pre->n == kD - 1 &&
                  pre->src == 0,
              "prefix item");
        std::vector<JumpItem> js;
        for (const JumpItem &j : T.jumps)
            if (j.raw == pre->out)
                js.push_back(j);
        // segments by source buffer, in the order of the jumps
        std::map<uint64_t, std::vector<Chunk>> seg;
        for (const Chunk &x : c)
            if (x.src)
                seg[x.src].push_back(x);
        CHECK(js.size() == seg.size(), "request %u: %zu jumps for %zu segments", r, js.size(), seg.size());
        const uint32_t S = (uint32_t)js.size();
        if (S > 0)
            live_slots.push_back(Slot{js[0].out, r, split_tick, last_tick[r]});
        for (uint32_t k = 0; k < S; k++) {
            CHECK(js[k].N == kN && js[k].D == (k == 0 ? 1u : kD), "jump %u of request %u", k, r);
            CHECK(k == 0 || js[k].out == js[0].out + 4ull * k * kN, "jump outputs not consecutive buffers");
            auto sit = seg.find(js[k].out);
            CHECK(sit != seg.end(), "segment %u has no chunks", k);
            if (sit == seg.end())
                continue;
            const auto &sc = sit->second;
            CHECK(sc.front().tick == split_tick, "segment %u does not start in the split tick", k);
            for (size_t i = 0; i < sc.size(); i++) {
                if (i)
                    CHECK(sc[i].pos == sc[i - 1].pos + sc[i - 1].n && sc[i].tick > sc[i - 1].tick, "segment chunks");
                const bool last = i + 1 == sc.size();
                const uint16_t fl = sc[i].kind & ~0xff;
                const uint16_t want = !last ? mtgp_impl::kStateToSrc : (k + 1 == S ? 0 : mtgp_impl::kKeepState);
                CHECK(fl == want, "request %u segment %u chunk %zu flags %x want %x", r, k, i, fl, want);
            }
            if (k > 0) {
                const auto &prev = seg[js[k - 1].out];
                CHECK(sc.front().pos == prev.front().pos + (prev.back().pos + prev.back().n - prev.front().pos),
                      "segment %u does not follow segment %u", k, k - 1);
            } else {
                CHECK(sc.front().pos == plain_end, "segment 0 does not start where the plain chunks end");
            }
        }
    }
    // generator order: the next request starts after the previous one's last chunk
    for (uint32_t g = 0; g < G; g++)
        for (size_t i = 1; i < order[g].size(); i++) {
            const uint32_t a = order[g][i - 1], bq = order[g][i];
            CHECK(first_tick[bq] > last_tick[a],
                  "generator %u: request %u starts in tick %zu, before %u ends in %zu", g, bq, first_tick[bq], a,
                  last_tick[a]);
        }
    // two split requests live at once (from the launch of one's split tick to
    // the completion of its last tick) use different state buffers
    auto live = [&](size_t from, size_t to) {
        return std::make_pair(g_ticks[from].launch_seq, g_ticks[to].retire_seq < 0 ? g_seq : g_ticks[to].retire_seq);
    };
    for (size_t i = 0; i < live_slots.size(); i++)
        for (size_t j = i + 1; j < live_slots.size(); j++) {
            const Slot &x = live_slots[i], &y = live_slots[j];
            const auto a = live(x.from, x.to), c = live(y.from, y.to);
            CHECK(!(x.base == y.base && a.first < c.second && c.first < a.second),
                  "requests %u and %u share state buffers while both live", x.r, y.r);
        }
    // staging blocks of ticks in flight do not overlap; pool buffers of two live split requests differ
    struct Rng {
        uint64_t lo, hi;
        long from, to;
    };
    std::vector<Rng> blocks;
    for (const Tick &t : g_ticks) {
        if (t.prefix.empty())
            continue;
        uint64_t lo = UINT64_MAX, hi = 0;
        for (const WorkItem &p : t.prefix) {
            lo = std::min(lo, p.out);
            hi = std::max<uint64_t>(hi, p.out + 4ull * (kD + kN));
        }
        for (const JumpItem &j : t.jumps) {
            lo = std::min(lo, j.poly);
            hi = std::max<uint64_t>(hi, j.poly + 8ull * mtgp_impl::jump_poly_words(kN, kD));
        }
        blocks.push_back(Rng{lo, hi, t.launch_seq, t.retire_seq < 0 ? g_seq : t.retire_seq});
    }
    for (size_t i = 0; i < blocks.size(); i++)
        for (size_t j = i + 1; j < blocks.size(); j++) {
            const bool live_together = blocks[i].from < blocks[j].to && blocks[j].from < blocks[i].to;
            const bool overlap = blocks[i].lo < blocks[j].hi && blocks[j].lo < blocks[i].hi;
            CHECK(!(live_together && overlap), "staging blocks of ticks %zu and %zu overlap while both in flight", i, j);
        }
    std::printf("G=%u ready=%u reqs=%u chunk=%llu depth=%u maxseg=%u segchunks=%u slots=%u: %zu ticks, %d split "
                "requests, %ld polls\n",
                G, ready, nreq, (unsigned long long)chunk, depth, maxseg, segchunks, slots, g_ticks.size(), nsplit,
                polls);
    mtgp_server_destroy(s);
    std::free(arena);
}

int main()
{
    run(64, 48, 400, 1 << 14, 2, 8, 2, 16, 1 << 16);
    run(16, 16, 600, 1 << 12, 3, 8, 4, 2, 1 << 14);
    run(8, 6, 300, 1 << 13, 1, 64, 1, 1, 1 << 15);
    run(32, 32, 800, 1 << 14, 2, 3, 2, 4, 1 << 16);
    if (failures)
        std::printf("%d failures\n", failures);
    else
        std::printf("split selftest ok\n");
    return failures ? 1 : 0;
}
