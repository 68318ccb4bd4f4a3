// Recursion-parameter search in the manner of MTGPDC (the paper's section 5),
// on the host.
//
// A candidate is (M, R) with sh1 = 13 and sh2 = 4 fixed as in section 5: the
// 32-bit ID is embedded in the 4x32 matrix R (its 16 high bits in the 16
// MSBs of the first row, its 16 low bits in the second row above the four
// LSBs), the four LSBs of the rows are drawn until I + R44 is invertible
// (a necessary condition for the last line of the recursion to be
// invertible), and the other bits of R and M are random. The candidate's
// characteristic polynomial is the minimal polynomial (Berlekamp-Massey) of
// one bit of its raw words when that has degree p; it is irreducible -- and
// since 2^p - 1 is prime, primitive, so the period is 2^p - 1 -- when it has
// no small factor (a sieve) and x^(2^p) = x modulo it. Tempering does not
// change the period; its search by equidistribution (SIS) is not done here
// and the tempering table is drawn at random.
#include "../../include/mtgp.h"
#include "mtgp_f2.h"

#include <sched.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <vector>

namespace mtgp_impl {
namespace {

// SplitMix64 (Steele, Lea and Flood, 2014): one counter-based stream per
// candidate, so the result does not depend on the thread count.
struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    uint32_t below(uint32_t n) { return (uint32_t)(next() % n); }
};

constexpr uint32_t kSh1 = 13, kSh2 = 4;
constexpr uint32_t kSieve = 256;   // reject factors of degree <= 256 before the full test

struct Candidate {
    uint32_t M;
    uint32_t rows[4];   // rows of R, first row = table entry of nibble 1000 (MSB first)
    uint32_t tbl[16];
};

uint32_t pow2_floor(uint32_t v)
{
    uint32_t r = 1;
    while (r * 2 <= v)
        r *= 2;
    return r;
}

// F2-linear table of R: entry j is the XOR of the rows selected by j's bits,
// the first row by the nibble's MSB.
void fill_table(Candidate &c)
{
    for (uint32_t j = 0; j < 16; j++) {
        uint32_t v = 0;
        for (uint32_t a = 0; a < 4; a++)
            if ((j >> (3 - a)) & 1)
                v ^= c.rows[a];
        c.tbl[j] = v;
    }
}

// u -> u ^ (tbl[u & 0xf] & 0xf) on the low nibble is a bijection
bool nibble_map_invertible(const uint32_t *tbl)
{
    uint32_t seen = 0;
    for (uint32_t j = 0; j < 16; j++)
        seen |= 1u << ((j ^ tbl[j]) & 0xf);
    return seen == 0xffff;
}

Candidate draw(uint32_t p, uint32_t id, SplitMix64 &rng)
{
    const uint32_t N = (p + 31) / 32;
    Candidate c;
    // 2 < M < N - floor2(N) (section 5); small states fall back to 2 <= M <= N-1
    const uint32_t hi = N - pow2_floor(N);
    if (hi > 4)
        c.M = 3 + rng.below(hi - 3);
    else
        c.M = 2 + rng.below(N - 2);
    for (uint32_t a = 0; a < 4; a++)
        c.rows[a] = (uint32_t)rng.next() & ~0xfu;
    c.rows[0] = (c.rows[0] & 0x0000fff0u) | (id & 0xffff0000u);            // 16 MSBs of the ID
    c.rows[1] = (c.rows[1] & 0xfff00000u) | ((id & 0xffffu) << 4);        // 16 LSBs, above the 4 LSBs
    do {
        for (uint32_t a = 0; a < 4; a++)
            c.rows[a] = (c.rows[a] & ~0xfu) | (uint32_t)(rng.next() & 0xf);
        fill_table(c);
    } while (!nibble_map_invertible(c.tbl));
    return c;
}

// Bit 31 of the raw words x_N, x_{N+1}, ... (nbits of them) of the recursion
// from a state seeded like the library's generators, packed.
std::vector<uint64_t> raw_plane(uint32_t p, const Candidate &c, int64_t nbits)
{
    const uint32_t N = (p + 31) / 32;
    const uint32_t mask = 0xffffffffu << (32 * N - p);
    std::vector<uint32_t> x((size_t)N + (size_t)nbits);
    uint32_t v = 5489u;
    x[0] = v;
    for (uint32_t i = 1; i < N; i++) {
        v = 1812433253u * (v ^ (v >> 30)) + i;
        x[i] = v;
    }
    std::vector<uint64_t> bits((size_t)(nbits / 64 + 1), 0);
    for (int64_t i = 0; i < nbits; i++) {
        uint32_t t = x[(size_t)i + 1] ^ (x[(size_t)i] & mask);
        t ^= t << kSh1;
        const uint32_t u = t ^ (x[(size_t)i + c.M] >> kSh2);
        const uint32_t y = u ^ c.tbl[u & 0xf];
        x[(size_t)i + N] = y;
        if (y >> 31)
            bits[(size_t)(i >> 6)] |= 1ull << (i & 63);
    }
    return bits;
}

struct Outcome {
    bool full_degree = false, sieved = false, found = false;
};

Outcome test(uint32_t p, const Candidate &c)
{
    Outcome o;
    const int64_t nbits = 2 * (int64_t)p + 64;
    const std::vector<uint64_t> bits = raw_plane(p, c, nbits);
    const f2::Poly phi = f2::minpoly(bits.data(), nbits);
    if (phi.deg != (int64_t)p)
        return o;
    o.full_degree = true;
    o.found = f2::irreducible_prime_degree(phi, kSieve, &o.sieved);
    return o;
}

bool is_prime(uint32_t v)
{
    if (v < 2)
        return false;
    for (uint32_t d = 2; d * d <= v; d++)
        if (v % d == 0)
            return false;
    return true;
}

uint64_t candidate_seed(uint64_t seed, uint32_t id, uint64_t index)
{
    SplitMix64 s{seed ^ ((uint64_t)id << 32)};
    s.s += index * 0x632be59bd9b4e019ull;
    return s.next();
}

}  // namespace
}  // namespace mtgp_impl

using namespace mtgp_impl;

extern "C" int mtgp_search_params(uint32_t mexp, uint32_t id, uint64_t seed, uint64_t max_draws, uint32_t threads,
                                  mtgp_param_set *out, mtgp_search_stats *stats)
{
    if (!out || !is_prime(mexp) || mexp < 67 || mexp > 65536 || max_draws == 0)
        return MTGP_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    if (threads == 0) {
        // the CPUs this process may run on, at most 16
        cpu_set_t set;
        CPU_ZERO(&set);
        const int n = sched_getaffinity(0, sizeof(set), &set) == 0 ? CPU_COUNT(&set) : 1;
        threads = (uint32_t)std::min(16, std::max(1, n));
    }
    std::atomic<uint64_t> next{0};
    std::atomic<uint64_t> best{UINT64_MAX};
    std::atomic<uint64_t> n_full{0}, n_sieved{0}, n_tested{0};
    std::mutex mu;
    Candidate found{};
    auto work = [&]() {
        for (;;) {
            const uint64_t i = next.fetch_add(1);
            if (i >= max_draws || i >= best.load())
                return;
            SplitMix64 rng{candidate_seed(seed, id, i)};
            const Candidate c = draw(mexp, id, rng);
            const Outcome o = test(mexp, c);
            n_tested++;
            n_full += o.full_degree;
            n_sieved += o.sieved;
            if (o.found) {
                std::lock_guard<std::mutex> lock(mu);
                if (i < best.load()) {
                    best = i;
                    found = c;
                }
            }
        }
    };
    std::vector<std::thread> pool;
    for (uint32_t k = 1; k < threads; k++)
        pool.emplace_back(work);
    work();
    for (std::thread &t : pool)
        t.join();
    if (stats) {
        stats->draws = best.load() == UINT64_MAX ? max_draws : best.load() + 1;
        stats->evaluated = n_tested.load();
        stats->full_degree = n_full.load();
        stats->sieve_passed = n_sieved.load();
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (best.load() == UINT64_MAX)
        return MTGP_ENOTFOUND;
    out->mexp = mexp;
    out->pos = found.M;
    out->sh1 = kSh1;
    out->sh2 = kSh2;
    // tables in the parameter-set convention: entry 1 << b is basis word b,
    // so bit 3 of an index (the nibble's MSB) selects the first row
    for (uint32_t j = 0; j < 16; j++)
        out->param_tbl[j] = found.tbl[j];
    // a random F2-linear tempering table (the period does not depend on it)
    SplitMix64 rng{candidate_seed(seed, id, best.load()) ^ 0x5bd1e995ull};
    uint32_t trow[4];
    for (uint32_t a = 0; a < 4; a++)
        trow[a] = (uint32_t)rng.next();
    for (uint32_t j = 0; j < 16; j++) {
        uint32_t v = 0;
        for (uint32_t b = 0; b < 4; b++)
            if ((j >> b) & 1)
                v ^= trow[b];
        out->temper_tbl[j] = v;
    }
    return MTGP_OK;
}
