// Host-code self-test of the library's C++ sources that touch no device
// (F2 polynomial arithmetic, the parameter search, the dimension of
// equidistribution), built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_host_sanitizers.py. Prints "host selftest ok" and returns 0
// when every check holds.
#include "../../include/mtgp.h"
#include "../../paper_1005_4973_amd/csrc/mtgp_f2.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

using namespace mtgp_impl::f2;

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next64()
{
    // SplitMix64 (Steele, Lea, Flood 2014)
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static int failures = 0;
#define CHECK(c, ...)                                                       \
    do {                                                                    \
        if (!(c)) {                                                         \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);                \
            std::printf(__VA_ARGS__);                                       \
            std::printf("\n");                                              \
            failures++;                                                     \
        }                                                                   \
    } while (0)

static Poly random_poly(int64_t deg)
{
    Poly p;
    p.w.resize((size_t)(deg / 64 + 1));
    for (auto &w : p.w)
        w = next64();
    const int top = (int)(deg & 63);
    p.w.back() &= (top == 63) ? ~0ull : ((2ull << top) - 1);
    p.w.back() |= 1ull << top;   // degree exactly deg
    p.trim();
    return p;
}

static bool same(const Poly &a, const Poly &b) { return a.deg == b.deg && a.w == b.w; }

static void test_clmul()
{
    for (size_t na : {1u, 2u, 3u, 7u, 64u, 175u})
        for (size_t nb : {1u, 5u, 64u, 176u}) {
            std::vector<uint64_t> a(na), b(nb), r1(na + nb + 1), r2(na + nb + 1);
            for (auto &w : a)
                w = next64();
            for (auto &w : b)
                w = next64();
            clmul_reference(a.data(), na, b.data(), nb, r1.data());
            clmul_fast(a.data(), na, b.data(), nb, r2.data());
            CHECK(r1 == r2, "clmul %zu x %zu words", na, nb);
        }
    // Karatsuba against the shift-and-xor definition, around its base size
    // and through odd splits
    for (size_t n : {1u, 2u, 15u, 16u, 17u, 31u, 33u, 65u, 100u, 364u}) {
        std::vector<uint64_t> a(n), b(n), r1(2 * n + 1), r2(2 * n);
        for (auto &w : a)
            w = next64();
        for (auto &w : b)
            w = next64();
        clmul_reference(a.data(), n, b.data(), n, r1.data());
        clmul_karatsuba(a.data(), b.data(), n, r2.data());
        CHECK(r1[2 * n] == 0 && std::equal(r2.begin(), r2.end(), r1.begin()), "karatsuba %zu words", n);
    }
}

// ring operations against the plain definitions (mod of the plain product)
static void test_ring()
{
    // table reduction below 64, Barrett from 64 on (64, 128, 4096 and 11264
    // are word multiples)
    for (int64_t D : {8, 63, 64, 65, 127, 128, 521, 2203, 4095, 4096, 4097, 11213, 11214, 11264, 23209}) {
        const Poly m = random_poly(D);
        SquareMod ring(m);
        const size_t nw = ring.words();
        for (int t = 0; t < 4; t++) {
            const Poly a = mod(random_poly(D + 40), m), b = mod(random_poly(D + 7), m);
            std::vector<uint64_t> aw(nw, 0), bw(nw, 0), r(nw, 0);
            std::copy(a.w.begin(), a.w.end(), aw.begin());
            std::copy(b.w.begin(), b.w.end(), bw.begin());
            ring.mul(aw.data(), bw.data(), r.data());
            CHECK(same(Poly::from_words(r.data(), (int64_t)nw * 64 - 1), mod(mul(a, b), m)), "mul D=%lld",
                  (long long)D);
            ring.square(aw.data(), r.data());
            CHECK(same(Poly::from_words(r.data(), (int64_t)nw * 64 - 1), mod(mul(a, a), m)), "square D=%lld",
                  (long long)D);
            std::vector<uint64_t> xa = aw;
            ring.times_x(xa.data());
            Poly x;
            x.w = {2};
            x.deg = 1;
            CHECK(same(Poly::from_words(xa.data(), (int64_t)nw * 64 - 1), mod(mul(a, x), m)), "times_x D=%lld",
                  (long long)D);
        }
        // x^e mod m by the ring against e repeated multiplications by x
        Poly r = Poly::one();
        Poly x;
        x.w = {2};
        x.deg = 1;
        for (uint64_t e = 1; e <= 300; e++) {
            r = mod(mul(r, x), m);
            if (e % 37 == 0 || e == 300)
                CHECK(same(powmod_x(e, m), r), "powmod D=%lld e=%llu", (long long)D, (unsigned long long)e);
        }
        // a large exponent: x^(2^20) = (x^(2^10))^(2^10)
        Poly big = powmod_x(1u << 20, m), half = powmod_x(1u << 10, m), acc = half;
        for (int k = 0; k < 10; k++)
            acc = mod(mul(acc, acc), m);
        CHECK(same(big, acc), "powmod 2^20 D=%lld", (long long)D);
    }
}

// Berlekamp-Massey on the output of the LFSR of a known primitive
// trinomial, x^89 + x^38 + 1 (Zierler and Brillhart's table).
static void test_minpoly()
{
    const int64_t L = 89, n = 4 * L;
    std::vector<uint8_t> s((size_t)n, 0);
    s[0] = 1;
    for (int64_t i = L; i < n; i++)
        s[(size_t)i] = s[(size_t)(i - L)] ^ s[(size_t)(i - L + 38)];
    std::vector<uint64_t> bits((size_t)(n / 64 + 1), 0);
    for (int64_t i = 0; i < n; i++)
        if (s[(size_t)i])
            bits[(size_t)(i >> 6)] |= 1ull << (i & 63);
    const Poly phi = minpoly(bits.data(), n);
    CHECK(phi.deg == L && phi.bit(0) && phi.bit(38) && phi.bit(89), "minpoly degree %lld", (long long)phi.deg);
    int terms = 0;
    for (uint64_t w : phi.w)
        terms += __builtin_popcountll(w);
    CHECK(terms == 3, "minpoly terms %d", terms);
    bool sieved = false;
    CHECK(irreducible_prime_degree(phi, 10, &sieved) && sieved, "x^89 + x^38 + 1 irreducible");
    Poly red = phi;
    red.w[0] ^= 2;   // x^89 + x^38 + x + 1 has the root 1
    red.trim();
    CHECK(!irreducible_prime_degree(red, 10, &sieved), "reducible rejected");

    // against trial division by every polynomial of degree <= 8, for random
    // polynomials of the prime degree 17 (the sieve reaches p - 1 = 16 with
    // sieve 256, only 4 with sieve 4, none with 0)
    int irreducible = 0;
    for (int trial = 0; trial < 3000; trial++) {
        Poly m;
        m.w = {(next64() & 0x1ffffull) | (1ull << 17) | 1ull};
        m.trim();
        bool divisible = false;
        for (uint64_t dv = 2; dv < 512 && !divisible; dv++) {
            Poly dp;
            dp.w = {dv};
            dp.trim();
            Poly rem;
            divide(m, dp, &rem);
            divisible = rem.deg < 0;
        }
        for (uint32_t sv : {0u, 4u, 256u}) {
            const bool irr = irreducible_prime_degree(m, sv, nullptr);
            CHECK(irr == !divisible, "degree 17 poly %llx sieve %u", (unsigned long long)m.w[0], sv);
        }
        irreducible += !divisible;
    }
    CHECK(irreducible > 50, "degree 17: %d irreducible of 3000", irreducible);
    // the sieve only rejects: the same decisions at degree 89 without it
    for (int trial = 0; trial < 400; trial++) {
        Poly m = random_poly(89);
        m.w[0] |= 1;
        CHECK(irreducible_prime_degree(m, 0, nullptr) == irreducible_prime_degree(m, 256, nullptr),
              "degree 89 sieve 0 vs 256");
    }
}

static void test_search_and_equidistribution()
{
    mtgp_param_set ps;
    mtgp_search_stats st;
    std::memset(&ps, 0, sizeof(ps));
    const int rc = mtgp_search_params(521, 3, 12345, 200000, 4, &ps, &st);
    CHECK(rc == MTGP_OK, "search 521 rc=%d", rc);
    if (rc == MTGP_OK) {
        uint32_t k[32] = {0}, delta = 0;
        const int e = mtgp_equidistribution(&ps, 1, 32, k, &delta);
        CHECK(e == MTGP_OK, "equidistribution rc=%d", e);
        for (int v = 1; v <= 32 && e == MTGP_OK; v++)
            CHECK(k[v - 1] >= 1 && k[v - 1] <= 521u / (uint32_t)v, "k(%d) = %u", v, k[v - 1]);
    }
    CHECK(mtgp_search_params(520, 3, 1, 10, 1, &ps, &st) == MTGP_EINVAL, "even exponent rejected");
}

int main()
{
    test_clmul();
    test_ring();
    test_minpoly();
    test_search_and_equidistribution();
    if (failures) {
        std::printf("host selftest: %d failures\n", failures);
        return 1;
    }
    std::printf("host selftest ok\n");
    return 0;
}
