// Polynomials over F2 (host side) for jump-ahead: packed little-endian words,
// bit k of word k/64 is the coefficient of x^k.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace mtgp_impl {
namespace f2 {

struct Poly {
    std::vector<uint64_t> w;
    int64_t deg = -1;   // -1 for the zero polynomial

    bool bit(int64_t k) const
    {
        return k >= 0 && (size_t)(k >> 6) < w.size() && ((w[(size_t)(k >> 6)] >> (k & 63)) & 1);
    }
    void trim();
    static Poly one();
    static Poly from_words(const uint64_t *src, int64_t deg);
};

Poly mul(const Poly &a, const Poly &b);
Poly square(const Poly &a);
Poly mod(const Poly &a, const Poly &m);
Poly divide(const Poly &a, const Poly &m, Poly *rem);
Poly gcd(Poly a, Poly b);
Poly lcm(const Poly &a, const Poly &b);
Poly mulmod(const Poly &a, const Poly &b, const Poly &m);
Poly powmod_x(uint64_t e, const Poly &m);     // x^e mod m

// Minimal polynomial (characteristic form, monic, degree = linear complexity)
// of the bit sequence s_0 .. s_{n-1}, packed like a polynomial.
Poly minpoly(const uint64_t *bits, int64_t n);

// Arithmetic modulo a fixed polynomial m of degree D >= 8. From
// kBarrettMinDegree on, the reduction is Barrett's with Karatsuba products
// (two products of about D/64-word operands per reduction); below it, eight
// coefficients at a time: for every value c of the byte above x^D, the
// multiple q(c) m whose coefficients of x^D .. x^{D+7} spell c is stored
// pre-shifted for the eight byte positions within a 64-bit word, so one
// reduction step is one word-aligned XOR. (That table holds 2048 entries of
// D/64 words: at the generators' degrees it no longer fits in cache, and
// Barrett's form measured 4x to 19x faster from D = 521 to 44497.) Operands
// and results are reduced polynomials of words() words. Not thread-safe (one
// work buffer); build one per thread.
constexpr int64_t kBarrettMinDegree = 64;

class SquareMod {
public:
    explicit SquareMod(const Poly &m);
    size_t words() const { return nw_; }                         // words of a reduced polynomial
    void square(const uint64_t *a, uint64_t *r);                 // r = a^2 mod m
    void mul(const uint64_t *a, const uint64_t *b, uint64_t *r); // r = a b mod m
    void times_x(uint64_t *a);                                   // a = x a mod m, in place
    void reduce(uint64_t *t);   // t (2 words() + 2 words, degree <= 2D - 2) mod m, in its low words() words

private:
    int64_t D_;
    size_t nw_, tw_;                 // reduced words, table entry words
    std::vector<uint64_t> table_;    // [8 alignments][256 bytes][tw_ words]
    std::vector<uint64_t> work_;     // 2 nw_ + 2 words
    std::vector<uint64_t> m_;        // m's words
    std::vector<uint64_t> mu_;       // Barrett: floor(x^(2D) / m), nw_ + 1 words (empty: table reduction)
    std::vector<uint64_t> mpad_;     // Barrett: m in nw_ + 1 words
    std::vector<uint64_t> bar_;      // Barrett: products and Karatsuba scratch
};

// Carry-less products of word arrays (out has na + nb + 1 words): the
// shift-and-xor definition and the one the library uses (64-bit carry-less
// multiplications where the CPU has them), for checking one against the other.
void clmul_reference(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out);
void clmul_fast(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out);
// The Karatsuba form for two n-word operands (out has 2n words).
void clmul_karatsuba(const uint64_t *a, const uint64_t *b, size_t n, uint64_t *out);

// Irreducibility of m when its degree p is prime: m(0) = m(1) = 1, no factor
// of degree <= min(sieve, p - 1) (gcd(m, x^(2^k) - x) = 1 for those k, a
// filter that rejects most reducible m before the full test), and
// x^(2^p) = x mod m. *sieved is set when the sieve passed.
bool irreducible_prime_degree(const Poly &m, uint32_t sieve, bool *sieved);

}  // namespace f2
}  // namespace mtgp_impl
