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

}  // namespace f2
}  // namespace mtgp_impl
