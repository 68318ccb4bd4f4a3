// Polynomial arithmetic over F2 for jump-ahead, on the host.
//
// A jump of J steps maps a state S to F^J S. If psi is a polynomial with
// psi(F) S = 0, then F^J S = h(F) S for h = x^J mod psi, and h(F) S is the
// sum of the states S, F S, F^2 S, ... selected by h's coefficients -- a
// correlation of h with the stream of raw words (the paper's section 7 on
// jumping ahead; the minimal polynomial of a bit sequence comes from the
// Berlekamp-Massey algorithm, as in section 5).
//
// Polynomials are packed little-endian: bit k of word k/64 is the coefficient
// of x^k.
#include "mtgp_f2.h"

#include <immintrin.h>

#include <algorithm>
#include <array>
#include <cstring>

namespace mtgp_impl {
namespace f2 {

// ---------------------------------------------------------------------------
// basics
// ---------------------------------------------------------------------------

void Poly::trim()
{
    int64_t d = (int64_t)w.size() * 64 - 1;
    while (d >= 0 && !bit(d))
        d--;
    deg = d;
    w.resize(d < 0 ? 0 : (size_t)(d / 64 + 1));
}

Poly Poly::one()
{
    Poly p;
    p.w.assign(1, 1);
    p.deg = 0;
    return p;
}

Poly Poly::from_words(const uint64_t *src, int64_t deg)
{
    Poly p;
    if (deg < 0)
        return p;
    p.w.assign(src, src + deg / 64 + 1);
    p.trim();
    return p;
}

// dst ^= src << shift (dst must be large enough)
static void xor_shl(uint64_t *dst, const uint64_t *src, size_t nsrc, int64_t shift)
{
    const int64_t ws = shift >> 6;
    const int bs = (int)(shift & 63);
    if (bs == 0) {
        for (size_t i = 0; i < nsrc; i++)
            dst[ws + (int64_t)i] ^= src[i];
        return;
    }
    uint64_t carry = 0;
    for (size_t i = 0; i < nsrc; i++) {
        dst[ws + (int64_t)i] ^= (src[i] << bs) | carry;
        carry = src[i] >> (64 - bs);
    }
    if (carry)
        dst[ws + (int64_t)nsrc] ^= carry;
}

// Carry-less product by shift-and-xor over the set bits of b (the plain
// definition; the fallback where the CPU has no carry-less multiply).
static void clmul_words_plain(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out)
{
    std::memset(out, 0, (na + nb + 1) * sizeof(uint64_t));
    for (size_t j = 0; j < nb; j++) {
        uint64_t bw = b[j];
        while (bw) {
            const int t = __builtin_ctzll(bw);
            bw &= bw - 1;
            xor_shl(out, a, na, (int64_t)(j * 64 + t));
        }
    }
}

// The same product from 64 x 64-bit carry-less multiplications (x86
// PCLMULQDQ): word i of a times word j of b lands in words i + j and i + j + 1.
__attribute__((target("pclmul,sse4.1"))) static void clmul_words_pclmul(const uint64_t *a, size_t na,
                                                                         const uint64_t *b, size_t nb,
                                                                         uint64_t *out)
{
    std::memset(out, 0, (na + nb + 1) * sizeof(uint64_t));
    for (size_t i = 0; i < na; i++) {
        const __m128i ai = _mm_cvtsi64_si128((long long)a[i]);
        for (size_t j = 0; j < nb; j++) {
            const __m128i p = _mm_clmulepi64_si128(ai, _mm_cvtsi64_si128((long long)b[j]), 0x00);
            out[i + j] ^= (uint64_t)_mm_cvtsi128_si64(p);
            out[i + j + 1] ^= (uint64_t)_mm_extract_epi64(p, 1);
        }
    }
}

// n x n words -> 2n words, column by column: word k collects the low halves
// of the products a_i b_j with i + j = k and the high halves of those with
// i + j = k - 1, accumulated in a 128-bit register.
__attribute__((target("pclmul,sse4.1"))) static void clmul_square_pclmul(const uint64_t *a, const uint64_t *b,
                                                                          size_t n, uint64_t *out)
{
    __m128i carry = _mm_setzero_si128();
    for (size_t k = 0; k + 1 < 2 * n; k++) {
        __m128i acc = carry;
        const size_t i0 = k < n ? 0 : k - n + 1, i1 = k < n ? k : n - 1;
        for (size_t i = i0; i <= i1; i++)
            acc = _mm_xor_si128(acc, _mm_clmulepi64_si128(_mm_cvtsi64_si128((long long)a[i]),
                                                          _mm_cvtsi64_si128((long long)b[k - i]), 0x00));
        out[k] = (uint64_t)_mm_cvtsi128_si64(acc);
        carry = _mm_srli_si128(acc, 8);
    }
    out[2 * n - 1] = (uint64_t)_mm_cvtsi128_si64(carry);
}

static bool have_pclmul()
{
    static const bool yes = __builtin_cpu_supports("pclmul");
    return yes;
}

// out[0 .. na + nb] = a * b (carry-less)
static void clmul_words(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out)
{
    if (have_pclmul())
        clmul_words_pclmul(a, na, b, nb, out);
    else
        clmul_words_plain(a, na, b, nb, out);
}

// Karatsuba (A. Karatsuba and Yu. Ofman, 1962) over 64-bit words:
// out[0 .. 2n) = a * b for n-word a and b, from three half-size products per
// level; below kKaraBase words the word-by-word product above. ws holds at
// least kara_scratch(n) words.
constexpr size_t kKaraBase = 16;

static size_t kara_scratch(size_t n) { return 4 * n + 8 * 64; }

static void clmul_kara(const uint64_t *a, const uint64_t *b, size_t n, uint64_t *out, uint64_t *ws)
{
    if (n <= kKaraBase) {
        if (have_pclmul()) {
            clmul_square_pclmul(a, b, n, out);
        } else {
            uint64_t tmp[2 * kKaraBase + 1];
            clmul_words_plain(a, n, b, n, tmp);   // its top word is zero
            std::copy(tmp, tmp + 2 * n, out);
        }
        return;
    }
    const size_t h = n / 2, hh = n - h;   // low and high halves, hh >= h
    clmul_kara(a, b, h, out, ws);                      // a_lo b_lo -> out[0, 2h)
    clmul_kara(a + h, b + h, hh, out + 2 * h, ws);     // a_hi b_hi -> out[2h, 2n)
    uint64_t *as = ws, *bs = ws + hh, *z1 = ws + 2 * hh;
    for (size_t i = 0; i < hh; i++) {
        as[i] = a[h + i] ^ (i < h ? a[i] : 0);
        bs[i] = b[h + i] ^ (i < h ? b[i] : 0);
    }
    clmul_kara(as, bs, hh, z1, ws + 4 * hh);           // (a_lo + a_hi)(b_lo + b_hi)
    for (size_t i = 0; i < 2 * h; i++)
        z1[i] ^= out[i];
    for (size_t i = 0; i < 2 * hh; i++)
        z1[i] ^= out[2 * h + i];
    for (size_t i = 0; i < 2 * hh; i++)                // middle term at word h
        out[h + i] ^= z1[i];
}

void clmul_karatsuba(const uint64_t *a, const uint64_t *b, size_t n, uint64_t *out)
{
    std::vector<uint64_t> ws(kara_scratch(n));
    clmul_kara(a, b, n, out, ws.data());
}

void clmul_reference(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out)
{
    clmul_words_plain(a, na, b, nb, out);
}

void clmul_fast(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *out)
{
    clmul_words(a, na, b, nb, out);
}

Poly mul(const Poly &a, const Poly &b)
{
    Poly r;
    if (a.deg < 0 || b.deg < 0)
        return r;
    r.w.resize(a.w.size() + b.w.size() + 1);
    clmul_words(a.w.data(), a.w.size(), b.w.data(), b.w.size(), r.w.data());
    r.trim();
    return r;
}

Poly square(const Poly &a)
{
    Poly r;
    if (a.deg < 0)
        return r;
    r.w.assign(2 * a.w.size(), 0);
    for (size_t i = 0; i < a.w.size(); i++) {
        uint64_t v = a.w[i];
        uint64_t lo = 0, hi = 0;
        for (int k = 0; k < 32; k++) {
            lo |= ((v >> k) & 1ull) << (2 * k);
            hi |= ((v >> (k + 32)) & 1ull) << (2 * k);
        }
        r.w[2 * i] = lo;
        r.w[2 * i + 1] = hi;
    }
    r.trim();
    return r;
}

// a mod m by shift-and-xor from the top down.
Poly mod(const Poly &a, const Poly &m)
{
    Poly r = a;
    if (m.deg < 0 || r.deg < m.deg)
        return r;
    for (int64_t d = r.deg; d >= m.deg; d--)
        if (r.bit(d))
            xor_shl(r.w.data(), m.w.data(), m.w.size(), d - m.deg);
    r.trim();
    return r;
}

Poly divide(const Poly &a, const Poly &m, Poly *rem)
{
    Poly q, r = a;
    if (m.deg < 0)
        return q;
    if (r.deg >= m.deg) {
        q.w.assign((size_t)((r.deg - m.deg) / 64 + 1), 0);
        for (int64_t d = r.deg; d >= m.deg; d--)
            if (r.bit(d)) {
                xor_shl(r.w.data(), m.w.data(), m.w.size(), d - m.deg);
                q.w[(size_t)((d - m.deg) >> 6)] |= 1ull << ((d - m.deg) & 63);
            }
    }
    q.trim();
    r.trim();
    if (rem)
        *rem = r;
    return q;
}

Poly gcd(Poly a, Poly b)
{
    while (b.deg >= 0) {
        Poly r = mod(a, b);
        a = b;
        b = r;
    }
    return a;
}

Poly lcm(const Poly &a, const Poly &b)
{
    if (a.deg < 0)
        return b;
    if (b.deg < 0)
        return a;
    const Poly g = gcd(a, b);
    return mul(a, divide(b, g, nullptr));
}

Poly mulmod(const Poly &a, const Poly &b, const Poly &m) { return mod(mul(a, b), m); }

Poly powmod_x(uint64_t e, const Poly &m)
{
    if (m.deg >= 8) {
        // square-and-multiply-by-x in the ring of m, squarings by table
        SquareMod sm(m);
        const size_t nw = sm.words();
        std::vector<uint64_t> r(nw, 0), t(nw, 0);
        r[0] = 1;
        int top = 63;
        while (top >= 0 && !((e >> top) & 1))
            top--;
        for (int k = top; k >= 0; k--) {
            sm.square(r.data(), t.data());
            r.swap(t);
            if ((e >> k) & 1)
                sm.times_x(r.data());
        }
        return Poly::from_words(r.data(), (int64_t)nw * 64 - 1);
    }
    Poly r = Poly::one();
    if (m.deg <= 0)
        return Poly();
    r = mod(r, m);
    int top = 63;
    while (top >= 0 && !((e >> top) & 1))
        top--;
    for (int k = top; k >= 0; k--) {
        r = mod(square(r), m);
        if ((e >> k) & 1) {
            // r *= x
            Poly s;
            s.w.assign(r.w.size() + 1, 0);
            xor_shl(s.w.data(), r.w.data(), r.w.size(), 1);
            s.trim();
            r = mod(s, m);
        }
    }
    return r;
}

// ---------------------------------------------------------------------------
// Berlekamp-Massey (J. L. Massey, 1969) on a packed bit sequence.
// ---------------------------------------------------------------------------

Poly minpoly(const uint64_t *bits, int64_t n)
{
    // Work on the reversed sequence, so that s_j, s_{j-1}, ..., s_{j-L} is a
    // forward run of bits starting at reversed position n-1-j. The reversed
    // sequence is kept in 64 copies shifted by 0..63 bits, so the run at any
    // position is read as aligned words and the discrepancy is a tight
    // AND/XOR loop.
    const size_t nw = (size_t)(n / 64 + 4);
    std::vector<uint64_t> rs(nw + 1, 0);
    for (int64_t j = 0; j < n; j++)
        if ((bits[j >> 6] >> (j & 63)) & 1)
            rs[(size_t)((n - 1 - j) >> 6)] |= 1ull << ((n - 1 - j) & 63);
    std::vector<uint64_t> shifted(64 * nw);   // shifted[s * nw + k] = bits [64k + s, 64k + s + 64)
    for (int sft = 0; sft < 64; sft++)
        for (size_t k = 0; k < nw; k++)
            shifted[(size_t)sft * nw + k] = sft ? (rs[k] >> sft) | (rs[k + 1] << (64 - sft)) : rs[k];
    // C: connection polynomial (c_0 = 1) of degree <= L; B: the one before the
    // last length change, of degree <= LB (the length then). C needs n/64 + 4
    // words; only the low LB/64 + 1 words of B can be non-zero.
    std::vector<uint64_t> C(nw, 0), B(nw, 0), T(nw, 0);
    C[0] = 1;
    B[0] = 1;
    int64_t L = 0, LB = 0, m = 1;
    auto add_shifted_B = [&]() {
        const size_t nb = std::min(nw - (size_t)(m >> 6) - 1, (size_t)(LB / 64 + 1));
        xor_shl(C.data(), B.data(), nb, m);
    };
    for (int64_t j = 0; j < n; j++) {
        const int64_t base = n - 1 - j;
        const uint64_t *run = shifted.data() + (size_t)(base & 63) * nw + (size_t)(base >> 6);
        const size_t full = (size_t)(L / 64);   // words of C below the last, partial one
        uint64_t acc = 0;
        for (size_t w = 0; w < full; w++)
            acc ^= C[w] & run[w];
        const int top = (int)(L - (int64_t)full * 64);   // bits 0 .. top of the last word
        const uint64_t last = top == 63 ? ~0ull : ((1ull << (top + 1)) - 1);
        acc ^= C[full] & last & run[full];
        if (!__builtin_parityll(acc)) {
            m++;
        } else if (2 * L <= j) {
            // B <- C (its low L/64 + 1 words hold all of it), C <- C + x^m B
            const size_t cw = (size_t)(L / 64 + 1);
            std::copy(C.begin(), C.begin() + (ptrdiff_t)cw, T.begin());
            add_shifted_B();
            std::fill(B.begin(), B.begin() + (ptrdiff_t)(LB / 64 + 1), 0);
            std::copy(T.begin(), T.begin() + (ptrdiff_t)cw, B.begin());
            LB = L;
            L = j + 1 - L;
            m = 1;
        } else {
            add_shifted_B();
            m++;
        }
    }
    // characteristic form: phi(x) = x^L C(1/x), phi_i = c_{L-i}
    Poly phi;
    phi.w.assign((size_t)(L / 64 + 1), 0);
    for (int64_t i = 0; i <= L; i++)
        if ((C[(size_t)((L - i) >> 6)] >> ((L - i) & 63)) & 1)
            phi.w[(size_t)(i >> 6)] |= 1ull << (i & 63);
    phi.trim();
    return phi;
}

// ---------------------------------------------------------------------------
// Squaring modulo m, and the irreducibility test for prime degree.
// ---------------------------------------------------------------------------

// 16-bit spread of a byte: bit k moves to bit 2k (squaring over F2 only
// spreads the coefficients).
static const uint16_t *spread_table()
{
    // built once, thread-safely (function-local static initialisation)
    static const std::array<uint16_t, 256> t = [] {
        std::array<uint16_t, 256> v{};
        for (int c = 0; c < 256; c++) {
            uint16_t s = 0;
            for (int k = 0; k < 8; k++)
                s |= (uint16_t)(((c >> k) & 1) << (2 * k));
            v[(size_t)c] = s;
        }
        return v;
    }();
    return t.data();
}

SquareMod::SquareMod(const Poly &m) : D_(m.deg)
{
    spread_table();
    nw_ = (size_t)((D_ + 63) / 64);
    m_ = m.w;
    if (D_ >= kBarrettMinDegree) {
        // mu = floor(x^(2D) / m), degree D; m and mu padded to nw_ + 1 words
        Poly x2d;
        x2d.w.assign((size_t)(2 * D_ / 64 + 1), 0);
        x2d.w[(size_t)(2 * D_ >> 6)] = 1ull << ((2 * D_) & 63);
        x2d.deg = 2 * D_;
        const Poly mu = divide(x2d, m, nullptr);
        const size_t n1 = nw_ + 1;
        mu_.assign(n1, 0);
        std::copy(mu.w.begin(), mu.w.end(), mu_.begin());
        mpad_.assign(n1, 0);
        std::copy(m.w.begin(), m.w.end(), mpad_.begin());
        bar_.assign(6 * n1 + kara_scratch(n1), 0);
        tw_ = 0;
        work_.assign(2 * nw_ + 2, 0);
        return;
    }
    tw_ = (size_t)((D_ + 8 + 56) / 64 + 1);
    // q(c): the byte q with bits D .. D+7 of q m equal to c
    std::vector<uint8_t> q_of(256, 0);
    for (int q = 0; q < 256; q++) {
        int top = 0;
        for (int b = 0; b < 8; b++)
            if ((q >> b) & 1)
                for (int k = 0; k < 8; k++)
                    if (m.bit(D_ + k - b))
                        top ^= 1 << k;
        q_of[(size_t)top] = (uint8_t)q;
    }
    table_.assign(8 * 256 * tw_, 0);
    for (int a = 0; a < 8; a++)
        for (int c = 0; c < 256; c++) {
            uint64_t *dst = table_.data() + ((size_t)a * 256 + (size_t)c) * tw_;
            const int q = q_of[(size_t)c];
            for (int b = 0; b < 8; b++)
                if ((q >> b) & 1)
                    xor_shl(dst, m.w.data(), m.w.size(), 8 * a + b);
        }
    work_.assign(2 * nw_ + 2 + tw_, 0);
}

void SquareMod::square(const uint64_t *a, uint64_t *r)
{
    const uint16_t *sp = spread_table();
    uint64_t *t = work_.data();
    std::fill(work_.begin(), work_.end(), 0);
    for (size_t i = 0; i < nw_; i++) {
        const uint64_t v = a[i];
        uint64_t lo = 0, hi = 0;
        for (int k = 0; k < 4; k++) {
            lo |= (uint64_t)sp[(v >> (8 * k)) & 0xff] << (16 * k);
            hi |= (uint64_t)sp[(v >> (32 + 8 * k)) & 0xff] << (16 * k);
        }
        t[2 * i] = lo;
        t[2 * i + 1] = hi;
    }
    reduce(t);
    std::copy(t, t + nw_, r);
}

void SquareMod::mul(const uint64_t *a, const uint64_t *b, uint64_t *r)
{
    uint64_t *t = work_.data();
    std::fill(work_.begin(), work_.end(), 0);
    if (!mu_.empty())
        clmul_kara(a, b, nw_, t, bar_.data());   // 2 nw_ words, degree <= 2D - 2
    else
        clmul_words(a, nw_, b, nw_, t);          // 2 nw_ + 1 words
    reduce(t);
    std::copy(t, t + nw_, r);
}

void SquareMod::times_x(uint64_t *a)
{
    // a <<= 1, then clear x^D with one multiple of m (a is reduced: only
    // x^D can appear above degree D - 1)
    uint64_t carry = 0;
    for (size_t i = 0; i < nw_; i++) {
        const uint64_t v = a[i];
        a[i] = (v << 1) | carry;
        carry = v >> 63;
    }
    const bool top = ((D_ & 63) == 0) ? carry != 0 : ((a[(size_t)(D_ >> 6)] >> (D_ & 63)) & 1) != 0;
    if (top) {
        for (size_t i = 0; i < m_.size() && i < nw_; i++)
            a[i] ^= m_[i];
    }
}

// dst[0 .. nd) = (src >> shift) for src of ns words (zero beyond)
static void shr_words(const uint64_t *src, size_t ns, int64_t shift, uint64_t *dst, size_t nd)
{
    const size_t ws = (size_t)(shift >> 6);
    const int bs = (int)(shift & 63);
    for (size_t i = 0; i < nd; i++) {
        const size_t k = ws + i;
        uint64_t v = k < ns ? src[k] >> bs : 0;
        if (bs && k + 1 < ns)
            v |= src[k + 1] << (64 - bs);
        dst[i] = v;
    }
}

void SquareMod::reduce(uint64_t *t)
{
    if (!mu_.empty()) {
        // Barrett reduction over F2[x] (P. Barrett, 1986): for deg t <= 2D - 1
        // the quotient floor(t / m) is exactly floor(floor(t / x^D) mu / x^D),
        // with no correction step, so t mod m = t + q m in the low D bits
        const size_t n1 = nw_ + 1;
        uint64_t *th = bar_.data(), *p1 = th + n1, *q = p1 + 2 * n1, *p2 = q + n1, *ws = p2 + 2 * n1;
        shr_words(t, 2 * nw_ + 1, D_, th, n1);
        clmul_kara(th, mu_.data(), n1, p1, ws);
        shr_words(p1, 2 * n1, D_, q, n1);
        clmul_kara(q, mpad_.data(), n1, p2, ws);
        for (size_t i = 0; i < nw_; i++)
            t[i] ^= p2[i];
        return;
    }
    // clear the bytes above x^D, top down: byte j covers x^(D+8j) .. x^(D+8j+7)
    for (int64_t j = (D_ - 2) / 8; j >= 0; j--) {
        const int64_t e = D_ + 8 * j;
        const size_t wi = (size_t)(e >> 6);
        const int sh = (int)(e & 63);
        uint64_t c = t[wi] >> sh;
        if (sh > 56)
            c |= t[wi + 1] << (64 - sh);
        c &= 0xff;
        if (!c)
            continue;
        // q(c) m shifted by 8j: word offset 8j / 64, alignment (8j mod 64) / 8
        const int64_t s = 8 * j;
        const uint64_t *src = table_.data() + ((size_t)((s & 63) >> 3) * 256 + (size_t)c) * tw_;
        uint64_t *dst = t + (size_t)(s >> 6);
        for (size_t k = 0; k < tw_; k++)
            dst[k] ^= src[k];
    }
}

bool irreducible_prime_degree(const Poly &m, uint32_t sieve, bool *sieved)
{
    if (sieved)
        *sieved = false;
    const int64_t p = m.deg;
    if (p < 8 || !m.bit(0))
        return false;   // x divides m (or too small for the byte tables)
    int terms = 0;
    for (uint64_t w : m.w)
        terms += __builtin_popcountll(w);
    if ((terms & 1) == 0)
        return false;   // m(1) = 0: x + 1 divides m
    SquareMod sm(m);
    const size_t nw = sm.words();
    std::vector<uint64_t> r(nw, 0), t(nw, 0), acc(nw, 0), d(nw, 0);
    r[0] = 2;     // x
    acc[0] = 1;   // product of x^(2^k) - x since the last check
    // An irreducible factor of degree j divides x^(2^k) - x exactly when j
    // divides k. For k < p (p prime) an irreducible m has no such factor, so
    // the sieve stops below p. The terms are multiplied together and checked
    // with one gcd at k = 2, 4, 8, ... and at the sieve's end: m shares a
    // factor with the product iff it shares one with a term.
    const int64_t last = std::min<int64_t>(sieve, p - 1);
    int64_t check = 2;
    for (int64_t k = 1; k <= p; k++) {
        sm.square(r.data(), t.data());
        r.swap(t);
        if (k <= last) {
            d = r;
            d[0] ^= 2;
            sm.mul(acc.data(), d.data(), t.data());
            acc.swap(t);
            if (k == check || k == last) {
                Poly g;
                g.w = acc;
                g.trim();
                if (gcd(m, g).deg > 0)   // (g = 0: m divides the product)
                    return false;
                std::fill(acc.begin(), acc.end(), 0);
                acc[0] = 1;
                check *= 2;
            }
            if (k == last && sieved)
                *sieved = true;
        }
    }
    r[0] ^= 2;
    for (uint64_t w : r)
        if (w)
            return false;
    return true;
}

}  // namespace f2
}  // namespace mtgp_impl
