/*
 * F2 tools for checking the MTGP oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * - Berlekamp-Massey over F2 (J. L. Massey, "Shift-register synthesis and BCH
 *   decoding", IEEE Trans. IT 1969): the shortest linear recurrence of a bit
 *   sequence. The paper computes MTGP characteristic polynomials this way
 *   (section 5, recursion-parameter search).
 * - Irreducibility of a polynomial of prime degree p over F2: phi is
 *   irreducible iff it has no root in F2 and x^(2^p) = x (mod phi), because
 *   the only subfield of GF(2^p) is F2 when p is prime. With 2^p - 1 prime
 *   (p a Mersenne exponent) an irreducible phi is primitive, which is the
 *   period criterion of section 3.3 and section 5.
 *
 * Polynomials are bit arrays: bit k of word k/64 is the coefficient of x^k.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline int getbit(const uint64_t *a, int64_t k) { return (int)((a[k >> 6] >> (k & 63)) & 1u); }
static inline void flipbit(uint64_t *a, int64_t k) { a[k >> 6] ^= (uint64_t)1 << (k & 63); }

/* dst ^= src << shift, over `words` words of dst (src has `words` words too). */
static void xor_shifted(uint64_t *dst, const uint64_t *src, int64_t words, int64_t shift)
{
    int64_t ws = shift >> 6, bs = shift & 63;
    for (int64_t i = words - 1; i >= ws; i--) {
        uint64_t v = src[i - ws] << bs;
        if (bs && i - ws - 1 >= 0)
            v |= src[i - ws - 1] >> (64 - bs);
        dst[i] ^= v;
    }
}

/* 64 sequence bits starting at bit position `pos` of packed array s (bits
 * beyond `nbits` read as zero). */
static uint64_t window64(const uint64_t *s, int64_t nwords, int64_t pos)
{
    int64_t w = pos >> 6, b = pos & 63;
    uint64_t lo = (w < nwords) ? s[w] : 0;
    uint64_t hi = (w + 1 < nwords) ? s[w + 1] : 0;
    return b ? (lo >> b) | (hi << (64 - b)) : lo;
}

/*
 * Berlekamp-Massey. Input: n bits s[0..n-1], one byte each (0/1).
 * Output: connection polynomial C(x) = 1 + c_1 x + ... + c_L x^L written to
 * `conn` as bytes conn[0..L] (conn must hold n+1 bytes); returns L, the linear
 * complexity, so that s_i = sum_{j=1..L} c_j s_{i-j} for all L <= i < n.
 * Returns -1 on allocation failure.
 */
int64_t orc_bm(const uint8_t *s_bytes, int64_t n, uint8_t *conn)
{
    int64_t words = (n + 1 + 63) / 64 + 1;
    /* rs: the sequence reversed, so that the window of s_{i}, s_{i-1}, ...
     * is a contiguous run of rs starting at n-1-i. */
    uint64_t *rs = calloc((size_t)words, 8);
    uint64_t *C = calloc((size_t)words, 8);
    uint64_t *B = calloc((size_t)words, 8);
    uint64_t *T = calloc((size_t)words, 8);
    if (!rs || !C || !B || !T) {
        free(rs); free(C); free(B); free(T);
        return -1;
    }
    for (int64_t i = 0; i < n; i++)
        if (s_bytes[i] & 1)
            flipbit(rs, n - 1 - i);
    C[0] = 1;
    B[0] = 1;
    int64_t L = 0, m = 1;
    for (int64_t i = 0; i < n; i++) {
        /* discrepancy d = sum_{j=0..L} c_j s_{i-j} */
        uint64_t acc = 0;
        int64_t base = n - 1 - i;   /* rs[base + j] = s_{i-j} */
        for (int64_t j = 0; j <= L; j += 64) {
            uint64_t cw = C[j >> 6];
            uint64_t sw = window64(rs, words, base + j);
            if (L - j < 63)
                cw &= (((uint64_t)1 << (L - j + 1)) - 1);
            acc ^= cw & sw;
        }
        int d = __builtin_parityll(acc);
        if (!d) {
            m++;
        } else if (2 * L <= i) {
            memcpy(T, C, (size_t)words * 8);
            xor_shifted(C, B, words, m);
            L = i + 1 - L;
            memcpy(B, T, (size_t)words * 8);
            m = 1;
        } else {
            xor_shifted(C, B, words, m);
            m++;
        }
    }
    for (int64_t k = 0; k <= L; k++)
        conn[k] = (uint8_t)getbit(C, k);
    free(rs); free(C); free(B); free(T);
    return L;
}

/* a = a^2 mod phi, phi of degree p (bits), all arrays of `words` words;
 * tmp has 2*words words. */
static void sqr_mod(uint64_t *a, const uint64_t *phi, int64_t p, int64_t words, uint64_t *tmp)
{
    memset(tmp, 0, (size_t)(2 * words) * 8);
    for (int64_t k = 0; k < p; k++)
        if (getbit(a, k))
            flipbit(tmp, 2 * k);
    /* reduce degrees 2p-2 .. p */
    for (int64_t k = 2 * p - 2; k >= p; k--)
        if (getbit(tmp, k))
            xor_shifted(tmp, phi, 2 * words, k - p);   /* phi has x^p, clears bit k */
    memcpy(a, tmp, (size_t)words * 8);
}

/*
 * phi given as bytes phi[0..p] (coefficient of x^k), phi[p] = 1, p prime.
 * Returns 1 if irreducible, 0 if not, -1 on bad input / allocation failure.
 */
int orc_irreducible_prime_degree(const uint8_t *phi_bytes, int64_t p)
{
    if (p < 2 || !(phi_bytes[p] & 1))
        return -1;
    if (!(phi_bytes[0] & 1))
        return 0;                         /* x divides phi */
    int ones = 0;
    for (int64_t k = 0; k <= p; k++)
        ones ^= phi_bytes[k] & 1;
    if (!ones)
        return 0;                         /* x + 1 divides phi */
    int64_t words = (2 * p + 64) / 64 + 1;
    uint64_t *phi = calloc((size_t)(2 * words), 8);
    uint64_t *a = calloc((size_t)words, 8);
    uint64_t *tmp = calloc((size_t)(2 * words), 8);
    if (!phi || !a || !tmp) {
        free(phi); free(a); free(tmp);
        return -1;
    }
    for (int64_t k = 0; k <= p; k++)
        if (phi_bytes[k] & 1)
            flipbit(phi, k);
    flipbit(a, 1);                        /* a = x */
    for (int64_t i = 0; i < p; i++)
        sqr_mod(a, phi, p, words, tmp);   /* a = x^(2^(i+1)) mod phi */
    int is_x = getbit(a, 1);
    for (int64_t k = 0; k < p && is_x; k++)
        if (k != 1 && getbit(a, k))
            is_x = 0;
    free(phi); free(a); free(tmp);
    return is_x;
}
