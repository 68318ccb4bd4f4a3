/*
 * MTGP oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, deliberately unoptimised CPU implementation of what the
 * MTGP generator computes, written from the paper's definitions. It exists to
 * check the HIP library; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it. It shares no code, header, table or constant
 * generator with the library.
 *
 * Sources in the paper (Saito & Matsumoto, "Variants of Mersenne Twister
 * Suitable for Graphic Processors"):
 *   - N = ceil(p/w), r = wN - p, BITMASK(w,r): section 3.3 (Notation) and 3.6.
 *   - recursion: Definition "recursion parameters", section 3.6, equations
 *     (algolrec) and its C form (algolrec-C).
 *   - tempering: Definition "tempering parameter", section 3.7, equations
 *     (mtgp-tempering), (algoltmp) and the C form (algoltmp-C).
 *   - single precision output: section 6, equation (C): the float table has
 *     nine MSBs 001111111 followed by MSBs of the tempering table; 1.0 is
 *     subtracted for [0,1).
 *   - continuation: section 8 (the state is stored back after each call).
 *
 * Readings where the paper is silent or garbled (each listed in the design
 * notes):
 *   - seeding is not specified by the paper; the state x_0..x_{N-1} is filled
 *     with the MT19937 initialisation recurrence (Matsumoto & Nishimura):
 *     x_0 = seed, x_i = 1812433253 * (x_{i-1} ^ (x_{i-1} >> 30)) + i.
 *   - section 6 says the float table keeps "27" MSBs of tmptbl, which cannot
 *     fit after a 9-bit prefix; the reading taken is 23 (the fraction width).
 *   - output k (k = 0, 1, ...) of a fresh generator is o_{N+k}; the N seed
 *     words are never emitted.
 *
 * Evaluation here is the definition itself: an array x[0 .. N+n) is filled in
 * index order, x[N+i] from x[M+i], x[1+i] and x[i] (section 3.1), and each
 * output is tempered with x[M-1+i]. The two products with 4 x w matrices
 * (the recursion's (u's four LSBs) R and the tempering's (t's four LSBs) T)
 * are formed as the definitions state them, a row vector times a matrix:
 * the XOR of the rows of R (or T) that the four bits select. The parameter
 * set carries R and T as the 16 products (0000)R .. (1111)R (and likewise
 * for T), as the paper stores them; the rows are read off the products of
 * the unit vectors, and a table that is not the product table of its rows is
 * rejected.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t mexp;            /* Mersenne exponent p */
    uint32_t pos;             /* middle position M */
    uint32_t sh1, sh2;        /* shift parameters */
    uint32_t param_tbl[16];   /* rectbl: (b3 b2 b1 b0) R for the 16 nibbles */
    uint32_t temper_tbl[16];  /* tmptbl: (b3 b2 b1 b0) T */
} orc_params;

enum { ORC_U32 = 0, ORC_F12 = 1, ORC_F01 = 2 };

/* N = ceil(p / w) with w = 32 (section 3.3). */
uint32_t orc_nwords(uint32_t mexp) { return (mexp + 31u) / 32u; }

/* MT19937 initialisation recurrence (seeding reading, see header). */
void orc_seed(uint32_t seed, uint32_t nwords, uint32_t *x)
{
    x[0] = seed;
    for (uint32_t i = 1; i < nwords; i++)
        x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + i;
}

/* A 4 x 32 matrix over F2 as its rows row[0] (top) .. row[3] (bottom). */
typedef struct {
    uint32_t row[4];
} orc_mat4;

/* The row vector (b_0 b_1 b_2 b_3) of the four LSBs of v, written most
 * significant first (b_0 = bit 3 of v, b_3 = bit 0), times the matrix:
 * the XOR of the rows j with b_j = 1 (sections 3.6 and 3.7). Each row is
 * taken through the mask 0 - b_j (all ones when b_j = 1, zero otherwise),
 * so the selection needs no branch on the data. */
static uint32_t orc_vec4_times(uint32_t v, const orc_mat4 *a)
{
    uint32_t acc = 0;
    for (int j = 0; j < 4; j++)
        acc ^= a->row[j] & (0u - ((v >> (3 - j)) & 1u));
    return acc;
}

/* The matrix whose product table is tbl[0..15] (tbl[v] = (v as a 4-bit row
 * vector) times the matrix): row j is the product of the unit vector with its
 * one at position j, i.e. tbl[1 << (3 - j)]. Returns -1 if tbl is not the
 * product table of those rows (it then describes no matrix). */
static int orc_matrix_of(const uint32_t tbl[16], orc_mat4 *a)
{
    for (int j = 0; j < 4; j++)
        a->row[j] = tbl[1u << (3 - j)];
    for (uint32_t v = 0; v < 16; v++)
        if (orc_vec4_times(v, a) != tbl[v])
            return -1;
    return 0;
}

/* One output word of kind `kind` from x_{N+i} (new word) and x_{M-1+i}
 * (the tempering word), section 3.7 (Definition of the tempering parameter)
 * and section 6. */
static uint32_t orc_output(const orc_mat4 *T, uint32_t x_new, uint32_t x_tmp, int kind)
{
    uint32_t t = x_tmp ^ (x_tmp >> 16);
    t = t ^ (t >> 8);
    const uint32_t h = orc_vec4_times(t, T);   /* h(x_{M-1+i}) = (t's four LSBs) T */
    if (kind == ORC_U32)
        return x_new ^ h;

    /* Section 6: the single-precision table entry has the nine MSBs
     * 001111111 and then the 23 MSBs of the tempering value; the output is
     * (x >> 9) ^ that entry. */
    uint32_t sngl = 0x3f800000u | (h >> 9);
    uint32_t bits = (x_new >> 9) ^ sngl;
    if (kind == ORC_F12)
        return bits;

    float f;
    memcpy(&f, &bits, 4);
    f = f - 1.0f;            /* section 6: subtract 1.0 for [0,1) */
    memcpy(&bits, &f, 4);
    return bits;
}

/*
 * Generate n outputs of `kind` from `state` (N words x_0..x_{N-1} in sequence
 * order), and replace `state` with x_n..x_{n+N-1} so that a later call
 * continues the stream (section 8). Returns 0, or -1 for parameters outside
 * the definition (M not in [2, N-1], shift above 31, mexp < 65), -2 on
 * allocation failure.
 */
int orc_generate(const orc_params *p, uint32_t *state, uint64_t n, int kind, uint32_t *out)
{
    if (p->mexp < 65 || p->sh1 > 31 || p->sh2 > 31 || kind < 0 || kind > 2)
        return -1;
    const uint64_t N = orc_nwords(p->mexp);
    const uint64_t M = p->pos;
    if (M < 2 || M > N - 1)
        return -1;
    orc_mat4 R, T;
    if (orc_matrix_of(p->param_tbl, &R) != 0 || orc_matrix_of(p->temper_tbl, &T) != 0)
        return -1;
    const uint32_t r = (uint32_t)(32u * N - p->mexp);
    const uint32_t mask = 0xffffffffu << r;   /* BITMASK(w,r): w-r MSBs set */

    uint32_t *x = (uint32_t *)malloc((size_t)(N + n) * sizeof(uint32_t));
    if (!x)
        return -2;
    memcpy(x, state, (size_t)N * sizeof(uint32_t));

    for (uint64_t i = 0; i < n; i++) {
        /* recursion, section 3.6 (Definition of the recursion parameters),
         * its four steps in the stated order: the w - r MSBs of x_i with r
         * zero bits, the sh1 and sh2 shifts, then u plus (u's four LSBs) R */
        uint32_t t = x[1 + i] ^ (x[i] & mask);
        t = t ^ (t << p->sh1);
        uint32_t u = t ^ (x[M + i] >> p->sh2);
        x[N + i] = u ^ orc_vec4_times(u, &R);
        /* tempering with x_{M-1+i}, section 3.7 */
        out[i] = orc_output(&T, x[N + i], x[M - 1 + i], kind);
    }

    memcpy(state, x + n, (size_t)N * sizeof(uint32_t));
    free(x);
    return 0;
}

/* Same recursion, but only advance the state (no output array). */
int orc_advance(const orc_params *p, uint32_t *state, uint64_t n)
{
    const uint64_t chunk = 1u << 20;
    uint32_t *scratch = (uint32_t *)malloc((size_t)chunk * sizeof(uint32_t));
    if (!scratch)
        return -2;
    int rc = 0;
    while (n > 0 && rc == 0) {
        uint64_t k = n < chunk ? n : chunk;
        rc = orc_generate(p, state, k, ORC_U32, scratch);
        n -= k;
    }
    free(scratch);
    return rc;
}

/*
 * Bit sequence for Berlekamp-Massey: bit `bit` (0 = LSB) of the first n
 * uint32 outputs, one byte per bit.
 */
int orc_output_bits(const orc_params *p, const uint32_t *state, uint64_t n, int bit, uint8_t *bits)
{
    const uint32_t N = orc_nwords(p->mexp);
    uint32_t *st = (uint32_t *)malloc(N * sizeof(uint32_t));
    uint32_t *o = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (!st || !o) {
        free(st);
        free(o);
        return -2;
    }
    memcpy(st, state, N * sizeof(uint32_t));
    int rc = orc_generate(p, st, n, ORC_U32, o);
    for (uint64_t i = 0; rc == 0 && i < n; i++)
        bits[i] = (uint8_t)((o[i] >> bit) & 1u);
    free(st);
    free(o);
    return rc;
}
