/* The C oracle (oracle/mtgp_oracle.c, oracle/f2.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: generation of every kind across lengths and
 * continuation, the bit sequences and Berlekamp-Massey, the irreducibility
 * test. Built and run by tests/test_host_sanitizers.py; prints "oracle
 * selftest ok" and returns 0 when the checks hold. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t mexp, pos, sh1, sh2;
    uint32_t param_tbl[16];
    uint32_t temper_tbl[16];
} orc_params;

uint32_t orc_nwords(uint32_t mexp);
void orc_seed(uint32_t seed, uint32_t nwords, uint32_t *x);
int orc_generate(const orc_params *p, uint32_t *state, uint64_t n, int kind, uint32_t *out);
int orc_advance(const orc_params *p, uint32_t *state, uint64_t n);
int orc_output_bits(const orc_params *p, const uint32_t *state, uint64_t n, int bit, uint8_t *bits);
int64_t orc_bm(const uint8_t *s_bytes, int64_t n, uint8_t *conn);
int orc_irreducible_prime_degree(const uint8_t *phi_bytes, int64_t p);

static uint32_t lcg = 12345u;
static uint32_t rnd(void) { lcg = lcg * 1664525u + 1013904223u; return lcg; }

static void span(uint32_t rows[4], uint32_t tbl[16])
{
    for (uint32_t v = 0; v < 16; v++) {
        uint32_t acc = 0;
        for (int b = 0; b < 4; b++)
            if ((v >> b) & 1u)
                acc ^= rows[b];
        tbl[v] = acc;
    }
}

int main(void)
{
    int fails = 0;
    const uint32_t mexps[3] = {89, 521, 11213};
    for (int e = 0; e < 3; e++) {
        orc_params p;
        memset(&p, 0, sizeof(p));
        p.mexp = mexps[e];
        const uint32_t N = orc_nwords(p.mexp);
        p.pos = 2 + rnd() % (N - 2);
        p.sh1 = 1 + rnd() % 31;
        p.sh2 = 1 + rnd() % 31;
        uint32_t r[4], t[4];
        for (int k = 0; k < 4; k++) {
            r[k] = rnd();
            t[k] = rnd();
        }
        span(r, p.param_tbl);
        span(t, p.temper_tbl);
        uint32_t *st = malloc(N * 4), *st2 = malloc(N * 4), *out = malloc(5000 * 4), *out2 = malloc(5000 * 4);
        orc_seed(7, N, st);
        memcpy(st2, st, N * 4);
        for (int kind = 0; kind < 3; kind++)
            if (orc_generate(&p, st, 1000, kind, out) != 0)
                fails++;
        /* continuation: 3000 at once equals the three calls above */
        if (orc_generate(&p, st2, 3000, 0, out2) != 0)
            fails++;
        if (memcmp(st, st2, N * 4) != 0) {
            printf("FAIL continuation p=%u\n", p.mexp);
            fails++;
        }
        if (orc_advance(&p, st, 5000) != 0)
            fails++;
        /* bit sequences and Berlekamp-Massey: degree at most p */
        const int64_t nb = 2 * (int64_t)p.mexp + 64;
        uint8_t *bits = malloc((size_t)nb), *conn = calloc((size_t)nb + 1, 1);   /* one byte per bit */
        if (orc_output_bits(&p, st, (uint64_t)nb, 0, bits) != 0)
            fails++;
        const int64_t L = orc_bm(bits, nb, conn);
        if (L < 1 || L > (int64_t)p.mexp) {
            printf("FAIL bm degree %lld p=%u\n", (long long)L, p.mexp);
            fails++;
        }
        free(bits);
        free(conn);
        /* a table that is no matrix's product table is rejected */
        p.temper_tbl[7] ^= 0x40;
        if (orc_generate(&p, st, 10, 0, out) == 0) {
            printf("FAIL non-linear table accepted\n");
            fails++;
        }
        free(st);
        free(st2);
        free(out);
        free(out2);
    }
    /* x^89 + x^38 + 1 is irreducible; x^89 + x^38 + x + 1 is not (root 1) */
    uint8_t phi[90];   /* one byte per coefficient */
    memset(phi, 0, sizeof(phi));
    phi[0] = phi[38] = phi[89] = 1;
    if (orc_irreducible_prime_degree(phi, 89) != 1) {
        printf("FAIL trinomial irreducible\n");
        fails++;
    }
    phi[1] = 1;
    if (orc_irreducible_prime_degree(phi, 89) != 0) {
        printf("FAIL reducible accepted\n");
        fails++;
    }
    if (fails) {
        printf("oracle selftest: %d failures\n", fails);
        return 1;
    }
    printf("oracle selftest ok\n");
    return 0;
}
