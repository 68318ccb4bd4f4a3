"""Pins of the oracle against what the paper and the mathematics fix (no GPU).

Each test names the property it pins and the passage it comes from. The
oracle is the C implementation in oracle/mtgp_oracle.c; oracle/pyref.py is a
second reading in the paper's matrix notation.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import pyref as P
from paper_1005_4973_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ps_of(d):
    return I.ParamSet(d["mexp"], d["pos"], d["sh1"], d["sh2"], tuple(d["param_tbl"]), tuple(d["temper_tbl"]))


def fullperiod_sets():
    with open(os.path.join(GOLDEN, "fullperiod_sets.json")) as f:
        return [ps_of(d) for d in json.load(f)["sets"]]


def table_of(rows):
    return tuple(I.span_table(rows))


# ---------------------------------------------------------------------------
# Worked examples traced by hand from section 3.6 (recursion) and section 3.7
# (tempering), the products with R and T written as their product tables
# (rectbl, tmptbl). N = 3 (p = 89, r = 7, BITMASK = 0xffffff80), M = 2.
# ---------------------------------------------------------------------------

def test_hand_trace_small_words():
    # rectbl[j] = j << 4, tmptbl[j] = j << 8; state (x0, x1, x2) = (0, 1, 0); sh1 = sh2 = 1.
    #  i=0: t = 1 ^ (0 & mask) = 1; t ^= t<<1 -> 3; u = 3 ^ (x2>>1) = 3; x3 = 3 ^ 0x30 = 0x33;
    #       tempering word x1 = 1 -> nibble 1 -> o = 0x33 ^ 0x100 = 0x133
    #  i=1: t = 0 ^ (1 & mask) = 0; u = 0 ^ (0x33>>1) = 0x19; x4 = 0x19 ^ 0x90 = 0x89;
    #       tempering word x2 = 0 -> o = 0x89
    #  i=2: t = 0x33; t ^= 0x66 -> 0x55; u = 0x55 ^ (0x89>>1 = 0x44) = 0x11; x5 = 0x11 ^ 0x10 = 0x01;
    #       tempering word x3 = 0x33 -> nibble 3 -> o = 0x01 ^ 0x300 = 0x301
    #  i=3: t = 0x89 ^ (0x33 & mask = 0) = 0x89; t ^= 0x112 -> 0x19b; u = 0x19b ^ (0x01>>1) = 0x19b;
    #       x6 = 0x19b ^ rectbl[0xb] = 0x19b ^ 0xb0 = 0x12b;
    #       tempering word x4 = 0x89 -> nibble 9 -> o = 0x12b ^ 0x900 = 0x82b
    ps = I.ParamSet(89, 2, 1, 1, table_of([0x10, 0x20, 0x40, 0x80]), table_of([0x100, 0x200, 0x400, 0x800]))
    st = np.array([0, 1, 0], dtype=np.uint32)
    out = O.generate(ps, st, 4)
    assert [hex(v) for v in out] == ["0x133", "0x89", "0x301", "0x82b"]
    assert [hex(v) for v in st] == ["0x89", "0x1", "0x12b"]


def test_hand_trace_mask_and_tempering_shifts():
    # rectbl[j] = j << 28, tmptbl[j] = j; state (0xffffffff, 0, 0x00010200); sh1 = 3, sh2 = 5.
    #  i=0: t = 0 ^ (0xffffffff & 0xffffff80) = 0xffffff80; t ^= t<<3 (0xfffffc00) -> 0x380;
    #       u = 0x380 ^ (0x00010200>>5 = 0x810) = 0xb90; nibble 0 -> x3 = 0xb90;
    #       tempering word x1 = 0 -> o = 0xb90
    #  i=1: t = 0x00010200 ^ (0 & mask) ; t ^= t<<3 (0x00081000) -> 0x00091200;
    #       u = 0x00091200 ^ (0xb90>>5 = 0x5c) = 0x0009125c; nibble 0xc -> x4 = 0xc009125c;
    #       tempering word x2 = 0x00010200: t = 0x00010201; t ^= t>>8 (0x102) -> 0x00010303;
    #       nibble 3 -> o = 0xc009125c ^ 3 = 0xc009125f
    #  i=2: t = 0xb90 ^ (0x00010200 & mask) = 0x00010990; t ^= t<<3 (0x00084c80) -> 0x00094510;
    #       u = 0x00094510 ^ (0xc009125c>>5 = 0x06004892) = 0x06090d82; nibble 2 -> x5 = 0x26090d82;
    #       tempering word x3 = 0xb90: t = 0xb90; t ^= 0xb -> 0xb9b; nibble 0xb -> o = 0x26090d89
    ps = I.ParamSet(89, 2, 3, 5, table_of([1 << 28, 1 << 29, 1 << 30, 1 << 31]), table_of([1, 2, 4, 8]))
    st = np.array([0xFFFFFFFF, 0, 0x00010200], dtype=np.uint32)
    out = O.generate(ps, st, 3)
    assert [hex(v) for v in out] == ["0xb90", "0xc009125f", "0x26090d89"]


# ---------------------------------------------------------------------------
# Two readings of the paper agree: the oracle (the definitions' steps, the
# 4 x w products by row selection) vs pyref (the transition and output as
# bit matrices).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mexp", [65, 89, 107, 127, 521, 607, 608])
def test_definition_steps_equal_matrix_form(mexp):
    # 65 and 608 are the extremes of the mask: r = 31 (one bit of x_i kept)
    # and r = 0 (the whole word)
    for s in range(3):
        ps = I.draw_param_set(mexp, I.SplitMix64(31 * mexp + s), I.M_POLICY_FULL)
        st = O.seed_state(100 + s, mexp)
        for kind in (O.U32, O.F12, O.F01):
            a = O.generate(ps, st.copy(), 150, kind)
            b, fin = P.generate(ps, list(st), 150, kind)
            np.testing.assert_array_equal(a, b)
        st2 = st.copy()
        O.generate(ps, st2, 150)
        np.testing.assert_array_equal(st2, fin)


# ---------------------------------------------------------------------------
# P1: F2-linearity (section 3.3: transition and output are F2-linear).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mexp", [11213, 23209, 44497])
def test_f2_linearity(mexp):
    ps = I.draw_param_set(mexp, I.SplitMix64(mexp), I.M_POLICY_WIDE)
    N = O.nwords(mexp)
    s1 = I.random_state(N, 1)
    s2 = I.random_state(N, 2)
    s12 = s1 ^ s2
    n = 3 * N + 17
    a1, a2, a12 = s1.copy(), s2.copy(), s12.copy()
    o1 = O.generate(ps, a1, n)
    o2 = O.generate(ps, a2, n)
    o12 = O.generate(ps, a12, n)
    np.testing.assert_array_equal(o12, o1 ^ o2)
    np.testing.assert_array_equal(a12, a1 ^ a2)
    # float [1,2) bits are affine: constant 0x3f800000 survives an odd XOR count
    f1 = O.generate(ps, s1.copy(), n, O.F12)
    f2 = O.generate(ps, s2.copy(), n, O.F12)
    f12 = O.generate(ps, s12.copy(), n, O.F12)
    np.testing.assert_array_equal(f12, f1 ^ f2 ^ np.uint32(0x3F800000))


# ---------------------------------------------------------------------------
# P2: the state has p = 32N - r dimensions (section 3.3), so every output bit
# sequence has a minimal polynomial of degree <= p. With r = 0 (no masked
# bits) the same parameters give degrees above p, which shows the test sees
# a dropped mask.
# ---------------------------------------------------------------------------

def test_bm_degree_at_most_p():
    ps = I.single_stream()[0][0]
    N = O.nwords(ps.mexp)
    st = O.seed_state(1234, ps.mexp)
    nbits = 2 * 32 * N
    for bit in (0, 7, 31):
        L, _ = O.berlekamp_massey(O.output_bits(ps, st, nbits, bit))
        assert L <= ps.mexp, (bit, L)
        assert L > ps.mexp // 2        # a synthetic set need not reach p, but is far from trivial
    # planted: the full-period sets (degree exactly p, irreducible; see the
    # period test) lose that property when their masked bits are kept
    # (p' = 32N, r = 0), so a dropped mask cannot pass the period test
    for fp in fullperiod_sets():
        Nf = O.nwords(fp.mexp)
        unmasked = I.ParamSet(32 * Nf, fp.pos, fp.sh1, fp.sh2, fp.param_tbl, fp.temper_tbl)
        stf = O.seed_state(1234, fp.mexp)
        L, conn = O.berlekamp_massey(O.output_bits(unmasked, stf, 2 * 32 * Nf + 64, 0))
        assert L != fp.mexp or not O.irreducible_prime_degree(O.char_poly_from_conn(conn)), fp.mexp


# ---------------------------------------------------------------------------
# P3: period 2^p - 1 (section 3.3 criterion; section 5: Mersenne p makes an
# irreducible characteristic polynomial primitive).
# ---------------------------------------------------------------------------

def test_fullperiod_sets_bm_and_irreducible():
    for ps in fullperiod_sets():
        p = ps.mexp
        st = O.seed_state(42, p)
        polys = set()
        for bit in range(32):
            L, conn = O.berlekamp_massey(O.output_bits(ps, st, 2 * p + 64, bit))
            assert L == p, (p, bit, L)
            polys.add(conn.tobytes())
        assert len(polys) == 1           # one characteristic polynomial for all bits
        phi = O.char_poly_from_conn(np.frombuffer(polys.pop(), dtype=np.uint8))
        assert O.irreducible_prime_degree(phi)


def test_irreducibility_test_against_trinomials_and_brute_force():
    # primitive trinomials x^p + x^k + 1 for Mersenne exponents p (Zierler-Brillhart tables)
    for p, k in [(89, 38), (127, 1), (521, 32), (607, 105), (1279, 216)]:
        phi = np.zeros(p + 1, dtype=np.uint8)
        phi[[0, k, p]] = 1
        assert O.irreducible_prime_degree(phi)
        phi[k] = 0
        phi[k + 1] = 1
        if (p, k + 1) not in [(127, 7)]:
            assert not O.irreducible_prime_degree(phi)

    # small prime degrees: compare with trial division by every lower-degree polynomial
    def poly_mod(a, b):
        db = b.bit_length() - 1
        while a and a.bit_length() - 1 >= db:
            a ^= b << (a.bit_length() - 1 - db)
        return a

    for p in (5, 7, 11, 13):
        for f in range(1 << p, 1 << (p + 1)):
            brute = all(poly_mod(f, g) != 0 for g in range(2, 1 << (p // 2 + 1)))
            coeffs = np.array([(f >> k) & 1 for k in range(p + 1)], dtype=np.uint8)
            assert O.irreducible_prime_degree(coeffs) == brute, (p, f)


def test_berlekamp_massey_brute_force_tiny():
    # linear complexity by exhaustive search over recurrences of each length
    rng = I.SplitMix64(5)
    for _ in range(60):
        n = 12
        s = [rng.next_u32() & 1 for _ in range(n)]
        best = None
        for L in range(0, n + 1):
            for c in range(1 << L):
                ok = all(s[i] == (sum(((c >> (j - 1)) & 1) * s[i - j] for j in range(1, L + 1)) & 1)
                         for i in range(L, n))
                if ok:
                    best = L
                    break
            if best is not None:
                break
        L, _ = O.berlekamp_massey(s)
        assert L == best


# ---------------------------------------------------------------------------
# P4: brute-force transition matrices on toy instances (section 3.3: the
# recursion is the iteration of a fixed linear map F on F2^p).
# ---------------------------------------------------------------------------

def oracle_step(ps):
    def step(words):
        st = np.array(words, dtype=np.uint32)
        O.generate(ps, st, 1)
        return [int(v) for v in st]
    return step


def pyref_step(ps):
    def step(words):
        _, fin = P.generate(ps, words, 1)
        return [int(v) for v in fin]
    return step


def test_transition_matrix_two_readings_and_powers():
    for mexp in (89, 107):
        ps = I.draw_param_set(mexp, I.SplitMix64(mexp * 7), I.M_POLICY_FULL)
        N = O.nwords(mexp)
        r = 32 * N - mexp
        F1 = P.transition_matrix(oracle_step(ps), N, r)
        F2 = P.transition_matrix(pyref_step(ps), N, r)
        np.testing.assert_array_equal(F1, F2)
        st = O.seed_state(9, mexp)
        v0 = P.state_to_pvec(list(st), r)
        for k in (1, 2, 5, 40, 333):
            s = st.copy()
            O.advance(ps, s, k)
            np.testing.assert_array_equal(P.state_to_pvec(list(s), r), P.matmul2(v0[None, :], P.matpow2(F1, k))[0])


def test_fullperiod_transition_order():
    for ps in fullperiod_sets():
        if ps.mexp > 127:
            continue
        N = O.nwords(ps.mexp)
        r = 32 * N - ps.mexp
        F = P.transition_matrix(oracle_step(ps), N, r)
        eye = np.eye(F.shape[0], dtype=np.uint8)
        assert not np.array_equal(F, eye)
        np.testing.assert_array_equal(P.matpow2(F, (1 << ps.mexp) - 1), eye)
    # a set rejected by the search has no such order (generic case)
    ps = I.draw_param_set(89, I.SplitMix64(3), I.M_POLICY_FULL)
    st = O.seed_state(1, 89)
    L, conn = O.berlekamp_massey(O.output_bits(ps, st, 2 * 89 + 64, 31))
    if not (L == 89 and O.irreducible_prime_degree(O.char_poly_from_conn(conn))):
        F = P.transition_matrix(oracle_step(ps), 3, 7)
        assert not np.array_equal(P.matpow2(F, (1 << 89) - 1), np.eye(89, dtype=np.uint8))


# ---------------------------------------------------------------------------
# P5: section 3.2 -- rounds of W <= N - M steps reproduce the sequential
# stream; W = N - M + 1 does not (the bound is tight).
# ---------------------------------------------------------------------------

def test_round_parallel_emulation():
    mexp = 521  # N = 17
    N = 17
    for M in (2, 5, 11, 16):
        base = I.draw_param_set(mexp, I.SplitMix64(M), I.M_POLICY_FULL)
        ps = I.ParamSet(mexp, M, base.sh1, base.sh2, base.param_tbl, base.temper_tbl)
        st = O.seed_state(3, mexp)
        n = 90
        ref = O.generate(ps, st.copy(), n)
        for width in range(1, N - M + 1):
            out, _ = P.round_parallel(ps, list(st), n, width, L=N + width)
            np.testing.assert_array_equal(out, ref)
        out, _ = P.round_parallel(ps, list(st), n, N - M + 1, L=2 * N + 2)
        assert not np.array_equal(out, ref)


# ---------------------------------------------------------------------------
# P6: float outputs, section 6.
# ---------------------------------------------------------------------------

def test_float_closed_forms():
    ps = I.single_stream()[0][0]
    st = O.seed_state(77, ps.mexp)
    n = 50000
    u = O.generate(ps, st.copy(), n, O.U32)
    f12 = O.generate(ps, st.copy(), n, O.F12)
    f01 = O.generate(ps, st.copy(), n, O.F01)
    # fraction = 23 MSBs of the 32-bit output, exponent of 1.0
    np.testing.assert_array_equal(f12, np.uint32(0x3F800000) | (u >> np.uint32(9)))
    v12 = f12.view(np.float32)
    v01 = f01.view(np.float32)
    np.testing.assert_array_equal(v01, v12 - np.float32(1.0))
    assert v12.min() >= 1.0 and v12.max() <= 2.0 - 2.0 ** -23
    assert v01.min() >= 0.0 and v01.max() <= 1.0 - 2.0 ** -23
    # value is (u >> 9) * 2^-23 exactly
    np.testing.assert_array_equal(v01.astype(np.float64), (u >> np.uint32(9)).astype(np.float64) * 2.0 ** -23)
    # +0.0 (not -0.0) when the fraction is zero
    ps0 = I.ParamSet(89, 2, 1, 1, (0,) * 16, (0,) * 16)
    z = O.generate(ps0, np.zeros(3, dtype=np.uint32), 5, O.F01)
    assert (z == 0).all()


# ---------------------------------------------------------------------------
# P7: continuation (section 8: the state is stored back so the next call
# continues the stream).
# ---------------------------------------------------------------------------

def test_continuation_splits():
    ps = I.single_stream()[0][0]
    N = O.nwords(ps.mexp)
    st = O.seed_state(1234, ps.mexp)
    total = 3 * N + 101
    ref = O.generate(ps, st.copy(), total)
    for a in (0, 1, 5, N - 1, N, N + 1, 2 * N + 3, total):
        s = st.copy()
        x = O.generate(ps, s, a)
        y = O.generate(ps, s, total - a)
        np.testing.assert_array_equal(np.concatenate([x, y]), ref)


# ---------------------------------------------------------------------------
# Special cases: zero tables.
# ---------------------------------------------------------------------------

def test_zero_tempering_gives_raw_words():
    ps = I.single_stream()[0][0]
    raw = I.ParamSet(ps.mexp, ps.pos, ps.sh1, ps.sh2, ps.param_tbl, (0,) * 16)
    st = O.seed_state(5, ps.mexp)
    n = 2000
    out = O.generate(raw, st.copy(), n)
    # with no tempering, output k is the new word x_{N+k}: after n steps the
    # last N outputs are the state words
    s = st.copy()
    O.advance(raw, s, n)
    N = O.nwords(ps.mexp)
    np.testing.assert_array_equal(out[n - N:], s)


def test_sh1_zero_cancels_t():
    # t ^= t << 0 gives t = 0: x_{N+i} depends on x_{M+i} alone
    base = I.single_stream()[0][0]
    ps = I.ParamSet(base.mexp, base.pos, 0, base.sh2, base.param_tbl, (0,) * 16)
    N = O.nwords(ps.mexp)
    st = I.random_state(N, 8)
    out = O.generate(ps, st.copy(), 10)
    st2 = st.copy()
    st2[0] ^= 0xDEADBEEF
    st2[1] ^= 0x12345678
    out2 = O.generate(ps, st2, 10)
    np.testing.assert_array_equal(out, out2)


# ---------------------------------------------------------------------------
# Seeding reading (the paper is silent): MT19937's initialisation recurrence,
# as implemented by numpy's legacy MT19937 seeding.
# ---------------------------------------------------------------------------

def test_seeding_matches_mt19937_init():
    for seed in (0, 1, 1234, 5489, 0xFFFFFFFF):
        key = np.random.RandomState(seed).get_state()[1].astype(np.uint32)
        st = np.zeros(624, dtype=np.uint32)
        O.lib().orc_seed(seed, 624, st.ctypes.data)
        np.testing.assert_array_equal(st, key)
    for mexp in I.MEXPS:
        assert O.seed_state(1234, mexp).any()


def test_oracle_rejects_out_of_definition_parameters():
    ps = I.single_stream()[0][0]
    N = O.nwords(ps.mexp)
    st = O.seed_state(1, ps.mexp)
    # tables must be the products (v)R and (v)T of 4 x w matrices (sections
    # 3.6 and 3.7): one flipped bit in an entry that is not a unit vector's
    # product leaves no matrix with that table
    flip = lambda t, v: t[:v] + (t[v] ^ 0x40,) + t[v + 1:]
    for bad in (I.ParamSet(ps.mexp, 1, 1, 1, ps.param_tbl, ps.temper_tbl),
                I.ParamSet(ps.mexp, N, 1, 1, ps.param_tbl, ps.temper_tbl),
                I.ParamSet(ps.mexp, 5, 32, 1, ps.param_tbl, ps.temper_tbl),
                I.ParamSet(ps.mexp, ps.pos, ps.sh1, ps.sh2, flip(ps.param_tbl, 7), ps.temper_tbl),
                I.ParamSet(ps.mexp, ps.pos, ps.sh1, ps.sh2, ps.param_tbl, flip(ps.temper_tbl, 12)),
                I.ParamSet(ps.mexp, ps.pos, ps.sh1, ps.sh2, flip(ps.param_tbl, 0), ps.temper_tbl)):
        with pytest.raises(ValueError):
            O.generate(bad, st.copy(), 4)


def test_inputs_recipe():
    params, n = I.independent_128()
    assert n == 1 << 22 and len(params) == 128 and len({p.key() for p in params}) == 128
    for p in params:
        assert 2 <= p.pos <= 95 and 1 <= p.sh1 <= 31 and 1 <= p.sh2 <= 31
        P.matrix_from_table(p.param_tbl)
        P.matrix_from_table(p.temper_tbl)
    ps, n1 = I.single_stream()
    assert n1 == 1 << 20 and 2 <= ps[0].pos <= 349


# ---------------------------------------------------------------------------
# Box-Muller normals from float [1,2) pairs (section 6 names the use)
# ---------------------------------------------------------------------------

def _f32_bits(values):
    return np.asarray(values, dtype=np.float32).view(np.uint32)


def test_normals_invert_to_their_uniforms():
    """The inverse transform recovers the pair: exp(-(z0^2 + z1^2) / 2) = 2 - a
    and atan2(z1, z0) / 2 pi = b - 1 (mod 1)."""
    ps = I.single_stream()[0][0]
    st = O.seed_state(77, ps.mexp)
    f12 = O.generate(ps, st.copy(), 20000, O.F12)
    z = O.normals(ps, st.copy(), 20000)
    f = f12.view(np.float32).astype(np.float64)
    a, b = f[0::2], f[1::2]
    z0, z1 = z[0::2], z[1::2]
    np.testing.assert_allclose(np.exp(-(z0 * z0 + z1 * z1) / 2.0), 2.0 - a, rtol=1e-12)
    frac = np.mod(np.arctan2(z1, z0) / (2.0 * np.pi), 1.0)
    d = np.abs(frac - (b - 1.0))
    assert np.all(np.minimum(d, 1.0 - d) < 1e-12)


def test_normals_special_values():
    a_max = np.nextafter(np.float32(2.0), np.float32(1.0))        # 2 - 2^-23: u1 = 2^-23
    r_max = np.sqrt(-2.0 * np.log(2.0 ** -23))
    z = O.normals_from_f12(_f32_bits([1.0, 1.7, a_max, 1.0, a_max, 1.25, a_max, 1.5]))
    np.testing.assert_array_equal(z[:2], [0.0, 0.0])               # u1 = 1: radius 0
    np.testing.assert_allclose(z[2:4], [r_max, 0.0], atol=1e-12)   # angle 0
    np.testing.assert_allclose(z[4:6], [0.0, r_max], atol=1e-12)   # angle pi/2
    np.testing.assert_allclose(z[6:8], [-r_max, 0.0], atol=1e-12)  # angle pi


def test_box_muller_binary32_arguments_are_exact():
    """The device evaluates the transform's arguments in binary32: 2 - a,
    b - 1 (sine) and b - 3/4 (cosine, the sine a quarter turn on). For every
    one of the 2^23 float [1,2) values each is exact, and b - 3/4 equals
    (b - 1) + 1/4, so the angle the hardware sine receives carries no
    rounding; the normals' tolerance only has to cover the log, square root
    and sine themselves."""
    x = (np.uint32(0x3F800000) | np.arange(1 << 23, dtype=np.uint32)).view(np.float32)
    x64 = x.astype(np.float64)
    for got, want in ((np.float32(2.0) - x, 2.0 - x64), (x - np.float32(1.0), x64 - 1.0),
                      (x - np.float32(0.75), x64 - 0.75)):
        np.testing.assert_array_equal(got.astype(np.float64), want)
    np.testing.assert_array_equal((x - np.float32(1.0)) + np.float32(0.25), x - np.float32(0.75))


def test_normals_are_standard_normal_and_consume_n_steps():
    from scipy import stats
    params = I.draw_param_sets([11213] * 4, 91)
    zs = []
    for g, ps in enumerate(params):
        st = O.seed_state(500 + g, ps.mexp)
        ref = st.copy()
        zs.append(O.normals(ps, st, 50000))
        O.advance(ps, ref, 50000)
        np.testing.assert_array_equal(st, ref)
    z = np.concatenate(zs)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    assert stats.kstest(z, stats.norm.cdf).pvalue > 1e-3
