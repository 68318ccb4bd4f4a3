"""The library's recursion-parameter search (section 5, MTGPDC), checked
with the oracle: a set it accepts must have a degree-p, irreducible
characteristic polynomial by the oracle's own Berlekamp-Massey and
irreducibility test, on several tempered output bits, and carry the ID.
The search runs on the host only, so these tests need no GPU.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1005_4973_amd import inputs as I


@pytest.fixture(scope="module")
def M():
    from paper_1005_4973_amd import mtgp
    try:
        mtgp.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip(f"library not built: {e}")
    return mtgp


def oracle_full_period(ps, bits=(31, 0, 13)):
    """Degree-p minimal polynomial, the same on every probed output bit, and
    irreducible (the oracle's test)."""
    p = ps.mexp
    st = O.seed_state(99, p)
    polys = set()
    for b in bits:
        L, conn = O.berlekamp_massey(O.output_bits(ps, st.copy(), 2 * p + 64, b))
        if L != p:
            return False
        polys.add(conn.tobytes())
    return len(polys) == 1 and O.irreducible_prime_degree(O.char_poly_from_conn(conn))


def as_input(ps):
    return I.ParamSet(ps.mexp, ps.pos, ps.sh1, ps.sh2, tuple(ps.param_tbl), tuple(ps.temper_tbl))


def check_structure(ps, ident):
    N = O.nwords(ps.mexp)
    assert ps.sh1 == 13 and ps.sh2 == 4
    fl = 1 << (N.bit_length() - 1)
    lo, hi = (3, N - fl - 1) if N - fl > 4 else (2, N - 1)
    assert lo <= ps.pos <= hi
    t = ps.param_tbl
    # F2-linear, first row = entry of nibble 1000
    for a in range(16):
        for b in range(16):
            assert t[a ^ b] == t[a] ^ t[b]
    assert t[8] >> 16 == ident >> 16                       # 16 MSBs of the ID
    assert (t[4] >> 4) & 0xFFFF == ident & 0xFFFF          # 16 LSBs, bits 19..4 of the second row
    # I + R44 invertible: u -> u ^ (tbl[u] & 0xf) permutes the nibbles
    assert sorted((j ^ t[j]) & 0xF for j in range(16)) == list(range(16))


@pytest.mark.parametrize("p", [521, 607, 1279, 2203])
def test_search_finds_full_period_sets(M, p):
    ident = 0xA5C3_0000 + p
    ps, stats = M.search_params(p, id=ident, seed=p)
    check_structure(ps, ident)
    assert oracle_full_period(as_input(ps))
    assert stats["draws"] >= 1 and stats["full_degree"] >= 1


def test_search_result_is_independent_of_thread_count(M):
    a, sa = M.search_params(607, id=7, seed=3, threads=1)
    b, sb = M.search_params(607, id=7, seed=3, threads=8)
    assert a == b and sa["draws"] == sb["draws"]


def test_distinct_ids_give_distinct_polynomials(M):
    polys = []
    for ident in (1, 2, 3):
        ps, _ = M.search_params(521, id=ident, seed=5)
        L, conn = O.berlekamp_massey(O.output_bits(as_input(ps), O.seed_state(1, 521), 2 * 521 + 64, 31))
        assert L == 521
        polys.append(conn.tobytes())
    assert len(set(polys)) == 3


def test_search_argument_errors(M):
    for bad in ((1000, 1), (64, 1), (521, 0)):          # not prime, too small, no draws
        with pytest.raises(M.MTGPError):
            M.search_params(bad[0], max_draws=bad[1])
    with pytest.raises(M.MTGPError) as e:
        M.search_params(11213, id=1, seed=1, max_draws=1, threads=1)   # one draw is not enough here
    assert e.value.code == -4


@pytest.mark.slow
def test_search_production_size_11213(M):
    """A full-period MTGP-11213 set with an ID embedded (the paper's MTGPDC took
    338 s on average per set); the oracle's irreducibility test alone takes
    about a minute at this degree."""
    ps, stats = M.search_params(11213, id=1, seed=11213)
    check_structure(ps, 1)
    assert oracle_full_period(as_input(ps), bits=(31, 0))
