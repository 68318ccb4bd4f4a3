"""Write fullperiod_sets.json: seeded MTGP parameter sets of maximal period
2^p - 1 for small Mersenne exponents p, found with the oracle only.

Search (section 5, recursion-parameter search, restated): draw M, sh1, sh2
and the 4x32 recursion matrix R at random, keep R only if I + R44 is
invertible over F2 (R44: the 4x4 block of the rows' four LSBs; a necessary
condition for the last line of the recursion to be invertible), then compute
the minimal polynomial of one output bit sequence with Berlekamp-Massey; a
degree-p polynomial that is irreducible is primitive because 2^p - 1 is prime,
so the generator has period 2^p - 1. Tempering tables are random (tempering
does not change the period).

Run from the repository root:  python tests/golden/make_fullperiod_sets.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1005_4973_amd import inputs as I  # noqa: E402

EXPONENTS = (89, 107, 127, 521, 607, 1279, 2203)


def det_gf2_4x4(rows):
    m = [r & 0xF for r in rows]
    rank = 0
    for bit in range(3, -1, -1):
        piv = next((i for i in range(rank, 4) if (m[i] >> bit) & 1), None)
        if piv is None:
            continue
        m[rank], m[piv] = m[piv], m[rank]
        for i in range(4):
            if i != rank and (m[i] >> bit) & 1:
                m[i] ^= m[rank]
        rank += 1
    return rank == 4


def search(p, seed):
    rng = I.SplitMix64(seed)
    tries = 0
    while True:
        tries += 1
        ps = I.draw_param_set(p, rng, I.M_POLICY_FULL)
        # rows of R as 32-bit words: entries 1, 2, 4, 8 of the span table
        rows = [ps.param_tbl[1 << b] for b in range(4)]
        # I + R44: add the unit nibble of each row's own bit position
        if not det_gf2_4x4([rows[b] ^ (1 << b) for b in range(4)]):
            continue
        st = O.seed_state(seed, p)
        bits = O.output_bits(ps, st, 2 * p + 64, 31)
        L, conn = O.berlekamp_massey(bits)
        if L != p:
            continue
        if O.irreducible_prime_degree(O.char_poly_from_conn(conn)):
            return ps, tries


def main():
    sets = []
    for p in EXPONENTS:
        ps, tries = search(p, 9000 + p)
        print(f"p={p}: found after {tries} draws (M={ps.pos}, sh1={ps.sh1}, sh2={ps.sh2})", flush=True)
        sets.append({"mexp": ps.mexp, "pos": ps.pos, "sh1": ps.sh1, "sh2": ps.sh2,
                     "param_tbl": list(ps.param_tbl), "temper_tbl": list(ps.temper_tbl),
                     "search_seed": 9000 + p, "draws": tries})
    doc = {"description": "MTGP parameter sets of period 2^p-1 (p a Mersenne exponent), found by "
                          "make_fullperiod_sets.py with the oracle's Berlekamp-Massey and "
                          "irreducibility test (paper section 5 procedure).",
           "sets": sets}
    with open(os.path.join(HERE, "fullperiod_sets.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
