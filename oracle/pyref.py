"""MTGP in the paper's matrix notation -- test infrastructure only, toy sizes.

A second, independent reading of the generator: words are row vectors in
F2^32 with the MSB as the left-most component (section 3.3, Notation), the
recursion is Definition "recursion parameters" in its vector form (section
3.6, equation algolrec), and tempering is Definition "tempering parameter"
(section 3.7, equation algoltmp):

    t <- x_{1+i} + (x_i^{w-r} | 0^r)
    t <- t + (t << sh1)
    u <- t + (x_{M+i} >> sh2)
    x_{N+i} <- u + (u^4) R              (u^4: the four LSBs of u, a row vector)

    t <- x_{M-1+i} + (x_{M-1+i} >> 16)
    t <- t + (t >> 8)
    o_{N+i} <- x_{N+i} + (t^4) T

Nothing here uses the 16-entry lookup tables as tables: the 4x32 matrices R
and T are recovered from them (row a of R is the image of the unit vector
with a one in component a, i.e. (1000)R, (0100)R, (0010)R, (0001)R) and every
product is an explicit vector-matrix product mod 2. The float outputs of
section 6 are formed as exact rationals (1 + sum of fraction bits 2^-k) and
encoded to IEEE-754 binary32 by Python's own float conversion.

Pure-Python/numpy loops: use only for small N and short streams.
"""
from __future__ import annotations

import struct
from fractions import Fraction
from typing import List, Sequence

import numpy as np

W = 32


def word_to_vec(x: int) -> np.ndarray:
    """32-bit integer -> row vector in F2^32, component 0 = MSB."""
    return np.array([(x >> (W - 1 - k)) & 1 for k in range(W)], dtype=np.uint8)


def vec_to_word(v: np.ndarray) -> int:
    x = 0
    for k in range(W):
        x = (x << 1) | int(v[k] & 1)
    return x


def shl(v: np.ndarray, s: int) -> np.ndarray:
    """Logical left shift: components move towards the MSB (index 0)."""
    out = np.zeros(W, dtype=np.uint8)
    if s < W:
        out[: W - s] = v[s:]
    return out


def shr(v: np.ndarray, s: int) -> np.ndarray:
    """Logical right shift: components move towards the LSB (index W-1)."""
    out = np.zeros(W, dtype=np.uint8)
    if s < W:
        out[s:] = v[: W - s]
    return out


def upper(v: np.ndarray, r: int) -> np.ndarray:
    """(x^{w-r} | 0^r): keep the w-r MSBs, zero the r LSBs."""
    out = v.copy()
    if r:
        out[W - r:] = 0
    return out


def low4(v: np.ndarray) -> np.ndarray:
    """The four LSBs as a row vector in F2^4 (most significant first)."""
    return v[W - 4:].copy()


def matrix_from_table(tbl: Sequence[int]) -> np.ndarray:
    """4x32 matrix whose products with the 16 nibble row vectors are the
    table entries; raises if the table is not such a product table."""
    rows = np.zeros((4, W), dtype=np.uint8)
    for a in range(4):
        unit = 1 << (3 - a)          # row vector with a one in component a
        rows[a] = word_to_vec(tbl[unit])
    for v in range(16):
        nib = np.array([(v >> (3 - a)) & 1 for a in range(4)], dtype=np.uint8)
        if vec_to_word((nib @ rows) % 2) != tbl[v]:
            raise ValueError("table is not F2-linear in the nibble")
    return rows


class MatrixMTGP:
    def __init__(self, ps):
        self.p = ps.mexp
        self.N = -(-ps.mexp // W)
        self.r = W * self.N - ps.mexp
        self.M = ps.pos
        self.sh1 = ps.sh1
        self.sh2 = ps.sh2
        self.R = matrix_from_table(ps.param_tbl)
        self.T = matrix_from_table(ps.temper_tbl)
        assert 2 <= self.M <= self.N - 1

    def next_word(self, x_i, x_i1, x_iM):
        t = (x_i1 + upper(x_i, self.r)) % 2
        t = (t + shl(t, self.sh1)) % 2
        u = (t + shr(x_iM, self.sh2)) % 2
        return (u + (low4(u) @ self.R)) % 2

    def temper(self, x_new, x_tmp):
        t = (x_tmp + shr(x_tmp, 16)) % 2
        t = (t + shr(t, 8)) % 2
        return (x_new + (low4(t) @ self.T)) % 2

    def run(self, state_words: Sequence[int], n: int):
        """Return (list of tempered output vectors, final state words)."""
        xs = [word_to_vec(w) for w in state_words]
        outs = []
        for i in range(n):
            x_new = self.next_word(xs[i], xs[i + 1], xs[i + self.M])
            xs.append(x_new)
            outs.append(self.temper(x_new, xs[i + self.M - 1]))
        final = [vec_to_word(v) for v in xs[n: n + self.N]]
        return outs, final


def f12_bits_from_vec(o: np.ndarray) -> int:
    """Section 6: float in [1,2) whose fraction is the 23 MSBs of the output."""
    val = Fraction(1)
    for k in range(1, 24):
        if o[k - 1]:
            val += Fraction(1, 1 << k)
    return struct.unpack("<I", struct.pack("<f", float(val)))[0]


def f01_bits_from_vec(o: np.ndarray) -> int:
    """Section 6: the [1,2) value minus 1, exactly."""
    val = Fraction(0)
    for k in range(1, 24):
        if o[k - 1]:
            val += Fraction(1, 1 << k)
    return struct.unpack("<I", struct.pack("<f", float(val)))[0]


def generate(ps, state_words: Sequence[int], n: int, kind: int = 0):
    """(outputs as uint32 words / float bit patterns, final state words)."""
    g = MatrixMTGP(ps)
    outs, final = g.run(state_words, n)
    if kind == 0:
        vals = [vec_to_word(o) for o in outs]
    elif kind == 1:
        vals = [f12_bits_from_vec(o) for o in outs]
    elif kind == 2:
        vals = [f01_bits_from_vec(o) for o in outs]
    else:
        raise ValueError(kind)
    return np.array(vals, dtype=np.uint32), np.array(final, dtype=np.uint32)


# ---------------------------------------------------------------------------
# Transition matrix on the p-bit state (section 3.3): the state after step i
# is (x_{i+1}^{w-r} | full x_{i+2} .. x_{i+N}); as a vector we list the w-r
# MSBs of the oldest word first, then the remaining N-1 words MSB-first.
# ---------------------------------------------------------------------------

def state_to_pvec(words: Sequence[int], r: int) -> np.ndarray:
    v = [word_to_vec(w) for w in words]
    head = v[0][: W - r]
    return np.concatenate([head] + v[1:]).astype(np.uint8)


def pvec_to_state(vec: np.ndarray, N: int, r: int) -> List[int]:
    head = np.zeros(W, dtype=np.uint8)
    head[: W - r] = vec[: W - r]
    words = [vec_to_word(head)]
    off = W - r
    for _ in range(N - 1):
        words.append(vec_to_word(vec[off: off + W]))
        off += W
    return words


def transition_matrix(step_fn, N: int, r: int) -> np.ndarray:
    """p x p matrix F with next = s F (row vectors), from stepping each unit
    state through `step_fn(words) -> next words`."""
    p = W * N - r
    F = np.zeros((p, p), dtype=np.uint8)
    for b in range(p):
        e = np.zeros(p, dtype=np.uint8)
        e[b] = 1
        nxt = step_fn(pvec_to_state(e, N, r))
        F[b] = state_to_pvec(nxt, r)
    return F


def matmul2(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return ((a.astype(np.int64) @ b.astype(np.int64)) % 2).astype(np.uint8)


def matpow2(F: np.ndarray, e: int) -> np.ndarray:
    result = np.eye(F.shape[0], dtype=np.uint8)
    base = F.copy()
    while e:
        if e & 1:
            result = matmul2(result, base)
        base = matmul2(base, base)
        e >>= 1
    return result


# ---------------------------------------------------------------------------
# Section 3.2: a ring X[0..L-1] and rounds of W steps whose reads all happen
# before any of the round's writes. The paper's claim is that this reproduces
# the sequential stream whenever W <= N - M (and L is large enough).
# ---------------------------------------------------------------------------

def round_parallel(ps, state_words: Sequence[int], n: int, width: int, L: int):
    g = MatrixMTGP(ps)
    N, M = g.N, g.M
    X = [np.zeros(W, dtype=np.uint8) for _ in range(L)]
    for k, w in enumerate(state_words):
        X[k % L] = word_to_vec(w)
    outs = []
    i0 = 0
    while i0 < n:
        steps = range(i0, min(i0 + width, n))
        # all reads of the round
        reads = [(X[i % L], X[(i + 1) % L], X[(i + M) % L], X[(i + M - 1) % L]) for i in steps]
        # then all writes
        for i, (xi, xi1, xim, xtmp) in zip(steps, reads):
            x_new = g.next_word(xi, xi1, xim)
            X[(i + N) % L] = x_new
            outs.append(vec_to_word(g.temper(x_new, xtmp)))
        i0 += width
    final = [vec_to_word(X[(n + k) % L]) for k in range(N)]
    return np.array(outs, dtype=np.uint32), np.array(final, dtype=np.uint32)
