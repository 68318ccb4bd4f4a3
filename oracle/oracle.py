"""ctypes wrapper around the C oracle (mtgp_oracle.c, f2.c) -- test infrastructure only.

Builds liborc.so with gcc (no fast-math, no FP contraction) on first use or
via build(). See mtgp_oracle.c for the definitions followed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from types import SimpleNamespace
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SOURCES = [os.path.join(HERE, "mtgp_oracle.c"), os.path.join(HERE, "f2.c")]

U32 = 0
F12 = 1
F01 = 2


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp] + SOURCES
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrcParams(ctypes.Structure):
    _fields_ = [("mexp", ctypes.c_uint32), ("pos", ctypes.c_uint32),
                ("sh1", ctypes.c_uint32), ("sh2", ctypes.c_uint32),
                ("param_tbl", ctypes.c_uint32 * 16), ("temper_tbl", ctypes.c_uint32 * 16)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_nwords.argtypes = [ctypes.c_uint32]
        L.orc_nwords.restype = ctypes.c_uint32
        L.orc_seed.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        L.orc_seed.restype = None
        L.orc_generate.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.c_int, ctypes.c_void_p]
        L.orc_generate.restype = ctypes.c_int
        L.orc_advance.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_void_p, ctypes.c_uint64]
        L.orc_advance.restype = ctypes.c_int
        L.orc_output_bits.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_int, ctypes.c_void_p]
        L.orc_output_bits.restype = ctypes.c_int
        L.orc_bm.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.orc_bm.restype = ctypes.c_int64
        L.orc_irreducible_prime_degree.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_irreducible_prime_degree.restype = ctypes.c_int
        _lib = L
    return _lib


def to_c(ps) -> OrcParams:
    p = OrcParams()
    p.mexp, p.pos, p.sh1, p.sh2 = ps.mexp, ps.pos, ps.sh1, ps.sh2
    for i in range(16):
        p.param_tbl[i] = ps.param_tbl[i]
        p.temper_tbl[i] = ps.temper_tbl[i]
    return p


def nwords(mexp: int) -> int:
    return int(lib().orc_nwords(mexp))


def seed_state(seed: int, mexp: int) -> np.ndarray:
    n = nwords(mexp)
    st = np.zeros(n, dtype=np.uint32)
    lib().orc_seed(seed & 0xFFFFFFFF, n, st.ctypes.data)
    return st


def generate(ps, state: np.ndarray, n: int, kind: int = U32) -> np.ndarray:
    """Generate n outputs; `state` (uint32[N], sequence order) is advanced in place."""
    assert state.dtype == np.uint32 and state.flags.c_contiguous
    out = np.zeros(max(n, 1), dtype=np.uint32)
    rc = lib().orc_generate(ctypes.byref(to_c(ps)), state.ctypes.data, n, kind, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected parameters (rc={rc})")
    return out[:n]


def normals_from_f12(f12_bits: np.ndarray) -> np.ndarray:
    """Gaussian deviates by the Box-Muller transform, in float64, of
    consecutive pairs of float [1,2) outputs given as bit patterns.

    Section 6 of the paper notes that the [1,2) outputs serve the Box-Muller
    transformation directly. Reading taken: for the pair (a, b) at positions
    2j, 2j+1, u1 = 2 - a lies in (0, 1] and u2 = b - 1 in [0, 1);
    r = sqrt(-2 ln u1), theta = 2 pi u2; output 2j = r cos(theta),
    output 2j+1 = r sin(theta). The pair count must be whole.
    """
    f = np.asarray(f12_bits, dtype=np.uint32).view(np.float32).astype(np.float64)
    assert f.size % 2 == 0, "normals come in pairs"
    a, b = f[0::2], f[1::2]
    r = np.sqrt(-2.0 * np.log(2.0 - a))
    theta = 2.0 * np.pi * (b - 1.0)
    out = np.empty(f.size, dtype=np.float64)
    out[0::2] = r * np.cos(theta)
    out[1::2] = r * np.sin(theta)
    return out


def normals(ps, state: np.ndarray, n: int) -> np.ndarray:
    """n Gaussian deviates (n even) from the float [1,2) stream; `state` is
    advanced by n steps, as for the other kinds."""
    return normals_from_f12(generate(ps, state, n, F12))


def advance(ps, state: np.ndarray, n: int) -> None:
    rc = lib().orc_advance(ctypes.byref(to_c(ps)), state.ctypes.data, n)
    if rc != 0:
        raise ValueError(f"oracle rejected parameters (rc={rc})")


def stream(ps, seed: int, n: int, kind: int = U32):
    """(outputs, final state) of a fresh generator seeded with `seed`."""
    st = seed_state(seed, ps.mexp)
    out = generate(ps, st, n, kind)
    return out, st


def output_bits(ps, state: np.ndarray, n: int, bit: int) -> np.ndarray:
    bits = np.zeros(n, dtype=np.uint8)
    rc = lib().orc_output_bits(ctypes.byref(to_c(ps)), state.ctypes.data, n, bit, bits.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle rejected parameters (rc={rc})")
    return bits


def berlekamp_massey(bits: Sequence[int]):
    """(L, connection polynomial as uint8 array c[0..L])."""
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
    conn = np.zeros(len(b) + 2, dtype=np.uint8)
    L = lib().orc_bm(b.ctypes.data, len(b), conn.ctypes.data)
    if L < 0:
        raise MemoryError
    return int(L), conn[: L + 1].copy()


def char_poly_from_conn(conn: np.ndarray) -> np.ndarray:
    """Reciprocal of the connection polynomial: phi(x) = x^L C(1/x), as coeffs phi[0..L]."""
    return conn[::-1].copy()


def irreducible_prime_degree(phi: np.ndarray) -> bool:
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.uint8))
    rc = lib().orc_irreducible_prime_degree(phi.ctypes.data, len(phi) - 1)
    if rc < 0:
        raise ValueError("bad polynomial")
    return rc == 1


# ---------------------------------------------------------------------------
# Dimension of equidistribution by its definition (section 3.4), for small p.
#
# For a generator of period 2^p - 1 (every nonzero state on one orbit), the
# v MSBs of k consecutive outputs are k-dimensionally equidistributed exactly
# when the map from the p-bit state to those k*v bits is onto, i.e. when the
# k*v output-bit functionals are linearly independent over F2. The functional
# of bit b of output i is read off the outputs of the p unit states.
# Pure Python Gaussian elimination: for p up to a few hundred.
# ---------------------------------------------------------------------------


def state_bit_positions(mexp: int):
    """(word, bit) of the p state bits: the 32 - r high bits of x_0 (the only
    ones the recursion reads, through the mask) and every bit of x_1 .. x_{N-1}."""
    N = nwords(mexp)
    r = 32 * N - mexp
    return [(0, b) for b in range(r, 32)] + [(w, b) for w in range(1, N) for b in range(32)]


def unit_state_outputs(ps, n: int, tempered: bool = True) -> np.ndarray:
    """cols[s, i] = uint32 output i from the s-th unit state. Untempered
    outputs are the raw words x_{i+N}: the same recursion with a zero
    tempering table."""
    if not tempered:
        ps = SimpleNamespace(mexp=ps.mexp, pos=ps.pos, sh1=ps.sh1, sh2=ps.sh2,
                             param_tbl=tuple(ps.param_tbl), temper_tbl=(0,) * 16)
    pos = state_bit_positions(ps.mexp)
    cols = np.zeros((len(pos), n), dtype=np.uint32)
    for s, (w, b) in enumerate(pos):
        st = np.zeros(nwords(ps.mexp), dtype=np.uint32)
        st[w] = np.uint32(1 << b)
        cols[s] = generate(ps, st, n, U32)
    return cols


def equidistribution_by_rank(cols: np.ndarray, width: int, vmax: int):
    """k(v) for v = 1 .. vmax of a full-period F2-linear generator whose
    `width`-bit outputs from the p unit states are cols[s, i]: the largest k
    such that the bit functionals of the v MSBs of outputs 0 .. k-1 are
    independent (k is capped at the number of outputs given; give p + 1)."""
    p, kmax = cols.shape
    weights = [1 << s for s in range(p)]

    def functional(i, j):   # bit width-1-j of output i, as a p-bit integer over the unit states
        bits = (cols[:, i] >> np.uint32(width - 1 - j)) & np.uint32(1)
        return sum(w for w, x in zip(weights, bits.tolist()) if x)

    rows = {}
    ks = []
    for v in range(1, vmax + 1):
        pivots = {}
        k = kmax
        for i in range(kmax):
            dependent = False
            for j in range(v):
                if (i, j) not in rows:
                    rows[(i, j)] = functional(i, j)
                x = rows[(i, j)]
                while x:
                    top = x.bit_length() - 1
                    if top in pivots:
                        x ^= pivots[top]
                    else:
                        pivots[top] = x
                        break
                if x == 0:
                    dependent = True
                    break
            if dependent:
                k = i
                break
        ks.append(k)
    return ks
