"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module holds no MTGP arithmetic: it only draws random numbers and lays
them out as the inputs the generator consumes (parameter sets, seeds, request
lists). Both the oracle and the HIP path receive what it produces; neither
side's recursion, tempering or float conversion lives here.

Parameter sets. The paper's published parameter sets (128 per period, section
3.8) are not available, so seeded synthetic sets stand in for them with the
paper's shapes: the 16-entry recursion and tempering tables are the F2 span of
four random 32-bit rows (the table for a 4x32 matrix, section 3.6 and 3.7),
shifts sh1, sh2 are drawn from [1, 31], and the middle position M follows
either the range [2, N-2] or the paper's thread-count rule N - M >= the
largest power of two not above N - 2 (section 3.5).

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written from its published
definition.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

MASK64 = (1 << 64) - 1

# Mersenne exponents of the three released MTGP periods (section 3.5).
MEXPS = (11213, 23209, 44497)

KIND_U32 = 0     # uint32 output
KIND_F12 = 1     # float32 in [1, 2)
KIND_F01 = 2     # float32 in [0, 1)
KIND_NAMES = {KIND_U32: "uint32", KIND_F12: "float32_1to2", KIND_F01: "float32_0to1"}


class SplitMix64:
    """SplitMix64 stream (64-bit state, golden-gamma increment)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def next_u32(self) -> int:
        return self.next_u64() >> 32

    def uniform_int(self, lo: int, hi: int) -> int:
        """Integer uniform in [lo, hi] (inclusive), by rejection."""
        span = hi - lo + 1
        assert span >= 1
        limit = (1 << 64) - ((1 << 64) % span)
        while True:
            v = self.next_u64()
            if v < limit:
                return lo + v % span

    def uniform01(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def words_for(mexp: int) -> int:
    """Number of 32-bit words that hold mexp bits (used for the M ranges)."""
    return -(-mexp // 32)


def pow2_floor(v: int) -> int:
    """Largest power of two not above v (v >= 1)."""
    return 1 << (v.bit_length() - 1)


def span_table(rows: Sequence[int]) -> List[int]:
    """16-entry table of the F2 span of four 32-bit rows: entry j is the XOR
    of rows[b] over the set bits b of j (bit 0 = least significant)."""
    assert len(rows) == 4
    tbl = []
    for j in range(16):
        v = 0
        for b in range(4):
            if (j >> b) & 1:
                v ^= rows[b]
        tbl.append(v & 0xFFFFFFFF)
    return tbl


@dataclass(frozen=True)
class ParamSet:
    """One MTGP parameter set as the C-ABI takes it."""
    mexp: int
    pos: int
    sh1: int
    sh2: int
    param_tbl: Tuple[int, ...]
    temper_tbl: Tuple[int, ...]

    def key(self):
        return (self.mexp, self.pos, self.sh1, self.sh2, self.param_tbl, self.temper_tbl)


M_POLICY_WIDE = "wide"     # M uniform in [2, N-2]
M_POLICY_PAPER = "paper"   # M uniform in [2, N - pow2_floor(N-2)]
M_POLICY_FULL = "full"     # M uniform in [2, N-1], the whole range the definition allows


def m_range(mexp: int, policy: str) -> Tuple[int, int]:
    n = words_for(mexp)
    if policy == M_POLICY_WIDE:
        return 2, n - 2
    if policy == M_POLICY_PAPER:
        return 2, n - pow2_floor(n - 2)
    if policy == M_POLICY_FULL:
        return 2, n - 1
    raise ValueError(policy)


def draw_param_set(mexp: int, rng: SplitMix64, policy: str = M_POLICY_PAPER) -> ParamSet:
    lo, hi = m_range(mexp, policy)
    pos = rng.uniform_int(lo, hi)
    sh1 = rng.uniform_int(1, 31)
    sh2 = rng.uniform_int(1, 31)
    rrows = [rng.next_u32() for _ in range(4)]
    trows = [rng.next_u32() for _ in range(4)]
    return ParamSet(mexp, pos, sh1, sh2, tuple(span_table(rrows)), tuple(span_table(trows)))


def draw_param_sets(mexps: Sequence[int], seed: int, policy: str = M_POLICY_PAPER) -> List[ParamSet]:
    """Distinct seeded parameter sets, one per entry of mexps (redraw on duplicate)."""
    rng = SplitMix64(seed)
    seen = set()
    out = []
    for mexp in mexps:
        while True:
            ps = draw_param_set(mexp, rng, policy)
            if ps.key() not in seen:
                seen.add(ps.key())
                out.append(ps)
                break
    return out


# ---------------------------------------------------------------------------
# Workloads (seeded). Generator g's state seed is 1234 + g.
# ---------------------------------------------------------------------------

STATE_SEED_BASE = 1234


def state_seeds(count: int) -> List[int]:
    return [STATE_SEED_BASE + g for g in range(count)]


def single_stream() -> Tuple[List[ParamSet], int]:
    """One MTGP-11213, M in [2, N-2], state seed 1234, 2^20 uint32 outputs."""
    return draw_param_sets([11213], 1000, M_POLICY_WIDE), 1 << 20


def independent_128() -> Tuple[List[ParamSet], int]:
    """128 distinct MTGP-11213 sets (paper M rule), 2^22 outputs each."""
    return draw_param_sets([11213] * 128, 2000, M_POLICY_PAPER), 1 << 22


def large_states(mexp: int, count: int = 256) -> Tuple[List[ParamSet], int]:
    """`count` sets at period 2^23209-1 or 2^44497-1, 2^24 uint32 outputs each."""
    assert mexp in (23209, 44497)
    return draw_param_sets([mexp] * count, 3000 + (mexp == 44497), M_POLICY_PAPER), 1 << 24


def large_states_wide_m(mexp: int = 23209, count: int = 256) -> Tuple[List[ParamSet], int]:
    """The large-state batch with M drawn from [2, N-2] (the single-stream
    configuration's rule) instead of the paper's: some generators get N - M of
    a few words, i.e. millions of dependent rounds for 2^24 outputs."""
    assert mexp in (23209, 44497)
    return draw_param_sets([mexp] * count, 3002 + (mexp == 44497), M_POLICY_WIDE), 1 << 24


@dataclass
class Request:
    gen: int
    n: int
    kind: int
    offset: int = 0   # output offset (elements) in a packed output buffer


def batched_uneven(count: int = 4096, seed: int = 4000, log2_lo: int = 10, log2_hi: int = 24):
    """Mixed exponents 2:1:1 (11213:23209:44497), lengths floor(2^(lo + (hi-lo)U)),
    kinds 50% uint32 / 25% float [1,2) / 25% float [0,1)."""
    assert count % 4 == 0
    mexps = [11213] * (count // 2) + [23209] * (count // 4) + [44497] * (count // 4)
    params = draw_param_sets(mexps, seed, M_POLICY_PAPER)
    rng = SplitMix64(seed + 1)
    reqs = []
    off = 0
    for g in range(count):
        n = int(math.floor(2.0 ** (log2_lo + (log2_hi - log2_lo) * rng.uniform01())))
        v = rng.uniform_int(0, 3)
        kind = KIND_U32 if v < 2 else (KIND_F12 if v == 2 else KIND_F01)
        reqs.append(Request(g, n, kind, off))
        off += n
    return params, reqs


def serving_trace(num_requests: int, rate_per_s: float, num_gens: int = 65536, seed: int = 5001,
                  median_log2: int = 16, sigma: float = 1.5, lo_log2: int = 10, hi_log2: int = 26):
    """Poisson arrivals (exponential gaps at rate_per_s), log-normal sizes with
    the given median, clipped to [2^lo, 2^hi]; 50% uint32 and 50% float32
    (split evenly between [1,2) and [0,1)); target generator uniform."""
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    for _ in range(num_requests):
        u = rng.uniform01()
        t += -math.log(1.0 - u) / rate_per_s
        # Box-Muller on two uniforms for the log-normal size
        u1 = 1.0 - rng.uniform01()
        u2 = rng.uniform01()
        z = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
        n = int(round((2.0 ** median_log2) * math.exp(sigma * z)))
        n = max(1 << lo_log2, min(1 << hi_log2, n))
        v = rng.uniform_int(0, 3)
        kind = KIND_U32 if v < 2 else (KIND_F12 if v == 2 else KIND_F01)
        gen = rng.uniform_int(0, num_gens - 1)
        out.append((t, gen, n, kind))
    return out


def serving_trace_arrays(num_requests: int, rate_per_s: float, num_gens: int = 65536, seed: int = 5001,
                         median_log2: int = 16, sigma: float = 1.5, lo_log2: int = 10, hi_log2: int = 26):
    """The serving_trace distributions drawn with numpy (PCG64 seeded by
    `seed`) for long traces: arrays (arrival s, gen, n, kind)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, num_requests))
    n = np.rint((2.0 ** median_log2) * np.exp(sigma * rng.standard_normal(num_requests))).astype(np.int64)
    n = np.clip(n, 1 << lo_log2, 1 << hi_log2)
    v = rng.integers(0, 4, num_requests)
    kind = np.where(v < 2, KIND_U32, np.where(v == 2, KIND_F12, KIND_F01))
    gen = rng.integers(0, num_gens, num_requests)
    return t, gen, n, kind


def serving_params(num_gens: int = 65536) -> List[ParamSet]:
    return draw_param_sets([11213] * num_gens, 5000, M_POLICY_PAPER)


def random_state(nwords: int, seed: int) -> np.ndarray:
    """Random full 32-bit words, for set_state / linearity tests."""
    rng = SplitMix64(seed)
    return np.array([rng.next_u32() for _ in range(nwords)], dtype=np.uint32)


def params_to_arrays(params: Sequence[ParamSet]):
    """Pack parameter sets into flat numpy arrays (for bulk C calls)."""
    g = len(params)
    hdr = np.zeros((g, 4), dtype=np.uint32)
    rec = np.zeros((g, 16), dtype=np.uint32)
    tmp = np.zeros((g, 16), dtype=np.uint32)
    for i, ps in enumerate(params):
        hdr[i] = (ps.mexp, ps.pos, ps.sh1, ps.sh2)
        rec[i] = ps.param_tbl
        tmp[i] = ps.temper_tbl
    return hdr, rec, tmp
