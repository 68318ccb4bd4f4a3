"""Bit-exact parity of the chunked launch form (mode 2) against the oracle.

The chunked form runs one wavefront per generator and keeps three chunks of
64 steps in flight; it serves generators with N - M >= 64 (depth + 2) for a
read-ahead depth of 1 or 2 chunks. These tests cover the edges of that
condition, every ring length, every output kind, lengths around the chunk
and eight-chunk block sizes, multi-wavefront workgroups, split plans and a
single generator's calls. Normals are compared within the tolerance the
other normal tests use; every other kind bit for bit.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1005_4973_amd import inputs as I

pytestmark = pytest.mark.gpu

CHUNK = 2             # launch mode of the chunked form
NORMAL_ATOL = 1.5e-5  # same bound as the other normal tests (Box-Muller reading N1)
LENGTHS = (1, 2, 63, 64, 65, 127, 511, 512, 513, 4097, 100003)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1005_4973_amd import mtgp
    mtgp.lib()
    return mtgp


def host_bits(t):
    import torch
    return t.view(torch.int32).cpu().numpy().view(np.uint32)


def host_f32(t):
    import torch
    return t.view(torch.float32).cpu().numpy().astype(np.float64)


def with_gap(mexp, gap, seed):
    """A seeded parameter set of exponent mexp with N - M = gap."""
    base = I.draw_param_set(mexp, I.SplitMix64(seed), I.M_POLICY_FULL)
    N = O.nwords(mexp)
    return I.ParamSet(mexp, N - gap, base.sh1, base.sh2, base.param_tbl, base.temper_tbl)


def check(M, b, params, states, reqs):
    import torch
    bufs = [torch.empty(max(n, 1), dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    b.generate([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    torch.cuda.synchronize()
    for (g, k, n), buf in zip(reqs, bufs):
        if k == 3:
            ref = O.normals(params[g], states[g], n)
            err = np.abs(host_f32(buf)[:n] - ref).max()
            assert err <= NORMAL_ATOL, f"gen={g} n={n} normal err={err}"
        else:
            ref = O.generate(params[g], states[g], n, k)
            np.testing.assert_array_equal(host_bits(buf)[:n], ref, err_msg=f"gen={g} kind={k} n={n}")


def test_chunk_edges_depths_kinds_lengths(M):
    """N - M at the edges of both read-ahead depths (192, 193, 255, 256,
    257) and far inside them, the three released state sizes and the
    largest accepted one (p = 65536, N = 2048, no mask), every kind, and
    lengths around 64 and 512 as consecutive calls."""
    params = [with_gap(11213, 192, 1), with_gap(11213, 193, 2), with_gap(11213, 255, 3), with_gap(11213, 256, 4),
              with_gap(11213, 257, 5), with_gap(11213, 349, 6), with_gap(23209, 512, 7), with_gap(23209, 724, 8),
              with_gap(44497, 1024, 9), with_gap(44497, 1389, 10), with_gap(65536, 1900, 11)]
    seeds = I.state_seeds(len(params))
    for depth in (1, 2):
        ok = [g for g, ps in enumerate(params) if ps.pos <= O.nwords(ps.mexp) - 64 * (depth + 2)]
        for threads in (64, 256, 1024):
            # 16 wavefronts of 2L + 32 words each fit the CU's LDS only for rings up to 1024
            use = [g for g in ok if threads < 1024 or O.nwords(params[g].mexp) <= 960]
            say(f"depth {depth} threads {threads} generators {use}")
            sub = [params[g] for g in use]
            b = M.Batch(sub, [seeds[g] for g in use])
            b.set_launch(CHUNK, threads, depth, 0, 0)
            states = {g: O.seed_state(seeds[use[g]], sub[g].mexp) for g in range(len(sub))}
            for i, n in enumerate(LENGTHS):
                kinds = [(g + i) % 4 for g in range(len(sub))]
                check(M, b, sub, states, [(g, kinds[g], n + (n & 1 if kinds[g] == 3 else 0))
                                          for g in range(len(sub))])
            for g in range(len(sub)):
                words, _ = b.get_state(g)
                np.testing.assert_array_equal(words, states[g], err_msg=f"depth={depth} threads={threads} gen={g}")
            b.close()


def test_chunk_ring_lengths(M):
    """Every ring length the kernel is built for (explicit lds_words), for a
    state that needs the smallest one: the ring wraps many times per call."""
    params = [with_gap(11213, 300, 21), with_gap(11213, 256, 22)]
    seeds = I.state_seeds(len(params))
    for L in (512, 1024, 2048, 4096):
        say(f"ring {L}")
        b = M.Batch(params, seeds)
        b.set_launch(CHUNK, 128, 2, L, 0)
        states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
        for n, k in ((70001, 0), (33333, 1), (4096, 2), (100002, 3)):
            check(M, b, params, states, [(g, k, n) for g in range(len(params))])
        b.close()


def test_chunk_rejects_what_it_cannot_run(M):
    """A generator with N - M below the depth's bound, a ring too short for N,
    and an unsupported depth or ring length are refused (MTGP_EINVAL)."""
    import torch
    params = [with_gap(11213, 191, 31), with_gap(11213, 255, 32), with_gap(44497, 1100, 33)]
    b = M.Batch(params, I.state_seeds(3))
    buf = torch.empty(1000, dtype=torch.int32, device="cuda")
    b.set_launch(CHUNK, 256, 1, 0, 0)
    with pytest.raises(M.MTGPError):
        b.generate([(0, 0, 1000, buf)])                 # N - M = 191 < 192
    b.generate([(1, 0, 1000, buf)])                     # 255 >= 192: runs
    b.set_launch(CHUNK, 256, 2, 0, 0)
    with pytest.raises(M.MTGPError):
        b.generate([(1, 0, 1000, buf)])                 # 255 < 256 at depth 2
    b.set_launch(CHUNK, 256, 2, 1024, 0)
    with pytest.raises(M.MTGPError):
        b.generate([(2, 0, 1000, buf)])                 # N = 1391 needs a ring of 2048
    for bad in ((CHUNK, 256, 3, 0, 0), (CHUNK, 256, 2, 768, 0), (CHUNK, 256, 2, 8192, 0)):
        with pytest.raises(M.MTGPError):
            b.set_launch(*bad)
    b.close()


def test_chunk_split_plan_replays(M):
    """A graph-captured split plan in the chunked form: jump-ahead segments
    of every kind, replayed three times, against the unsplit stream."""
    import torch
    params = I.draw_param_sets([11213] * 3 + [23209, 44497], 41)
    seeds = I.state_seeds(len(params))
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    b = M.Batch(params, seeds)
    b.set_launch(CHUNK, 256, 2, 0, 0)
    b.set_split(300)                                    # chunks per segment
    reqs = [(0, 0, 100003), (1, 1, 77777), (2, 3, 120000), (3, 2, 64000), (4, 0, 90001)]
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    plan = b.plan([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    for rep in range(3):
        say(f"split plan replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        for (g, k, n), buf in zip(reqs, bufs):
            if k == 3:
                err = np.abs(host_f32(buf) - O.normals(params[g], states[g], n)).max()
                assert err <= NORMAL_ATOL, f"rep={rep} gen={g} err={err}"
            else:
                np.testing.assert_array_equal(host_bits(buf), O.generate(params[g], states[g], n, k),
                                              err_msg=f"rep={rep} gen={g}")
    plan.close()
    for g in range(len(params)):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g])
    b.close()


def test_chunk_single_generator(M):
    """A single generator's calls in the chunked form (one wavefront), both
    depths, continuing across kinds."""
    ps = with_gap(23209, 600, 51)
    st = O.seed_state(5, ps.mexp)
    g = M.Generator(ps, 5)
    for depth in (1, 2):
        g.set_launch(CHUNK, 64, depth, 0)
        for n, k in ((1, 0), (65, 1), (100001, 2), (2 * 5003, 3), (512, 0)):
            out = g.generate(n, k)
            if k == 3:
                assert np.abs(host_f32(out) - O.normals(ps, st, n)).max() <= NORMAL_ATOL
            else:
                np.testing.assert_array_equal(host_bits(out), O.generate(ps, st, n, k), err_msg=f"n={n} k={k}")
    words, _ = g.get_state()
    np.testing.assert_array_equal(words, st)
    g.close()
