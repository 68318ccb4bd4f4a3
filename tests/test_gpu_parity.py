"""Bit-exact parity of the HIP path (through the C ABI) against the oracle.

Every output kind is compared bit for bit; integer-valued work has no
tolerance. Inputs are the seeded synthetic parameter sets of
paper_1005_4973_amd.inputs.
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O
from paper_1005_4973_amd import inputs as I

pytestmark = pytest.mark.gpu

KINDS = (I.KIND_U32, I.KIND_F12, I.KIND_F01)


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


def oracle_out(ps, seed, n, kind):
    out, st = O.stream(ps, seed, n, kind)
    return out, st


def pool():
    return ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4))


# ---------------------------------------------------------------------------

def test_single_stream_all_kinds(M):
    (ps,), n = I.single_stream()
    say(f"single_stream M={ps.pos} n={n}")
    for kind in KINDS:
        g = M.Generator(ps, 1234)
        out = g.generate(n, kind)
        words, consumed = g.get_state()
        ref, st = oracle_out(ps, 1234, n, kind)
        np.testing.assert_array_equal(host_bits(out), ref)
        np.testing.assert_array_equal(words, st)
        assert consumed == n
        g.close()


@pytest.mark.parametrize("mexp", [65, 89, 107, 521, 2203, 11213, 23209, 44497, 65536])
def test_m_sweep_and_ragged_lengths(M, mexp):
    """Every M class at the edges of its range (2, 3, N/2, N-3 .. N-1) and
    lengths around N, W and their multiples, for the three released state
    sizes, small ones, and the extremes of the accepted range (p = 65: N = 3,
    r = 31; p = 65536: N = 2048, r = 0, no mask)."""
    N = O.nwords(mexp)
    Ms = sorted({2, 3, N // 2, N - 3, N - 2, N - 1} & set(range(2, N)))
    base = I.draw_param_set(mexp, I.SplitMix64(mexp + 1), I.M_POLICY_FULL)
    for m in Ms:
        ps = I.ParamSet(mexp, m, base.sh1, base.sh2, base.param_tbl, base.temper_tbl)
        W = N - m
        lengths = sorted({1, 2, N - 1, N, N + 1, W - 1 if W > 1 else 1, W, W + 1, 2 * W + 3,
                          3 * N + 7, 5000})
        say(f"mexp={mexp} M={m} lengths={lengths}")
        for kind in KINDS:
            g = M.Generator(ps, 77)
            st = O.seed_state(77, mexp)
            for n in lengths:
                out = g.generate(n, kind)
                ref = O.generate(ps, st, n, kind)
                np.testing.assert_array_equal(host_bits(out), ref, err_msg=f"M={m} n={n} kind={kind}")
            words, _ = g.get_state()
            np.testing.assert_array_equal(words, st)
            g.close()


def test_continuation_mixed_kinds(M):
    (ps,), _ = I.single_stream()
    g = M.Generator(ps, 5)
    st = O.seed_state(5, ps.mexp)
    rng = I.SplitMix64(11)
    for i in range(30):
        n = rng.uniform_int(0, 3000)
        kind = KINDS[i % 3]
        out = g.generate(n, kind) if n > 0 else None
        ref = O.generate(ps, st, n, kind)
        if n > 0:
            np.testing.assert_array_equal(host_bits(out), ref)
    words, consumed = g.get_state()
    np.testing.assert_array_equal(words, st)


def test_set_state_and_linearity(M):
    (ps,), _ = I.single_stream()
    N = O.nwords(ps.mexp)
    s1 = I.random_state(N, 1)
    s2 = I.random_state(N, 2)
    outs = []
    for s in (s1, s2, s1 ^ s2):
        g = M.Generator(ps, 0)
        g.set_state(s, 0)
        outs.append(host_bits(g.generate(4 * N + 5)))
        ref = O.generate(ps, s.copy(), 4 * N + 5)
        np.testing.assert_array_equal(outs[-1], ref)
        g.close()
    np.testing.assert_array_equal(outs[2], outs[0] ^ outs[1])


def test_fullperiod_sets(M):
    import json
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fullperiod_sets.json")))
    for e in d["sets"]:
        ps = I.ParamSet(e["mexp"], e["pos"], e["sh1"], e["sh2"], tuple(e["param_tbl"]), tuple(e["temper_tbl"]))
        g = M.Generator(ps, 3)
        out = g.generate(20000)
        ref, _ = O.stream(ps, 3, 20000)
        np.testing.assert_array_equal(host_bits(out), ref)
        g.close()


def test_error_paths(M):
    import torch
    (ps,), _ = I.single_stream()
    g = M.Generator(ps, 1)
    buf = torch.empty(16, dtype=torch.int32, device="cuda")
    # misaligned output pointer
    rc = M.lib().mtgp_generate_uint32(g._h, 4, M.ctypes.c_void_p(buf.data_ptr() + 2), None)
    assert rc == M.MTGP_EINVAL
    # NULL output with n > 0
    assert M.lib().mtgp_generate_uint32(g._h, 4, None, None) == M.MTGP_EINVAL
    # n = 0 with NULL output is a no-op
    assert M.lib().mtgp_generate_uint32(g._h, 0, None, None) == M.MTGP_OK
    _, consumed = g.get_state()
    assert consumed == 0
    g.close()


# ---------------------------------------------------------------------------
# Batches
# ---------------------------------------------------------------------------

def check_batch_against_oracle(M, params, seeds, calls, plain=False):
    """calls: list of request lists [(gen, kind, n)]; outputs checked after each call."""
    import torch
    b = M.Batch(params, seeds)
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    for reqs in calls:
        bufs = [torch.empty(max(n, 1), dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
        rq = [(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)]
        (b.generate_plain if plain else b.generate)(rq)
        torch.cuda.synchronize()
        with pool() as ex:
            refs = list(ex.map(lambda r: O.generate(params[r[0]], states[r[0]], r[2], r[1]), reqs))
        for (g, k, n), buf, ref in zip(reqs, bufs, refs):
            np.testing.assert_array_equal(host_bits(buf)[:n], ref, err_msg=f"gen={g} kind={k} n={n}")
    for g in range(len(params)):
        words, _ = b.get_state(g)
        np.testing.assert_array_equal(words, states[g], err_msg=f"state gen={g}")
    b.close()


def test_batch_small_uneven_mixed(M):
    params, reqs = I.batched_uneven(count=64, seed=77, log2_lo=0, log2_hi=15)
    seeds = I.state_seeds(len(params))
    calls = [[(r.gen, r.kind, r.n) for r in reqs],
             [(r.gen, (r.kind + 1) % 3, r.n // 3 + 1) for r in reqs[::2]]]
    say("batch small uneven")
    check_batch_against_oracle(M, params, seeds, calls)
    check_batch_against_oracle(M, params, seeds, calls, plain=True)


def test_batch_independent_128_all_kinds(M):
    """128 MTGP-11213 generators, 2^22 outputs each, in one launch, per kind."""
    params, n = I.independent_128()
    seeds = I.state_seeds(len(params))
    say("independent_128 full size")
    calls = [[(g, kind, n) for g in range(len(params))] for kind in KINDS]
    check_batch_against_oracle(M, params, seeds, calls)


def test_batch_rejects_bad_requests(M):
    import torch
    params, _ = I.independent_128()
    b = M.Batch(params[:4], I.state_seeds(4))
    buf = torch.empty(64, dtype=torch.int32, device="cuda")
    with pytest.raises(M.MTGPError):
        b.generate([(0, 0, 8, buf), (0, 0, 8, buf)])          # same generator twice
    with pytest.raises(M.MTGPError):
        b.generate([(9, 0, 8, buf)])                          # no such generator
    with pytest.raises(M.MTGPError):
        b.generate([(1, 4, 8, buf)])                          # no such kind (3 is the normal kind)
    b.close()


# ---------------------------------------------------------------------------
# Launch shapes: every valid shape gives the same bits
# ---------------------------------------------------------------------------

RB = 4   # mode flag: recursion table from its F2 basis in registers instead of the LDS lookup
SHAPES = [
    (0, 64, 1, 0, 0), (0, 64, 4, 0, 0), (0, 256, 1, 0, 0), (0, 256, 4, 0, 0), (0, 512, 2, 0, 0),
    (0, 1024, 1, 0, 0), (0, 256, 4, 24000, 0), (1, 64, 1, 0, 0), (1, 64, 4, 0, 0), (1, 256, 6, 0, 0),
    (1, 128, 16, 0, 0), (1, 256, 8, 4096, 3),
    (0 | RB, 64, 4, 0, 0), (0 | RB, 256, 1, 0, 0), (0 | RB, 512, 2, 0, 0), (0 | RB, 1024, 1, 0, 0),
    (1 | RB, 64, 1, 0, 0), (1 | RB, 256, 6, 0, 0), (1 | RB, 128, 16, 0, 0),
]


def test_launch_shapes_parity(M):
    import torch
    params = (I.draw_param_sets([11213] * 4, 61, I.M_POLICY_WIDE) + I.draw_param_sets([23209] * 2, 62)
              + I.draw_param_sets([44497] * 2, 63) + I.draw_param_sets([89, 521, 2203], 64, I.M_POLICY_FULL))
    seeds = I.state_seeds(len(params))
    b = M.Batch(params, seeds)
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    rng = I.SplitMix64(99)
    for i, sh in enumerate(SHAPES):
        say(f"shape {sh}")
        b.set_launch(*sh)
        reqs = []
        for g in range(len(params)):
            # every kind under every shape; normals in even counts, where
            # N - M >= 2 leaves room for a pair in a round
            k = (g + i) % 4
            if k == 3 and O.nwords(params[g].mexp) - params[g].pos < 2:
                k = 0
            n = rng.uniform_int(1, 9000)
            reqs.append((g, k, n + (n & 1) if k == 3 else n))
        bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
        b.generate([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
        torch.cuda.synchronize()
        for (g, k, n), buf in zip(reqs, bufs):
            if k == 3:
                err = np.abs(host_f32(buf) - O.normals(params[g], states[g], n)).max()
                assert err <= NORMAL_ATOL, f"shape={sh} gen={g} normal err={err}"
            else:
                ref = O.generate(params[g], states[g], n, k)
                np.testing.assert_array_equal(host_bits(buf), ref, err_msg=f"shape={sh} gen={g}")
    b.set_launch(-1)
    for g in range(len(params)):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g])
    b.close()


def test_wide_workgroups_long_streams(M):
    """Workgroups wider than N - M: the wavefronts past the round width skip
    its work and only meet the barriers, through many rounds, window
    compactions and a partial last round."""
    import torch
    params = I.draw_param_sets([11213, 11213, 521], 66, I.M_POLICY_WIDE) + I.draw_param_sets([23209], 67)
    seeds = I.state_seeds(len(params))
    for mode, threads in ((0, 512), (0, 1024), (RB, 512)):
        say(f"mode {mode} threads {threads}")
        b = M.Batch(params, seeds)
        b.set_launch(mode, threads, 1, 0, 0)
        states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
        for n in (300007, 4099):
            reqs = [(g, g % 3, n) for g in range(len(params))]
            bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in reqs]
            b.generate([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
            torch.cuda.synchronize()
            for (g, k, n), buf in zip(reqs, bufs):
                ref = O.generate(params[g], states[g], n, k)
                np.testing.assert_array_equal(host_bits(buf), ref, err_msg=f"mode={mode} threads={threads} gen={g} n={n}")
        for g in range(len(params)):
            np.testing.assert_array_equal(b.get_state(g)[0], states[g])
        b.close()


def test_outputs_at_addresses_with_bit31_set(M):
    """Output windows whose device address has bit 31 of its low word set, in
    both launch forms (regression: the low half of the address must be
    zero-extended when it is made wave-uniform)."""
    import torch
    params = I.draw_param_sets([11213] * 3 + [23209], 65)
    seeds = I.state_seeds(len(params))
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    n = 5000
    need = 4 * n * len(params)
    big = torch.empty((1 << 29) + (1 << 22), dtype=torch.int32, device="cuda")   # 2 GiB + 16 MiB
    base = big.data_ptr()
    off = 0 if (base >> 31) & 1 else (1 << 31) - (base & 0x7FFFFFFF)
    off = (off + 255) & ~255
    assert off + need <= big.numel() * 4 and ((base + off) >> 31) & 1
    b = M.Batch(params, seeds)
    for sh in [(0, 256, 4, 0, 0), (1, 256, 4, 0, 0)]:
        say(f"bit-31 outputs, shape {sh}")
        b.set_launch(*sh)
        b.generate([(g, g % 3, n, base + off + 4 * n * g) for g in range(len(params))])
        torch.cuda.synchronize()
        host = host_bits(big[off // 4: off // 4 + n * len(params)])
        for g in range(len(params)):
            np.testing.assert_array_equal(host[g * n:(g + 1) * n], O.generate(params[g], states[g], n, g % 3),
                                          err_msg=f"shape={sh} gen={g}")
    b.close()
    del big
    torch.cuda.empty_cache()


def test_single_generator_shapes(M):
    (ps,), _ = I.single_stream()
    st = O.seed_state(21, ps.mexp)
    g = M.Generator(ps, 21)
    for sh in [(0, 64, 4, 0), (0, 256, 1, 0), (0, 1024, 1, 2000), (1, 64, 16, 0), (1, 64, 4, 1000),
               (0 | RB, 256, 4, 0), (1 | RB, 64, 8, 0), (-1, 0, 1, 0)]:
        g.set_launch(*sh)
        out = g.generate(7777, I.KIND_F01)
        np.testing.assert_array_equal(host_bits(out), O.generate(ps, st, 7777, I.KIND_F01), err_msg=str(sh))
    with pytest.raises(M.MTGPError):
        g.set_launch(0, 256, 1, 100)          # window smaller than 2N + W
    with pytest.raises(M.MTGPError):
        g.set_launch(0, 96, 1, 0)             # not a multiple of 64
    with pytest.raises(M.MTGPError):
        g.set_launch(1, 64, 5, 0)             # unsupported steps per lane
    g.close()


def test_plan_graph_replays(M):
    """A captured plan replayed several times, with eager work and syncs in
    between, continues every stream exactly."""
    import torch
    params, reqs0 = I.batched_uneven(count=16, seed=31, log2_lo=4, log2_hi=14)
    seeds = I.state_seeds(len(params))
    b = M.Batch(params, seeds)
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    planned = [r for r in reqs0 if r.gen < 12]
    bufs = {r.gen: torch.empty(r.n, dtype=torch.int32, device="cuda") for r in planned}
    plan = b.plan([(r.gen, r.kind, r.n, bufs[r.gen]) for r in planned])
    eager_gens = [12, 13, 14, 15]
    for rep in range(4):
        say(f"plan replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        for r in planned:
            ref = O.generate(params[r.gen], states[r.gen], r.n, r.kind)
            np.testing.assert_array_equal(host_bits(bufs[r.gen]), ref, err_msg=f"replay={rep} gen={r.gen}")
        # eager work on other generators between replays
        eb = [torch.empty(500 + rep, dtype=torch.int32, device="cuda") for _ in eager_gens]
        b.generate([(g, 0, 500 + rep, t) for g, t in zip(eager_gens, eb)])
        torch.cuda.synchronize()
        for g, t in zip(eager_gens, eb):
            np.testing.assert_array_equal(host_bits(t), O.generate(params[g], states[g], 500 + rep, 0))
        _ = (torch.arange(1000, device="cuda") * 3).sum().item()
    for g in range(len(params)):
        w, consumed = b.get_state(g)
        np.testing.assert_array_equal(w, states[g])
    plan.close()
    b.close()


# ---------------------------------------------------------------------------
# Jump-ahead: split plans give the unsplit stream's bits
# ---------------------------------------------------------------------------

def test_plan_split_jump_ahead(M):
    import json
    import torch
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fullperiod_sets.json")))
    full = [I.ParamSet(e["mexp"], e["pos"], e["sh1"], e["sh2"], tuple(e["param_tbl"]), tuple(e["temper_tbl"]))
            for e in d["sets"] if e["mexp"] >= 521]
    params = (I.draw_param_sets([11213] * 3, 71) + I.draw_param_sets([11213], 72, I.M_POLICY_WIDE)
              + I.draw_param_sets([23209], 73) + I.draw_param_sets([44497], 74)
              # state sizes for every lane width of the jump kernel (6 .. 16 words a lane)
              + I.draw_param_sets([15000, 65536, 12315, 16411, 18459, 24603, 26651, 28699], 76) + full)
    seeds = I.state_seeds(len(params))
    b = M.Batch(params, seeds)
    b.set_split(6)
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    rng = I.SplitMix64(75)
    reqs = [(g, g % 3, rng.uniform_int(30000, 90000)) for g in range(len(params))]
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    # an eager call first, so the plan starts mid-stream
    eb = [torch.empty(777, dtype=torch.int32, device="cuda") for _ in params]
    b.generate([(g, 0, 777, eb[g]) for g in range(len(params))])
    for g in range(len(params)):
        np.testing.assert_array_equal(host_bits(eb[g]), O.generate(params[g], states[g], 777, 0))
    plan = b.plan([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    for rep in range(3):
        say(f"split plan replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        for (g, k, n), buf in zip(reqs, bufs):
            ref = O.generate(params[g], states[g], n, k)
            np.testing.assert_array_equal(host_bits(buf), ref, err_msg=f"replay={rep} gen={g} mexp={params[g].mexp}")
        b.generate([(g, 1, 333, eb[g]) for g in range(len(params))])
        torch.cuda.synchronize()
        for g in range(len(params)):
            np.testing.assert_array_equal(host_bits(eb[g])[:333], O.generate(params[g], states[g], 333, 1))
    # the same requests as a plan with the recursion table's basis form
    b.set_launch(RB, 256, 1, 0, 0)
    plan2 = b.plan([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    say("split plan, basis form")
    plan2.launch()
    torch.cuda.synchronize()
    for (g, k, n), buf in zip(reqs, bufs):
        ref = O.generate(params[g], states[g], n, k)
        np.testing.assert_array_equal(host_bits(buf), ref, err_msg=f"basis form gen={g} mexp={params[g].mexp}")
    plan2.close()
    b.set_launch(-1)
    for g in range(len(params)):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g])
    # replacing a split generator's state makes the plan stale
    b.set_state(0, states[0], 0)
    with pytest.raises(M.MTGPError):
        plan.launch()
    plan.close()
    b.close()


def test_plan_phases(M):
    """PREPARE then GENERATE equals a whole launch, split or not."""
    import torch
    params = I.draw_param_sets([11213] * 4 + [23209] * 2, 81)
    seeds = I.state_seeds(len(params))
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    rng = I.SplitMix64(82)
    reqs = [(g, g % 3, rng.uniform_int(20000, 60000)) for g in range(len(params))]
    for split in (0, 8):
        say(f"plan phases split={split}")
        b = M.Batch(params, seeds)
        b.set_split(split)
        st = {g: v.copy() for g, v in states.items()}
        bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
        plan = b.plan([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
        for rep in range(2):
            plan.launch_phase(M.PHASE_PREPARE)
            plan.launch_phase(M.PHASE_GENERATE)
            torch.cuda.synchronize()
            for (g, k, n), buf in zip(reqs, bufs):
                np.testing.assert_array_equal(host_bits(buf), O.generate(params[g], st[g], n, k),
                                              err_msg=f"split={split} rep={rep} gen={g}")
        for g, (_, _, n) in enumerate(reqs):
            words, consumed = b.get_state(g)
            np.testing.assert_array_equal(words, st[g])
            assert consumed == 2 * n
        with pytest.raises(M.MTGPError):
            plan.launch_phase(7)
        plan.close()
        b.close()


def test_autotune_leaves_streams_and_keeps_parity(M):
    import torch
    params = I.draw_param_sets([11213] * 6 + [44497] * 2, 83)
    seeds = I.state_seeds(len(params))
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    n = 1 << 17
    out = torch.empty(len(params) * n, dtype=torch.int32, device="cuda")
    reqs = [(g, g % 3, n, out.data_ptr() + 4 * g * n) for g in range(len(params))]
    b = M.Batch(params, seeds)
    say("autotune")
    best = b.autotune(reqs, reps=2)
    say(f"autotune chose {best}")
    assert best["trials"] >= 2 and best["ms"] > 0 and best["mode"] in (-1, 0, 1, RB, 1 | RB)
    for g in range(len(params)):
        words, consumed = b.get_state(g)
        np.testing.assert_array_equal(words, states[g])
        assert consumed == 0
    plan = b.plan(reqs)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        host = host_bits(out)
        for g in range(len(params)):
            np.testing.assert_array_equal(host[g * n:(g + 1) * n], O.generate(params[g], states[g], n, g % 3),
                                          err_msg=f"rep={rep} gen={g}")
    plan.close()
    b.close()


# ---------------------------------------------------------------------------
# Box-Muller normals. binary32 on the device (hardware log2, square root and
# sine) against the float64 oracle: 2 - a, b - 1 and b - 1 + 1/4 are exact;
# over all 2^23 possible inputs, measured on gfx950, r = sqrt(-2 ln(2 - a))
# is within 4.7e-7 and sin, cos(2 pi (b - 1)) within 1.3e-7, so
# |z - z_ref| <= 4.7e-7 + 5.65 * 1.3e-7 + 0.5 ulp(z) ~= 1.5e-6 (r <= 5.65).
# The tolerance below keeps a factor of ten over that.
# ---------------------------------------------------------------------------

NORMAL_ATOL = 1.5e-5


def host_f32(t):
    return t.view(__import__("torch").float32).cpu().numpy().astype(np.float64)


def test_normals_single_generator_and_continuation(M):
    (ps,), _ = I.single_stream()
    st = O.seed_state(31, ps.mexp)
    g = M.Generator(ps, 31)
    for n in (2, 20000, 2 * 7777):
        z = g.generate(n, M.KIND_NORMAL_FLOAT32)
        ref = O.normals(ps, st, n)
        err = np.abs(host_f32(z) - ref).max()
        say(f"normals n={n} max |err| = {err:.3g}")
        assert err <= NORMAL_ATOL
    # the position advanced by exactly n per call: integer outputs continue bit-exactly
    out = g.generate(9999, M.KIND_UINT32)
    np.testing.assert_array_equal(host_bits(out), O.generate(ps, st, 9999, O.U32))
    with pytest.raises(M.MTGPError):
        g.generate(7, M.KIND_NORMAL_FLOAT32)          # odd count
    g.close()


@pytest.mark.parametrize("shape", [None, (1 | RB, 64, 16, 0, 0), (RB, 256, 4, 0, 0)])
def test_normals_batch_and_split_plan(M, shape):
    """Normals beside the other kinds in an eager batch and as a split plan,
    under the automatic shape, the wavefront form with the recursion basis
    (pairs split across DPP lanes, rounds of W & ~1 steps) and the workgroup
    form with the recursion basis."""
    import torch
    say(f"normals under shape {shape}")
    params = I.draw_param_sets([11213] * 3 + [23209, 44497], 93)
    seeds = I.state_seeds(len(params))
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    rng = I.SplitMix64(94)
    b = M.Batch(params, seeds)
    if shape is not None:
        b.set_launch(*shape)
    # eager batch: normals beside the other kinds, even ragged lengths
    reqs = [(g, [3, 0, 3, 1, 3][g], 2 * rng.uniform_int(1, 30000)) for g in range(len(params))]
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    b.generate([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    torch.cuda.synchronize()
    for (g, k, n), buf in zip(reqs, bufs):
        if k == 3:
            assert np.abs(host_f32(buf) - O.normals(params[g], states[g], n)).max() <= NORMAL_ATOL
        else:
            np.testing.assert_array_equal(host_bits(buf), O.generate(params[g], states[g], n, k))
    # a split plan of normals: segments hold whole pairs
    b.set_split(8)
    reqs = [(g, 3, 2 * rng.uniform_int(20000, 40000)) for g in range(len(params))]
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    plan = b.plan([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for (g, k, n), buf in zip(reqs, bufs):
            err = np.abs(host_f32(buf) - O.normals(params[g], states[g], n)).max()
            assert err <= NORMAL_ATOL, f"rep={rep} gen={g} err={err}"
    plan.close()
    for g in range(len(params)):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g])
    with pytest.raises(M.MTGPError):
        b.generate([(0, 3, 5, bufs[0])])                # odd count
    b.close()


def test_single_generator_split_calls(M):
    """Eager calls split into jump-ahead segments equal the unsplit stream,
    across lengths (the jump buffers are rebuilt), kinds and set_state."""
    params = I.draw_param_sets([11213], 95) + I.draw_param_sets([23209], 96)
    d = __import__("json").load(open(os.path.join(os.path.dirname(__file__), "golden", "fullperiod_sets.json")))
    e = [x for x in d["sets"] if x["mexp"] == 2203][0]
    params.append(I.ParamSet(e["mexp"], e["pos"], e["sh1"], e["sh2"], tuple(e["param_tbl"]), tuple(e["temper_tbl"])))
    for ps in params:
        st = O.seed_state(41, ps.mexp)
        g = M.Generator(ps, 41)
        g.set_split(8)
        for n, kind in ((100000, 0), (100000, 1), (2 * 40001, 3), (999, 0), (250001, 2), (100000, 0)):
            say(f"split call mexp={ps.mexp} n={n} kind={kind}")
            out = g.generate(n, kind)
            if kind == 3:
                assert np.abs(host_f32(out) - O.normals(ps, st, n)).max() <= NORMAL_ATOL
            else:
                np.testing.assert_array_equal(host_bits(out), O.generate(ps, st, n, kind),
                                              err_msg=f"mexp={ps.mexp} n={n} kind={kind}")
        words, consumed = g.get_state()
        np.testing.assert_array_equal(words, st)
        # a new state: the annihilator and the jump polynomials are rebuilt
        st2 = O.seed_state(777, ps.mexp)
        g.set_state(st2, 0)
        out = g.generate(100000, 0)
        np.testing.assert_array_equal(host_bits(out), O.generate(ps, st2, 100000, 0))
        # the segments take the generator's recursion-table form
        g.set_launch(RB, 256, 4, 0)
        out = g.generate(100000, 1)
        np.testing.assert_array_equal(host_bits(out), O.generate(ps, st2, 100000, 1))
        g.close()


def test_eager_batch_calls_split(M):
    """With a split limit, an eager batch call holding a long request runs as
    jump-ahead segments (a one-off plan, replaced by the next such call);
    outputs equal the unsplit stream across consecutive calls, a short call
    that stays unsplit, and every kind."""
    import torch
    params = I.draw_param_sets([11213] * 3, 97) + I.draw_param_sets([23209], 98)
    seeds = I.state_seeds(len(params))
    b = M.Batch(params, seeds)
    b.set_split(64)
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    calls = ((200004, (0, 1, 2, 0)), (998, (1, 0, 2, 3)), (150000, (3, 2, 1, 0)), (300002, (0, 0, 3, 0)))
    for n, kinds in calls:
        say(f"eager split call n={n} kinds={kinds}")
        bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in params]
        b.generate([(g, kinds[g], n, bufs[g]) for g in range(len(params))])
        torch.cuda.synchronize()
        for g in range(len(params)):
            if kinds[g] == 3:
                assert np.abs(host_f32(bufs[g]) - O.normals(params[g], states[g], n)).max() <= NORMAL_ATOL
            else:
                np.testing.assert_array_equal(host_bits(bufs[g]), O.generate(params[g], states[g], n, kinds[g]),
                                              err_msg=f"n={n} gen={g} kind={kinds[g]}")
    for g in range(len(params)):
        words, consumed = b.get_state(g)
        np.testing.assert_array_equal(words, states[g])
        assert consumed == sum(n for n, _ in calls)
    b.close()


# ---------------------------------------------------------------------------
# A searched, paper-shaped production-size set (section 5): sh1 = 13, sh2 = 4,
# an ID embedded in R, period 2^11213 - 1. The library's seeded host search
# produces it at test time (the same seed as the slow search test, whose
# oracle run pins its full period by Berlekamp-Massey and the irreducibility
# test); nothing is stored. The GPU's outputs are compared with the oracle's.
# ---------------------------------------------------------------------------

def test_searched_full_period_11213_set(M):
    import torch
    found, stats = M.search_params(11213, id=1, seed=11213)
    ps = I.ParamSet(found.mexp, found.pos, found.sh1, found.sh2, tuple(found.param_tbl), tuple(found.temper_tbl))
    say(f"searched set: M={ps.pos} sh1={ps.sh1} sh2={ps.sh2} after {stats['draws']} draws")
    assert (ps.sh1, ps.sh2) == (13, 4) and ps.param_tbl[8] >> 16 == 0 and (ps.param_tbl[4] >> 4) & 0xFFFF == 1
    # a batch of 64 states of the one set (the deployment the paper describes:
    # one parameter set per block of work, many seeds), every kind, ragged
    # lengths, then a split plan over the continued streams
    G = 64
    seeds = [11213 + 7 * g for g in range(G)]
    params = [ps] * G
    b = M.Batch(params, seeds)
    states = {g: O.seed_state(seeds[g], ps.mexp) for g in range(G)}
    rng = I.SplitMix64(11214)
    reqs = []
    for g in range(G):
        k = g % 4
        n = rng.uniform_int(1, 70000)
        reqs.append((g, k, n + (n & 1) if k == 3 else n))
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    b.generate([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    torch.cuda.synchronize()
    for (g, k, n), buf in zip(reqs, bufs):
        if k == 3:
            assert np.abs(host_f32(buf) - O.normals(ps, states[g], n)).max() <= NORMAL_ATOL, f"gen={g}"
        else:
            np.testing.assert_array_equal(host_bits(buf), O.generate(ps, states[g], n, k), err_msg=f"gen={g} kind={k}")
    b.set_split(64)
    reqs = [(g, g % 3, 200_000 + 997 * g) for g in range(8)]
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    plan = b.plan([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    for (g, k, n), buf in zip(reqs, bufs):
        np.testing.assert_array_equal(host_bits(buf), O.generate(ps, states[g], n, k), err_msg=f"split gen={g}")
    for g in range(G):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g], err_msg=f"end state gen={g}")
    b.close()


# The two larger released sizes, searched the same way at test time: the
# seeded call that the benchmark's search sections accept (p = 23209: seed
# 23209, accepted at draw 40901, about 20 s on 16 host cores; p = 44497: seed
# 44502, the sixth of its rounds of 4000 draws, accepted at draw 2327, about
# 11 s). Their full period is not re-derived by the oracle here (its
# irreducibility test would take tens of minutes at these degrees); the
# parity below does not depend on it.
@pytest.mark.parametrize("mexp,seed,draws", [(23209, 23209, 200000), (44497, 44502, 4000)])
def test_searched_large_sets(M, mexp, seed, draws):
    import torch
    say(f"search p={mexp} seed={seed}")
    found, stats = M.search_params(mexp, id=1, seed=seed, max_draws=draws)
    ps = I.ParamSet(found.mexp, found.pos, found.sh1, found.sh2, tuple(found.param_tbl), tuple(found.temper_tbl))
    say(f"searched set p={mexp}: M={ps.pos} after {stats['draws']} draws")
    assert (ps.sh1, ps.sh2) == (13, 4)
    G = 16
    seeds = [mexp + 3 * g for g in range(G)]
    b = M.Batch([ps] * G, seeds)
    states = {g: O.seed_state(seeds[g], ps.mexp) for g in range(G)}
    rng = I.SplitMix64(mexp + 1)
    reqs = []
    for g in range(G):
        k = g % 4
        n = rng.uniform_int(1, 90000)
        reqs.append((g, k, n + (n & 1) if k == 3 else n))
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    b.generate([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    torch.cuda.synchronize()
    for (g, k, n), buf in zip(reqs, bufs):
        if k == 3:
            assert np.abs(host_f32(buf) - O.normals(ps, states[g], n)).max() <= NORMAL_ATOL, f"gen={g}"
        else:
            np.testing.assert_array_equal(host_bits(buf), O.generate(ps, states[g], n, k), err_msg=f"gen={g} kind={k}")
    # jump-ahead segments over the continued streams (the orbit annihilator of
    # a full-period state has degree p)
    b.set_split(64)
    reqs = [(g, g % 3, 300_000 + 1009 * g) for g in range(6)]
    bufs = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
    plan = b.plan([(g, k, n, buf) for (g, k, n), buf in zip(reqs, bufs)])
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    for (g, k, n), buf in zip(reqs, bufs):
        np.testing.assert_array_equal(host_bits(buf), O.generate(ps, states[g], n, k), err_msg=f"split gen={g}")
    for g in range(G):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g], err_msg=f"end state gen={g}")
    b.close()
