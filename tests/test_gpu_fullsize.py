"""Parity at the workloads' full sizes, in the configurations the benchmark
times: autotuned jump-ahead plans for the 4096-request uneven batch (the
headline; every output of two replays, copied back in chunks), the 128 x 2^22
batch, the 256 x 2^24 large-state batches (under the paper's M rule and the
wide one), and the native request loop over 65536 states (every request).
The oracle runs on host threads (its C calls release the GIL).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O
from paper_1005_4973_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1005_4973_amd import mtgp
    mtgp.lib()
    return mtgp


def pool():
    return ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4))


def device_words(out, start, n):
    """n uint32 words of a device int32 tensor from word `start`."""
    return out[start:start + n].cpu().numpy().view(np.uint32)


@pytest.mark.timeout(600)
def test_independent_128_tuned_plans_full_size(M):
    """128 MTGP-11213 generators x 2^22 as uint32, float [1,2), float [0,1):
    the tuned split plans, replayed twice; all outputs compared."""
    import torch
    params, n = I.independent_128()
    G = len(params)
    seeds = I.state_seeds(G)
    kinds = (I.KIND_U32, I.KIND_F12, I.KIND_F01)
    b = M.Batch(params, seeds)
    outs = {k: torch.empty(G * n, dtype=torch.int32, device="cuda") for k in kinds}
    reqs = {k: [(g, k, n, outs[k].data_ptr() + 4 * g * n) for g in range(G)] for k in kinds}
    tuning = b.autotune(reqs[I.KIND_U32], reps=2)
    say(f"128 x 2^22 tuning {tuning}")
    plans = [b.plan(reqs[k]) for k in kinds]
    states = [O.seed_state(seeds[g], params[g].mexp) for g in range(G)]
    for rep in range(2):
        for p in plans:
            p.launch()
        torch.cuda.synchronize()
        for k in kinds:
            say(f"replay {rep} kind {k}")
            host = outs[k].cpu().numpy().view(np.uint32)
            with pool() as ex:
                refs = list(ex.map(lambda g: O.generate(params[g], states[g], n, k), range(G)))
            for g in range(G):
                np.testing.assert_array_equal(host[g * n:(g + 1) * n], refs[g], err_msg=f"rep={rep} kind={k} gen={g}")
    for g in range(G):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g])
    for p in plans:
        p.close()
    b.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mexp,split", [(23209, 8192), (44497, 8192)])
def test_large_states_full_size(M, mexp, split):
    """256 generators x 2^24 uint32 (16 GiB) as the benchmark's tuned split
    plan; every generator's complete stream compared (copied back 16
    generators at a time), and every final state."""
    import torch
    params, n = I.large_states(mexp)
    G = len(params)
    seeds = I.state_seeds(G)
    b = M.Batch(params, seeds)
    b.set_split(split)
    out = torch.empty(G * n, dtype=torch.int32, device="cuda")
    plan = b.plan([(g, 0, n, out.data_ptr() + 4 * g * n) for g in range(G)])
    say(f"p={mexp} split={split}")
    plan.launch()
    torch.cuda.synchronize()
    states = {g: O.seed_state(seeds[g], mexp) for g in range(G)}
    chunk = 16
    with pool() as ex:
        for g0 in range(0, G, chunk):
            gens = range(g0, min(G, g0 + chunk))
            host = device_words(out, g0 * n, len(gens) * n)
            refs = list(ex.map(lambda g: O.generate(params[g], states[g], n, 0), gens))
            for g, ref in zip(gens, refs):
                np.testing.assert_array_equal(host[(g - g0) * n:(g - g0 + 1) * n], ref, err_msg=f"p={mexp} gen={g}")
    say(f"p={mexp}: all {G} streams equal")
    for g in range(G):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g], err_msg=f"p={mexp} state gen={g}")
    plan.close()
    b.close()
    del out
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_large_states_wide_m_full_size(M):
    """The M-rule sensitivity batch (256 MTGP-23209 generators, M in [2, N-2],
    2^24 uint32 each) as the autotuned plan: thousands of jump-ahead segments,
    many of them for generators whose rounds are a few words wide; every
    stream and every end state compared."""
    import torch
    params, n = I.large_states_wide_m(23209)
    G = len(params)
    seeds = I.state_seeds(G)
    b = M.Batch(params, seeds)
    out = torch.empty(G * n, dtype=torch.int32, device="cuda")
    reqs = [(g, 0, n, out.data_ptr() + 4 * g * n) for g in range(G)]
    tuning = b.autotune(reqs, reps=1)
    say(f"wide-M tuning {tuning}")
    plan = b.plan(reqs)
    plan.launch()
    torch.cuda.synchronize()
    states = {g: O.seed_state(seeds[g], 23209) for g in range(G)}
    chunk = 16
    with pool() as ex:
        for g0 in range(0, G, chunk):
            gens = range(g0, min(G, g0 + chunk))
            host = device_words(out, g0 * n, len(gens) * n)
            refs = list(ex.map(lambda g: O.generate(params[g], states[g], n, 0), gens))
            for g, ref in zip(gens, refs):
                np.testing.assert_array_equal(host[(g - g0) * n:(g - g0 + 1) * n], ref,
                                              err_msg=f"gen={g} N-M={726 - params[g].pos}")
    say(f"wide M: all {G} streams equal")
    for g in range(G):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g], err_msg=f"state gen={g}")
    plan.close()
    b.close()
    del out
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_batched_uneven_full_size(M):
    """4096 requests, exponents 2:1:1, lengths log-uniform in [2^10, 2^24],
    mixed kinds, autotuned persistent plan replayed twice (the second replay's
    segments start from jumps over the states the first one left): every
    request's outputs compared after each replay (copied back about 1 GiB at
    a time), and every final state."""
    import torch
    params, reqs = I.batched_uneven()
    G = len(params)
    seeds = I.state_seeds(G)
    tot = sum(r.n for r in reqs)
    b = M.Batch(params, seeds)
    out = torch.empty(tot, dtype=torch.int32, device="cuda")
    rq = [(r.gen, r.kind, r.n, out.data_ptr() + 4 * r.offset) for r in reqs]
    tuning = b.autotune(rq, reps=1)
    say(f"uneven tuning {tuning}")
    plan = b.plan(rq)
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(G)}
    # requests are packed in order: compare them in groups of about 2^28 outputs
    groups, cur, size = [], [], 0
    for r in reqs:
        cur.append(r)
        size += r.n
        if size >= 1 << 28:
            groups.append(cur)
            cur, size = [], 0
    if cur:
        groups.append(cur)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        with pool() as ex:
            for grp in groups:
                base = grp[0].offset
                host = device_words(out, base, grp[-1].offset + grp[-1].n - base)
                refs = list(ex.map(lambda r: O.generate(params[r.gen], states[r.gen], r.n, r.kind), grp))
                for r, want in zip(grp, refs):
                    np.testing.assert_array_equal(
                        host[r.offset - base:r.offset - base + r.n], want,
                        err_msg=f"rep={rep} gen={r.gen} mexp={params[r.gen].mexp} n={r.n} kind={r.kind}")
        say(f"uneven replay {rep}: all {len(reqs)} requests equal")
    for g in range(G):
        np.testing.assert_array_equal(b.get_state(g)[0], states[g], err_msg=f"state gen={g}")
    plan.close()
    b.close()
    del out
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_native_server_full_size(M):
    """65536 resident MTGP-11213 states behind the library's request loop with
    the benchmark's arena and chunk, request sizes of the serving workload
    (log-normal, median 2^16, clipped to [2^10, 2^26]), all submitted at once;
    a quarter of the requests go to 64 busy generators so that FIFO order per
    generator matters. Every request is compared with the oracle's stream
    segment for its generator in arrival order."""
    import torch
    from paper_1005_4973_amd import serve
    G = 65536
    params = I.serving_params(G)
    seeds = I.state_seeds(G)
    trace = I.serving_trace(3000, rate_per_s=1.0, num_gens=G, seed=5001)
    trace = [(t, g % 64 if i % 4 == 0 else g, n, k) for i, (t, g, n, k) in enumerate(trace)]
    b = M.Batch(params, seeds)
    srv = serve.NativeServer(b, arena_bytes=8 << 30, chunk=1 << 18, depth=2)
    got = {}

    def keep(rid, view):
        got[rid] = view.cpu().numpy().view(np.uint32).copy()

    say(f"server: {len(trace)} requests")
    st = srv.run(trace, realtime=False, on_complete=keep)
    srv.close()
    assert st.completed == len(trace) and len(got) == len(trace)
    by_gen = {}
    for rid, (_, g, n, k) in enumerate(trace):
        by_gen.setdefault(g, []).append((rid, n, k))
    gens = sorted(by_gen)

    def check(g):
        s = O.seed_state(seeds[g], params[g].mexp)
        for rid, n, k in by_gen[g]:
            np.testing.assert_array_equal(got[rid], O.generate(params[g], s, n, k), err_msg=f"rid={rid} gen={g}")
        return s

    with pool() as ex:
        finals = list(ex.map(check, gens))
    for g, s in zip(gens, finals):   # the batch handle is used from this thread only
        np.testing.assert_array_equal(b.get_state(g)[0], s, err_msg=f"state gen={g}")
    b.close()
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_calls_beyond_2_32_outputs(M):
    """The largest single calls: 2^32 + 65541 uint32 outputs (17.2 GB) in one
    call, so that every count and offset on the path needs more than 32 bits.
    Five paths over the same generator and seed: one generator without split
    in each of the three launch forms (one workgroup, one wavefront, the
    chunked wavefront form run the whole call), the same with jump-ahead
    segments, and a batch plan with a split limit. Each is compared with the oracle on the
    first 4096 outputs, the 8192 around output 2^32, the last 1000, the end
    state and consumed count, and a short call that continues the stream."""
    import torch
    n = (1 << 32) + 65541
    ps = I.draw_param_sets([11213], 7100)[0]
    seed = 4242
    # windows [0, 4096), [2^32 - 4096, 2^32 + 4096), [n - 1000, n), in order
    mid_at, tail_at = (1 << 32) - 4096, n - 1000
    assert 4096 <= mid_at and mid_at + 8192 <= tail_at

    def advance(st, k):
        assert k >= 0
        while k > 0:
            step = min(k, 1 << 30)
            O.advance(ps, st, step)
            k -= step
            say(f"oracle: {k} steps to the next window")

    st = O.seed_state(seed, ps.mexp)
    head = O.generate(ps, st, 4096)
    advance(st, mid_at - 4096)
    mid = O.generate(ps, st, 8192)
    advance(st, tail_at - mid_at - 8192)
    tail = O.generate(ps, st, 1000)
    end_state = st.copy()
    after = O.generate(ps, st, 3001)
    out = torch.empty(n, dtype=torch.int32, device="cuda")

    def check(tag):
        torch.cuda.synchronize()
        np.testing.assert_array_equal(device_words(out, 0, 4096), head, err_msg=tag)
        np.testing.assert_array_equal(device_words(out, mid_at, 8192), mid, err_msg=tag)
        np.testing.assert_array_equal(device_words(out, tail_at, 1000), tail, err_msg=tag)

    # (mode, lanes, steps per lane or read-ahead): workgroup form, wavefront
    # form, chunked form (N - M = 280 for this set, enough for read-ahead 2)
    for split, launch in ((0, None), (0, (1, 64, 4)), (0, (2, 64, 2)), (1 << 14, None)):
        say(f"generator, split {split}, launch {launch}")
        out.zero_()
        g = M.Generator(ps, seed)
        if split:
            g.set_split(split)
        if launch:
            g.set_launch(*launch, 0)
        g.generate(n, M.KIND_UINT32, out)
        check(f"generator split={split} launch={launch}")
        words, consumed = g.get_state()
        np.testing.assert_array_equal(words, end_state)
        assert consumed == n
        nxt = g.generate(3001, M.KIND_UINT32)
        np.testing.assert_array_equal(nxt.cpu().numpy().view(np.uint32), after)
        g.close()
    say("batch plan, split 8192 rounds")
    out.zero_()
    b = M.Batch([ps], [seed])
    b.set_split(8192)
    p = b.plan([(0, M.KIND_UINT32, n, out.data_ptr())])
    p.launch()
    check("batch plan")
    words, consumed = b.get_state(0)
    np.testing.assert_array_equal(words, end_state)
    assert consumed == n
    p.close()
    b.close()
    del out
    torch.cuda.empty_cache()
