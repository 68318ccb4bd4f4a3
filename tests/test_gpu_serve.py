"""Serving on the GPU: a mixed trace through the continuous-batching server
gives every request the same bits as running its generator's requests alone,
and the oracle's stream segments."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1005_4973_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1005_4973_amd import mtgp, serve
    mtgp.lib()
    return torch, mtgp, serve


def bits(t):
    import torch
    return t.view(torch.int32).cpu().numpy().view(np.uint32)


def test_serving_alone_vs_mix(env):
    torch, mtgp, serve = env
    G = 512
    params = I.draw_param_sets([11213] * G, 5100)
    seeds = I.state_seeds(G)
    trace = I.serving_trace(600, rate_per_s=20000.0, num_gens=G, seed=5200, median_log2=12, sigma=1.5,
                            lo_log2=4, hi_log2=17)
    # concentrate some traffic on a few generators so FIFO order matters
    trace = [(t, g % 40 if i % 3 == 0 else g, n, k) for i, (t, g, n, k) in enumerate(trace)]
    say(f"mixed trace: {len(trace)} requests")
    b = mtgp.Batch(params, seeds)
    srv = serve.Server(serve.GpuExecutor(b), mem_budget_bytes=64 << 20, chunk=1 << 13, depth=2)
    st = srv.run(trace, realtime=True)
    assert st.completed == len(trace)
    mixed = {r.rid: bits(r.out) for r in srv.completed}
    b.close()
    # oracle: per generator in arrival order
    states = {}
    for rid, (_, g, n, k) in enumerate(trace):
        st_g = states.setdefault(g, O.seed_state(seeds[g], params[g].mexp))
        np.testing.assert_array_equal(mixed[rid], O.generate(params[g], st_g, n, k), err_msg=f"rid={rid}")
    # alone: a fresh batch serving only one generator's requests
    for g in (0, 1, 39):
        sub = [(rid, t) for rid, t in enumerate(trace) if t[1] == g]
        say(f"alone gen={g}: {len(sub)} requests")
        b1 = mtgp.Batch(params, seeds)
        s1 = serve.Server(serve.GpuExecutor(b1), mem_budget_bytes=64 << 20, chunk=1 << 13)
        s1.run([t for _, t in sub], realtime=False)
        for (rid, _), r in zip(sub, sorted(s1.completed, key=lambda r: r.rid)):
            np.testing.assert_array_equal(bits(r.out), mixed[rid])
        b1.close()


def test_native_server_alone_vs_mix(env):
    """The library's request loop: a mixed trace gives every request the
    oracle's stream segment for its generator in arrival order, including
    normals (within the normal kind's tolerance) and a small arena that makes
    requests wait for space."""
    torch, mtgp, serve = env
    G = 256
    params = I.draw_param_sets([11213] * G, 5300)
    seeds = I.state_seeds(G)
    trace = I.serving_trace(800, rate_per_s=40000.0, num_gens=G, seed=5400, median_log2=12, sigma=1.5,
                            lo_log2=4, hi_log2=17)
    # a few busy generators; every fifth request asks for normals (even n)
    trace = [(t, g % 24 if i % 3 == 0 else g, (n + 1) // 2 * 2 if i % 5 == 0 else n, 3 if i % 5 == 0 else k)
             for i, (t, g, n, k) in enumerate(trace)]
    say(f"native server trace: {len(trace)} requests")
    b = mtgp.Batch(params, seeds)
    srv = serve.NativeServer(b, arena_bytes=8 << 20, chunk=1 << 13, depth=2)
    got = {}
    st = srv.run(trace, realtime=True, on_complete=lambda rid, out: got.__setitem__(rid, bits(out)))
    assert st.completed == len(trace) and len(got) == len(trace)
    assert srv.pending() == (0, 0, 0)
    states = {}
    for rid, (_, g, n, k) in enumerate(trace):
        assert got[rid].size == n
        st_g = states.setdefault(g, O.seed_state(seeds[g], params[g].mexp))
        if k == 3:
            z = got[rid].view(np.float32).astype(np.float64)
            assert np.abs(z - O.normals(params[g], st_g, n)).max() <= 1.5e-5, f"rid={rid}"
        else:
            np.testing.assert_array_equal(got[rid], O.generate(params[g], st_g, n, k), err_msg=f"rid={rid}")
    # keep mode: a trace whose kept outputs outgrow the arena raises instead of waiting forever
    srv2 = serve.NativeServer(b, arena_bytes=1 << 20, chunk=1 << 13, depth=2)
    with pytest.raises(RuntimeError):
        srv2.run([(0.0, g, 1 << 17, 0) for g in range(4)], realtime=False, keep=True)
    srv2.close()
    srv.close()
    b.close()


@pytest.mark.skip(reason="split ticks are switched off in the library (mtgp_server_set_split refuses them): "
                         "the first device run of this test stopped answering and no cause has been shown yet")
def test_native_server_split_alone_vs_mix(env):
    """Jump-ahead inside the request loop: requests above the split limit on
    prepared generators run as concurrent segments (started in whatever tick
    their polynomials are ready, so some first advance by plain chunks),
    beside short requests, requests of unprepared generators and normals.
    Every request gets the oracle's stream segment for its generator in
    arrival order, and the generators end in the oracle's states."""
    torch, mtgp, serve = env
    G = 64
    params = I.draw_param_sets([11213] * 40 + [23209] * 16 + [44497] * 8, 5500)
    seeds = I.state_seeds(G)
    rng = I.SplitMix64(5501)
    trace, t = [], 0.0
    for i in range(400):
        t += 2e-5
        g = rng.uniform_int(0, G - 1) if i % 4 else rng.uniform_int(0, 11)
        if i % 9 == 0:
            n = rng.uniform_int(200_000, 600_000)        # above the split limit
        else:
            n = rng.uniform_int(1, 20_000)
        k = 3 if i % 7 == 0 else rng.uniform_int(0, 2)
        if k == 3:
            n += n & 1
        trace.append((t, g, n, k))
    # long requests on generators 0..47 can split; 48..63 have no annihilator
    b = mtgp.Batch(params, seeds)
    b.prepare_split(range(48))
    chunk = 1 << 14
    say(f"split server trace: {len(trace)} requests, {sum(1 for x in trace if x[2] >= 200_000)} long")
    srv = serve.NativeServer(b, arena_bytes=64 << 20, chunk=chunk, depth=2, split=(1 << 16, 8, 2, 16))
    got = {}
    st = srv.run(trace, realtime=True, on_complete=lambda rid, out: got.__setitem__(rid, bits(out)))
    assert st.completed == len(trace) and len(got) == len(trace)
    assert srv.pending() == (0, 0, 0)
    srv.close()
    states = {}
    for rid, (_, g, n, k) in enumerate(trace):
        assert got[rid].size == n
        st_g = states.setdefault(g, O.seed_state(seeds[g], params[g].mexp))
        if k == 3:
            z = got[rid].view(np.float32).astype(np.float64)
            assert np.abs(z - O.normals(params[g], st_g, n)).max() <= 1.5e-5, f"rid={rid}"
        else:
            np.testing.assert_array_equal(got[rid], O.generate(params[g], st_g, n, k), err_msg=f"rid={rid} g={g}")
    for g, st_g in states.items():
        words, consumed = b.get_state(g)
        np.testing.assert_array_equal(words, st_g, err_msg=f"end state g={g}")
        assert consumed == sum(n for (_, gg, n, _) in trace if gg == g)
    # the same generators alone: one long request each, served by a fresh server
    b2 = mtgp.Batch(params, seeds)
    b2.prepare_split([0, 41, 60])
    srv2 = serve.NativeServer(b2, arena_bytes=16 << 20, chunk=chunk, depth=2, split=(1 << 16, 8, 2, 4))
    got2 = {}
    alone = [(0.0, 0, 333_334, 0), (0.0, 41, 300_000, 1), (0.0, 60, 250_000, 2)]
    srv2.run(alone, realtime=False, on_complete=lambda rid, out: got2.__setitem__(rid, bits(out)))
    srv2.close()
    for rid, (_, g, n, k) in enumerate(alone):
        np.testing.assert_array_equal(got2[rid], O.generate(params[g], O.seed_state(seeds[g], params[g].mexp), n, k),
                                      err_msg=f"alone g={g}")
    b2.close()
    b.close()
