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
