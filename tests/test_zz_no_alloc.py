"""The allocation-free batch call (mtgp_batch_generate_static) against the
ordinary one (mtgp_batch_generate), through the C ABI: two identical batches
receive the same requests, one through each entry point, in two calls in a
row (the second smaller), and every output word and end state must match
bit for bit, in the automatic launch shape and in the chunked form."""
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
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1005_4973_amd import mtgp
    mtgp.lib()
    return mtgp


def bits(t):
    import torch
    return t.view(torch.int32).cpu().numpy().view(np.uint32)


def calls(rng, G, count, nmax):
    gens = list(range(G))
    out = []
    for g in gens[:count]:
        kind = rng.uniform_int(0, 3)
        n = rng.uniform_int(1, nmax)
        if kind == 3:
            n += n & 1          # normals come in pairs
        out.append((g, kind, n))
    return out


@pytest.mark.parametrize("shape", [None, (2, 256, 2, 0, 0)])
def test_static_call_matches_ordinary_call(M, shape):
    import torch
    params = I.draw_param_sets([11213] * 24 + [23209] * 8 + [44497] * 8, 123)
    seeds = I.state_seeds(len(params))
    a = M.Batch(params, seeds)          # allocation-free entry point
    b = M.Batch(params, seeds)          # ordinary entry point
    if shape is not None:
        a.set_launch(*shape)
        b.set_launch(*shape)
    rng = I.SplitMix64(7)
    for step, (count, nmax) in enumerate(((40, 300000), (13, 5000))):
        reqs = calls(rng, len(params), count, nmax)
        say(f"shape {shape} call {step}: {len(reqs)} requests, up to {nmax} outputs")
        out_a = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
        out_b = [torch.empty(n, dtype=torch.int32, device="cuda") for (_, _, n) in reqs]
        a.generate_static([(g, k, n, o) for (g, k, n), o in zip(reqs, out_a)])
        b.generate([(g, k, n, o) for (g, k, n), o in zip(reqs, out_b)])
        torch.cuda.synchronize()
        for (g, k, n), x, y in zip(reqs, out_a, out_b):
            np.testing.assert_array_equal(bits(x), bits(y), err_msg=f"call {step} gen {g} kind {k} n {n}")
    for g in range(len(params)):
        wa, ca = a.get_state(g)
        wb, cb = b.get_state(g)
        np.testing.assert_array_equal(wa, wb)
        assert ca == cb
    # and the first generator's stream is the oracle's
    st = O.seed_state(seeds[0], params[0].mexp)
    t = torch.empty(1000, dtype=torch.int32, device="cuda")
    a.generate_static([(0, 0, 1000, t)])
    torch.cuda.synchronize()
    O.advance(params[0], st, a.get_state(0)[1] - 1000)
    np.testing.assert_array_equal(bits(t), O.generate(params[0], st, 1000, 0))
    a.close()
    b.close()


def test_static_call_rejects(M):
    import torch
    params = I.draw_param_sets([11213] * 2, 5)
    a = M.Batch(params, I.state_seeds(2))
    t = torch.empty(64, dtype=torch.int32, device="cuda")
    with pytest.raises(M.MTGPError):
        a.generate_static([(0, 0, 64, t), (0, 1, 64, t)])       # one generator twice
    with pytest.raises(M.MTGPError):
        a.generate_static([(0, 0, 1, t)] * 4097)                 # beyond the item limit (checked first)
    a.generate_static([])                                        # nothing to do
    a.close()
