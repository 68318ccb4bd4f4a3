"""Serving loop on the CPU: the scheduler driven by an executor that computes
each chunk with the oracle (no GPU). Checks admission by footprint, FIFO per
generator, continuous batching, exact results, and failure handling."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1005_4973_amd import inputs as I
from paper_1005_4973_amd.serve import Executor, Server


class OracleExecutor(Executor):
    """Chunks run immediately on the CPU oracle, advancing each generator's
    oracle state in launch order; a handle turns ready after `delay` polls."""

    def __init__(self, params, seeds, delay=0, fail_on=None):
        self.params = params
        self.states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
        self.delay = delay
        self.fail_on = fail_on
        self.launches = 0
        self.ticks = []

    def alloc(self, req):
        req.out = np.zeros(req.n, dtype=np.uint32)

    def launch(self, chunks):
        self.launches += 1
        if self.fail_on is not None and self.launches == self.fail_on:
            raise RuntimeError("injected launch failure")
        gens = [c[0] for c in chunks]
        assert len(gens) == len(set(gens)), "a generator appears twice in one tick"
        for gen, kind, n, out, off in chunks:
            out[off:off + n] = O.generate(self.params[gen], self.states[gen], n, kind)
        self.ticks.append(len(chunks))
        return [self.delay]

    def ready(self, handle):
        if handle[0] <= 0:
            return True
        handle[0] -= 1
        return False

    def wait(self, handle):
        handle[0] = 0


def reference_outputs(params, seeds, trace):
    """Each request's expected words: per generator, in arrival order."""
    states = {g: O.seed_state(seeds[g], params[g].mexp) for g in range(len(params))}
    return [O.generate(params[g], states[g], n, k) for (_, g, n, k) in trace]


def small_setup(num_gens=24, num_reqs=120, seed=3):
    params = I.draw_param_sets([89, 521, 11213] * (num_gens // 3), 700 + seed, I.M_POLICY_FULL)
    seeds = I.state_seeds(len(params))
    trace = I.serving_trace(num_reqs, rate_per_s=1e6, num_gens=len(params), seed=seed,
                            median_log2=9, sigma=1.0, lo_log2=3, hi_log2=13)
    return params, seeds, trace


def test_results_exact_and_fifo():
    params, seeds, trace = small_setup()
    ex = OracleExecutor(params, seeds, delay=2)
    srv = Server(ex, mem_budget_bytes=1 << 20, chunk=1000, depth=2)
    st = srv.run(trace, realtime=False)
    assert st.completed == len(trace) and st.rejected == 0
    refs = reference_outputs(params, seeds, trace)
    byid = {r.rid: r for r in srv.completed}
    for i, ref in enumerate(refs):
        np.testing.assert_array_equal(byid[i].out, ref)
    # per generator, requests complete in arrival order
    for g in range(len(params)):
        done = [r for r in srv.completed if r.gen == g]
        assert [r.rid for r in sorted(done, key=lambda r: r.t_done)] == sorted(r.rid for r in done)
    # continuous batching: some ticks carry several generators
    assert max(ex.ticks) > 1


def test_same_alone_and_in_the_mix():
    params, seeds, trace = small_setup(seed=5)
    ex = OracleExecutor(params, seeds, delay=1)
    mixed = Server(ex, mem_budget_bytes=1 << 20, chunk=700)
    mixed.run(trace, realtime=False)
    got = {r.rid: r.out for r in mixed.completed}
    for g in (0, 7, 13):
        sub = [(i, t) for i, t in enumerate(trace) if t[1] == g]
        ex1 = OracleExecutor(params, seeds)
        alone = Server(ex1, mem_budget_bytes=1 << 20, chunk=700)
        alone.run([t for _, t in sub], realtime=False)
        for (i, _), r in zip(sub, sorted(alone.completed, key=lambda r: r.rid)):
            np.testing.assert_array_equal(r.out, got[i])


def test_admission_respects_budget_and_rejects_oversize():
    params, seeds, trace = small_setup(seed=9)
    budget = 40000                      # bytes: a few requests at a time
    ex = OracleExecutor(params, seeds, delay=1)
    srv = Server(ex, mem_budget_bytes=budget, chunk=500)
    peak = [0]
    orig = srv._admit

    def watch(now):
        orig(now)
        peak[0] = max(peak[0], srv.in_use)
        assert srv.in_use <= budget

    srv._admit = watch
    st = srv.run(trace, realtime=False)
    big = [r for r in trace if 4 * r[2] > budget]
    assert st.rejected == len(big)
    assert st.completed == len(trace) - len(big)
    assert 0 < peak[0] <= budget


def test_launch_failure_commits_nothing():
    params, seeds, trace = small_setup(seed=11)
    ex = OracleExecutor(params, seeds, fail_on=3)
    srv = Server(ex, mem_budget_bytes=1 << 20, chunk=600)
    with pytest.raises(RuntimeError):
        srv.run(trace, realtime=False)
    # the failed tick advanced neither the requests nor the generators' streams
    assert all(r.done == r.finished or r.done - r.finished <= 600 for q in srv.active.values() for r in q)
    ex.fail_on = None
    srv.run([], realtime=False)         # finish what was admitted
    refs = reference_outputs(params, seeds, trace)
    admitted = {r.rid: r for r in srv.completed}
    assert admitted, "nothing completed after recovery"
    for rid, r in admitted.items():
        np.testing.assert_array_equal(r.out, refs[rid])


def test_realtime_latencies_are_recorded():
    params, seeds, trace = small_setup(num_reqs=30, seed=13)
    trace = [(t * 1e-4, g, n, k) for (t, g, n, k) in [(i, *x[1:]) for i, x in enumerate(trace)]]
    ex = OracleExecutor(params, seeds)
    srv = Server(ex, mem_budget_bytes=1 << 20, chunk=1 << 12)
    st = srv.run(trace, realtime=True)
    d = st.as_dict()
    assert st.completed == len(trace)
    assert d["p50_ms"] >= 0 and d["p99_ms"] >= d["p50_ms"] and not math.isnan(d["p99_ms"])
