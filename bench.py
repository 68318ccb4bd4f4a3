"""Throughput benchmark of the MTGP HIP path on one MI355X.

Headline step (`value`): the batched uneven workload -- 4096 generators with
distinct seeded parameter sets, periods 2^11213-1, 2^23209-1, 2^44497-1 in
ratio 2:1:1, request lengths log-uniform in [2^10, 2^24] (7.16e9 numbers,
28.6 GB), 50 % uint32 and 25 % each float kind -- as one replay of a
HIP-graph-captured plan. The plan's launch shape and jump-ahead split limit
are autotuned once, before the timed region. A replay first computes the
start states of the long requests' segments (a raw-word prefix and the jump
correlations: the prepare phase), then runs the persistent generation
kernel over all requests and segments: each state is loaded into LDS, the
recursion runs with tempering and conversion, outputs leave with coalesced
stores, and each generator's end state is stored back. `value` counts every
number of the replay over the whole replay (both phases); `roofline` is the
generation kernel's algorithmic bytes over its own average duration, with
the end-to-end fraction beside it.

The same JSON line also reports:
  independent_128   128 MTGP-11213 generators, 2^22 outputs each as uint32,
                    float32 [1,2) and float32 [0,1) (three tuned plans)
  batched_plain     the headline workload as one launch per request (the
                    paper's one block per generator, run in sequence), and
                    the critical path of the tuned plan
  large_states      256 generators at p = 23209 and at p = 44497, 2^24 uint32 each
  large_states_wide_m  the p = 23209 batch with M uniform in [2, N-2]
  normals           the 128 generators, 2^22 Box-Muller normals each (float32)
  param_search      host-side search for full-period parameter sets (p = 4423,
                    11213, 23209) and the dimension of equidistribution k(v),
                    Delta of found sets
  single_stream     one MTGP-11213 generator, 2^20 uint32 per eager call, unsplit
                    and split into jump-ahead segments
  serving           65536 resident MTGP-11213 states behind the library's native
                    request loop: open-loop Poisson arrivals at swept rates,
                    log-normal sizes (median 2^16, sigma 1.5, clipped to
                    [2^10, 2^26]): p50/p99 latency and sustained numbers/s
`value` is numbers/s with states and parameters resident in HBM when the
timed region starts. The sections time a launch or replay with HIP events:
the median of 10 after 3 untimed ones (the plain one-launch-per-request
baseline runs once, by wall clock).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SECTIONS = ("batched_plain", "independent_128", "large_states", "large_states_wide_m", "normals", "single_stream",
            "serving", "param_search")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (default: host cores, max 16)")
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma-separated extra sections to run (empty for the headline only)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def gbs(nbytes, seconds):
    return nbytes / seconds / 1e9


def roof(nbytes, seconds):
    a = gbs(nbytes, seconds)
    return {"GBs": round(a, 1), "frac_of_8TBs": round(a / HBM_PEAK_GBS, 4)}


def cpu_baseline(params, reqs, threads, passes=8):
    """The oracle on the host cores: the headline workload's requests (every
    generator, its requested length and kind), `passes` times over, one
    request per task on `threads` threads; plus single-core rates for the
    three periods and the pure-Python matrix-form reading on a small sample."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_1005_4973_amd import inputs as I

    states = {r.gen: O.seed_state(I.STATE_SEED_BASE + r.gen, params[r.gen].mexp) for r in reqs}

    def run(r):
        O.generate(params[r.gen], states[r.gen], r.n, r.kind)
        return r.n

    order = sorted(reqs, key=lambda r: -r.n)   # longest first, as the GPU queue
    t0 = time.perf_counter()
    total = 0
    done_passes = 0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        # whole passes until about 10 s of work (at most `passes`)
        while done_passes < passes and (done_passes == 0 or time.perf_counter() - t0 < 10.0):
            total += sum(ex.map(run, order))
            done_passes += 1
    dt = time.perf_counter() - t0
    passes = done_passes
    single = {}
    for mexp in (11213, 23209, 44497):
        ps = I.draw_param_sets([mexp], 7000 + mexp % 97)[0]
        st = O.seed_state(1, mexp)
        m = 1 << 24
        t1 = time.perf_counter()
        O.generate(ps, st, m, O.U32)
        single[f"p{mexp}"] = round(m / (time.perf_counter() - t1) / 1e6, 1)
    # the second reading (matrix form, pure Python) on the single-stream set:
    # a 2^16-output sample, and what the whole 2^20-output stream would take
    from oracle import pyref as P
    (ps1,), n1 = I.single_stream()
    m = 1 << 16
    t1 = time.perf_counter()
    P.generate(ps1, list(O.seed_state(I.STATE_SEED_BASE, ps1.mexp)), m, O.U32)
    py_s = time.perf_counter() - t1
    return {"value": round(total / dt / 1e9, 4), "unit": "G numbers/s", "cores": threads, "kind": "oracle",
            "host_cpus_visible": len(os.sched_getaffinity(0)),
            "sample": f"the headline workload's {len(reqs)} requests (all lengths and kinds) x {passes} passes "
                      f"({total} numbers, {dt:.2f} s wall on {threads} threads)",
            "single_core_M_numbers_s": single,
            "matrix_form_python": {"numbers_s": round(m / py_s, 1), "sample": f"{m} outputs of the single stream",
                                   "single_stream_s": round(n1 / (m / py_s), 1)}}


# committed counter summaries (profiles/*_traffic.md) per workload; a
# launch's traffic is taken from the one recorded with the same kernel
# sources, split limit and resolved launch
TRAFFIC_HEADLINE = "batched_uneven_4096"
TRAFFIC_128 = "independent_128x4M"
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1005_4973_amd", "csrc", f) for f in ("mtgp_kernels.hip", "mtgp_internal.h")]


def launch_of(info):
    """The resolved generation launch of a plan (mtgp_plan_describe) as the
    fields a counter summary records."""
    return {k: info[k] for k in ("mode", "threads", "spl", "lds_words", "grid")}


def launch_str(launch):
    return " ".join(f"{k}={launch[k]}" for k in ("mode", "threads", "spl", "lds_words", "grid"))


def measured_traffic(launch, split_rounds, workload):
    """HBM bytes per launch of a generation kernel from the committed counter
    summaries of a workload (profiles/*_<workload>_traffic.md, or one given
    path), or None when none of them was taken with the same kernel sources,
    split limit (which sets the segments) and resolved launch."""
    import glob
    paths = [workload] if os.path.isfile(workload) else \
        sorted(glob.glob(os.path.join(ROOT, "profiles", f"*_{workload}_traffic.md")))
    for path in paths:
        t = _traffic_of(path, launch, split_rounds)
        if t is not None:
            return t
    return None


def _traffic_of(path, launch, split_rounds):
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("kernel_source_sha256_16:", "traffic_bytes_per_launch:", "split_rounds:",
                                      "launch:")))
    if fields.get("kernel_source_sha256_16", "").split()[0:1] != [h.hexdigest()[:16]]:
        return None
    if fields.get("split_rounds", "").strip() != str(split_rounds):
        return None
    if fields.get("launch", "").strip() != launch_str(launch):
        return None
    return int(fields["traffic_bytes_per_launch"].strip())


def kernel_name(launch):
    """The generation kernel a plan launches (for the roofline line)."""
    mode = launch["mode"]
    if (mode & 3) == 2:
        return "mtgp_chunk_kernel<{}, {}, 1>".format(launch["lds_words"], launch["spl"])
    return "mtgp_kernel<{}, {}>".format("true" if mode & 1 else "false", "true" if mode & 4 else "false")


def store_ceilings(torch, outs, ns, launch, fill=None):
    """Write ceilings of a plan's output layout: the store-only probe over the
    plan's own work items in queue order, on as many wavefronts as the launch
    runs items at once, with 4-byte plain stores (the generation kernels'
    pattern), 4-byte nontemporal and 16-byte plain stores; and a torch fill
    of the output buffer when given. GB/s of output bytes."""
    from paper_1005_4973_amd import probe
    units = launch["threads"] // 64 if launch["mode"] & 3 else 1
    waves = launch["grid"] * units
    nbytes = 4 * int(sum(int(v) for v in ns))
    res = {"waves": waves}
    for key, width, nt in (("probe_4B_plain", 1, False), ("probe_4B_nontemporal", 1, True),
                           ("probe_16B_plain", 4, False)):
        ms = probe.store_ms(outs, ns, waves, width, nt, reps=3)
        res[key] = round(nbytes / ms / 1e6, 1)
    if fill is not None:
        fill_ms = timed_ms(torch, lambda: fill.fill_(7), reps=5, warmup=1)
        res["torch_fill"] = round(4 * fill.numel() / fill_ms / 1e6, 1)
    return res


def phase_times(torch, plan, mtgp, stream, reps, warmup):
    """Replays of a plan as its two phases with HIP events on `stream` around
    each: per replay (prepare ms, generate ms), after `warmup` untimed
    replays. A GPU spin runs ahead of the timed replays, so that the host has
    queued them all before the first starts: an interval then holds the
    phase's kernels and no wait for the host's next submission. Untimed
    replays queued behind the spin run right before the timed ones, so the
    timed ones follow busy work, not the idle spin."""
    for _ in range(warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(reps)]
    with torch.cuda.stream(stream):
        torch.cuda._sleep(int(20e6))
    for _ in range(max(warmup, 10)):
        plan.launch(stream)
    for e in ev:
        e[0].record(stream)
        plan.launch_phase(mtgp.PHASE_PREPARE, stream)
        e[1].record(stream)
        plan.launch_phase(mtgp.PHASE_GENERATE, stream)
        e[2].record(stream)
    torch.cuda.synchronize()
    return [(a.elapsed_time(b), b.elapsed_time(c)) for a, b, c in ev]


def timed_steps(torch, plan, stream, steps, warmup):
    """Wall time of `steps` whole replays (mtgp_plan_launch, one graph launch
    each) after `warmup` untimed ones, with a device synchronisation on both
    sides of the timed region."""
    for _ in range(warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.launch(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def median(v):
    v = sorted(v)
    k = len(v) // 2
    return v[k] if len(v) % 2 else 0.5 * (v[k - 1] + v[k])


def roofline_block(alg_bytes, gen_ms, step_ms, launch, traffic, ceilings=None):
    """`roofline` object for a generation kernel: algorithmic bytes per launch
    over its average launch time, against the 8 TB/s HBM peak; the whole
    replay (prepare and generate) beside it, and the store-only ceilings of
    the same output layout when measured."""
    achieved = alg_bytes / (gen_ms / 1e3) / 1e9
    blk = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel_name(launch),
           "launch": launch, "avg_launch_ms": round(gen_ms, 4), "alg_bytes_per_launch": alg_bytes,
           "end_to_end": {"ms_per_replay": round(step_ms, 4),
                          "GBs": round(alg_bytes / (step_ms / 1e3) / 1e9, 1),
                          "frac": round(alg_bytes / (step_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}}
    if ceilings:
        blk["store_ceilings_GBs"] = ceilings
        blk["frac_of_store_ceiling"] = round(achieved / ceilings["probe_4B_plain"], 4)
    return blk


def timed_ms(torch, fn, reps=10, warmup=3):
    """Median over `reps` event-timed calls after `warmup` untimed ones."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    mid = len(times) // 2
    return times[mid] if len(times) % 2 else 0.5 * (times[mid - 1] + times[mid])


# ---------------------------------------------------------------------------
# headline: the batched uneven workload
# ---------------------------------------------------------------------------

def workload_bytes(params, reqs):
    """Algorithmic bytes of one launch over these requests: 4 per output, the
    state in and out (8N) and the 256-byte parameter record per request."""
    return sum(4 * r.n + 8 * state_words(params[r.gen].mexp) + 256 for r in reqs)


def headline(args, torch, I, mtgp, ctx):
    params, reqs = I.batched_uneven()
    G = len(params)
    tot = sum(r.n for r in reqs)
    batch = mtgp.Batch(params, I.state_seeds(G))
    out = torch.empty(tot, dtype=torch.int32, device="cuda")
    base = out.data_ptr()
    stream = torch.cuda.current_stream()
    rq = [(r.gen, r.kind, r.n, base + 4 * r.offset) for r in reqs]
    t0 = time.perf_counter()
    # launch shape and jump-ahead split limit (outputs are identical under
    # every choice; states are left untouched)
    tuning = batch.autotune(rq, reps=2, stream=stream)
    tune_s = time.perf_counter() - t0
    log(f"autotune: {tuning} in {tune_s:.1f} s")
    plan = batch.plan(rq)
    launch = launch_of(plan.describe())
    outs, ns = plan.items()
    wall = timed_steps(torch, plan, stream, args.steps, args.warmup)
    times = phase_times(torch, plan, mtgp, stream, args.steps, 1)
    plan.close()
    prep = sum(t[0] for t in times) / len(times)
    gen = sum(t[1] for t in times) / len(times)
    ceilings = store_ceilings(torch, outs, ns, launch, fill=out)
    alg = workload_bytes(params, reqs)
    ctx.update(params=params, reqs=reqs, batch=batch, out=out, tuning=tuning, launch=launch)
    return {
        "value": round(tot * args.steps / wall / 1e9, 3),
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "config": {"workload": "4096 generators, exponents 11213:23209:44497 in ratio 2:1:1 (distinct seeded "
                               "parameter sets, paper M rule), request lengths log-uniform in [2^10, 2^24], "
                               "kinds 50% uint32 / 25% float32 [1,2) / 25% float32 [0,1); one graph-captured "
                               "plan replay per step (jump-ahead segment states, then one persistent "
                               "generation launch)",
                   "generators": G, "numbers_per_step": tot, "bytes_per_step": 4 * tot,
                   "autotuned": tuning, "autotune_s": round(tune_s, 1)},
        "roofline": {**roofline_block(alg, gen, wall / args.steps * 1e3, launch,
                                      measured_traffic(launch, tuning["split_rounds"], TRAFFIC_HEADLINE), ceilings),
                     "avg_prepare_ms": round(prep, 4)},
    }


# ---------------------------------------------------------------------------
# extra sections
# ---------------------------------------------------------------------------

def independent_128(torch, I, mtgp, ctx):
    """128 MTGP-11213 generators x 2^22 outputs as uint32, float32 [1,2) and
    float32 [0,1): one tuned plan per kind, each replayed as its two phases."""
    params, n = I.independent_128()
    G = len(params)
    kinds = (I.KIND_U32, I.KIND_F12, I.KIND_F01)
    batch = mtgp.Batch(params, I.state_seeds(G))
    out = torch.empty(G * n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    reqs = {k: [(g, k, n, out.data_ptr() + 4 * g * n) for g in range(G)] for k in kinds}
    tuning = batch.autotune(reqs[I.KIND_U32], reps=3, stream=stream)
    res = {"generators": G, "mexp": 11213, "outputs_per_generator": n, "autotuned": tuning, "kinds": {}}
    alg = G * (4 * n + 8 * 351 + 256)
    steps = []
    for k, name in zip(kinds, ("uint32", "float32_1to2", "float32_0to1")):
        plan = batch.plan(reqs[k])
        launch = launch_of(plan.describe())
        outs, ns = plan.items()
        times = phase_times(torch, plan, mtgp, stream, 10, 3)
        plan.close()
        step = median([a + b for a, b in times])
        gen = median([b for a, b in times])
        steps.append(step)
        ceilings = store_ceilings(torch, outs, ns, launch) if k == I.KIND_U32 else None
        res["kinds"][name] = {"ms": round(step, 4), "G_numbers_s": round(G * n / step / 1e6, 2),
                              "roofline": {**roofline_block(alg, gen, step, launch,
                                                            measured_traffic(launch, tuning["split_rounds"],
                                                                             TRAFFIC_128)
                                                            if k == I.KIND_U32 else None, ceilings),
                                           "avg_prepare_ms": round(median([a for a, b in times]), 4)}}
    res["G_numbers_s_three_kinds"] = round(3 * G * n / sum(steps) / 1e6, 2)
    batch.close()
    del out
    torch.cuda.empty_cache()
    return res


def batched_plain(torch, I, mtgp, ctx):
    """The headline workload as one launch per request on one stream (one
    workgroup per generator, as the paper runs one block per generator), and
    the critical path of the tuned plan: its longest segment timed alone."""
    params, reqs, batch, out, tuning, launch = (ctx[k] for k in ("params", "reqs", "batch", "out", "tuning",
                                                                  "launch"))
    tot = sum(r.n for r in reqs)
    base = out.data_ptr()
    rq = [(r.gen, r.kind, r.n, base + 4 * r.offset) for r in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.generate_plain(rq)
    torch.cuda.synchronize()
    ms_p = (time.perf_counter() - t0) * 1e3
    # critical path: the segment with the most rounds under the tuned shape
    # and split limit, timed alone (same shape, no split)
    r_max, crit = 0, None
    for r in reqs:
        ps = params[r.gen]
        W = round_width(state_words(ps.mexp), ps.pos, launch)
        rounds = -(-r.n // W)
        S = -(-rounds // tuning["split_rounds"]) if tuning["split_rounds"] else 1
        J = -(-r.n // S)
        if -(-J // W) > r_max:
            r_max, crit = -(-J // W), (r, J)
    split = tuning["split_rounds"]
    batch.set_split(0)
    (r, J) = crit
    p1 = batch.plan([(r.gen, r.kind, J, base + 4 * r.offset)])
    ms_c = timed_ms(torch, lambda: p1.launch())
    p1.close()
    batch.set_split(split)
    head_ms = ctx.get("head_ms")
    return {"numbers": tot,
            "plain_one_launch_per_request": {"ms": round(ms_p, 1), "G_numbers_s": round(tot / ms_p / 1e6, 3)},
            "speedup_batched_vs_plain": round(ms_p / head_ms, 1) if head_ms else None,
            "critical_path": {"segment_rounds": r_max, "mexp": params[crit[0].gen].mexp, "segment_outputs": crit[1],
                              "alone_ms": round(ms_c, 3),
                              "makespan_over_bound": round(head_ms / ms_c, 2) if head_ms else None}}


def state_words(mexp):
    return (mexp + 31) // 32


def round_width(N, M, launch):
    """Steps a round of this generator computes under a resolved launch shape
    (mtgp_plan_describe): W = min(N - M, lanes * s), s the largest steps per
    lane allowed by the shape with lanes * s <= N - M (the library's own
    rule); a chunk of 64 steps in the chunked form."""
    mode = launch["mode"]
    if mode < 0:
        raise ValueError("round_width needs a resolved launch shape")
    if (mode & 3) == 2:
        return 64
    wave, threads, cap = bool(mode & 1), launch["threads"], launch["spl"]
    lanes = 64 if wave else threads
    cands = (16, 12, 8, 6, 4, 2, 1) if wave else (4, 2, 1)
    s = next((c for c in cands if c <= cap and lanes * c <= N - M), 1)
    return min(N - M, lanes * s)


def large_states(torch, I, mtgp, ctx):
    res = {}
    stream = torch.cuda.current_stream()
    for mexp, N in ((23209, 726), (44497, 1391)):
        params, n = I.large_states(mexp)
        G = len(params)
        batch = mtgp.Batch(params, I.state_seeds(G))
        out = torch.empty(G * n, dtype=torch.int32, device="cuda")
        rq = [(g, 0, n, out.data_ptr() + 4 * g * n) for g in range(G)]
        t0 = time.perf_counter()
        tuning = batch.autotune(rq, reps=2, stream=stream)
        tune_s = time.perf_counter() - t0
        plan = batch.plan(rq)
        launch = launch_of(plan.describe())
        outs, ns = plan.items()
        times = phase_times(torch, plan, mtgp, stream, 10, 3)
        plan.close()
        ceilings = store_ceilings(torch, outs, ns, launch)
        batch.close()
        del out
        torch.cuda.empty_cache()
        step = median([a + b for a, b in times])
        gen = median([b for a, b in times])
        alg = G * (4 * n + 8 * N + 256)
        res[f"p{mexp}"] = {"generators": G, "numbers": G * n, "ms": round(step, 3),
                           "G_numbers_s": round(G * n / step / 1e6, 2), **roof(alg, step / 1e3),
                           "roofline": {**roofline_block(alg, gen, step, launch,
                                                         measured_traffic(launch, tuning["split_rounds"],
                                                                          f"large_states_{mexp}"), ceilings),
                                        "avg_prepare_ms": round(median([a for a, b in times]), 4)},
                           "autotuned": tuning, "autotune_s": round(tune_s, 1)}
    return res


def large_states_wide_m(torch, I, mtgp, ctx):
    """Sensitivity of the large-state batch to the M rule: 256 MTGP-23209
    generators x 2^24 with M uniform in [2, N-2]. The generators with small
    N - M have millions of dependent rounds; the tuned plan splits them into
    jump-ahead segments. Reported with the segment that bounds the makespan."""
    params, n = I.large_states_wide_m(23209)
    G, N = len(params), 726
    batch = mtgp.Batch(params, I.state_seeds(G))
    out = torch.empty(G * n, dtype=torch.int32, device="cuda")
    rq = [(g, 0, n, out.data_ptr() + 4 * g * n) for g in range(G)]
    t0 = time.perf_counter()
    tuning = batch.autotune(rq, reps=1)
    tune_s = time.perf_counter() - t0
    plan = batch.plan(rq)
    launch = launch_of(plan.describe())
    ms = timed_ms(torch, lambda: plan.launch(), reps=5, warmup=1)
    plan.close()
    widths = [round_width(N, ps.pos, launch) for ps in params]
    rounds = [-(-n // w) for w in widths]
    S = [-(-r // tuning["split_rounds"]) if tuning["split_rounds"] else 1 for r in rounds]
    seg_len = [-(-n // s) for s in S]
    seg_rounds = [-(-j // w) for j, w in zip(seg_len, widths)]
    batch.close()
    del out
    torch.cuda.empty_cache()
    alg = G * (4 * n + 8 * N + 256)
    return {"generators": G, "numbers": G * n, "M_rule": "uniform in [2, N-2]", "min_N_minus_M": min(N - p.pos for p in params),
            "ms": round(ms, 3), "G_numbers_s": round(G * n / ms / 1e6, 2), **roof(alg, ms / 1e3),
            "segments": sum(S), "max_segment_rounds": max(seg_rounds), "unsplit_max_rounds": max(rounds),
            "autotuned": tuning, "autotune_s": round(tune_s, 1)}


def normals(torch, I, mtgp, ctx):
    """128 MTGP-11213 generators x 2^22 Gaussian deviates (Box-Muller on pairs of
    float [1,2) outputs), one tuned split plan replayed."""
    params, n = I.independent_128()
    G = len(params)
    batch = mtgp.Batch(params, I.state_seeds(G))
    out = torch.empty(G * n, dtype=torch.int32, device="cuda")
    rq = [(g, mtgp.KIND_NORMAL_FLOAT32, n, out.data_ptr() + 4 * g * n) for g in range(G)]
    tuning = batch.autotune(rq, reps=2)
    plan = batch.plan(rq)
    ms = timed_ms(torch, lambda: plan.launch())
    plan.close()
    batch.close()
    del out
    torch.cuda.empty_cache()
    alg = G * (4 * n + 8 * 351 + 256)
    return {"generators": G, "numbers": G * n, "ms": round(ms, 3), "G_normals_s": round(G * n / ms / 1e6, 2),
            **roof(alg, ms / 1e3), "autotuned": tuning}


def param_search(torch, I, mtgp, ctx):
    """Host-side recursion-parameter search (section 5): full-period sets with
    an ID embedded, seeded so the draw counts are fixed, at p = 4423, 11213
    and 23209; the paper's own search took 338 s per MTGP-11213 set on
    average (context only). Then the dimension of equidistribution k(v) and
    Delta (section 3.4) of the 11213 and 23209 sets, tempered and not. The
    paper's table for its released MTGP-23209 set gives Delta = 1141 after
    its tempering-parameter search; the sets here keep a random tempering
    matrix (that search is not done), so the figures are context, not a
    comparison."""
    threads = min(16, len(os.sched_getaffinity(0)))
    runs = []
    found = {}
    for mexp, ident in ((4423, 1), (11213, 1), (11213, 4)):
        ps, st = mtgp.search_params(mexp, id=ident, seed=mexp, threads=threads)
        runs.append({"mexp": mexp, "id": ident, "draws": st["draws"], "evaluated": st["evaluated"],
                     "seconds": st["seconds"]})
        found[(mexp, ident)] = ps
        log(f"param_search: p={mexp} id={ident}: {runs[-1]}")
    # p = 23209: the seeded search accepts draw 40901 (about 20 ms of one
    # core per candidate, most of it Berlekamp-Massey over 46k bits; about
    # 20 s on 16 cores); the draw limit only bounds the run.
    budget = 200000
    log("param_search: p=23209 search started")
    t0 = time.perf_counter()
    try:
        ps, st = mtgp.search_params(23209, id=1, seed=23209, max_draws=budget, threads=threads)
        runs.append({"mexp": 23209, "id": 1, "draws": st["draws"], "evaluated": st["evaluated"],
                     "full_degree": st["full_degree"], "sieve_passed": st["sieve_passed"],
                     "seconds": st["seconds"]})
        found[(23209, 1)] = ps
    except mtgp.MTGPError:
        runs.append({"mexp": 23209, "id": 1, "found": False, "draw_limit": budget,
                     "seconds": round(time.perf_counter() - t0, 1)})
    log(f"param_search: p=23209 id=1: {runs[-1]}")
    # dimension of equidistribution of the found sets: one core, host only
    equi = []
    for mexp in (11213, 23209):
        if (mexp, 1) not in found:
            continue
        ps = found[(mexp, 1)]
        e = {"mexp": mexp, "id": 1, "M": ps.pos, "sh1": ps.sh1, "sh2": ps.sh2}
        for name, tempered in (("tempered", True), ("untempered", False)):
            t0 = time.perf_counter()
            k, delta = mtgp.equidistribution(ps, tempered=tempered)
            e[name] = {"delta": delta, "k_min": min(k), "k": list(k), "seconds": round(time.perf_counter() - t0, 2)}
        if mexp == 23209:
            e["paper_table_delta_released_set"] = 1141
        equi.append(e)
        log(f"param_search: equidistribution p={mexp}: tempered delta {e['tempered']['delta']}, "
            f"untempered delta {e['untempered']['delta']}")
    return {"threads": threads, "runs": runs, "equidistribution": equi}


def param_search_44497(torch, I, mtgp, ctx):
    """Opt-in (minutes of host time, not in the default sections): the
    recursion-parameter search at p = 44497 with ID 1, the largest released
    size, then k(v) and Delta of the set found. The search runs as seeded
    rounds of a fixed number of draws (seed 44497 + round), so each round
    reports when it ends and the set found is fixed by the round schedule."""
    threads = min(16, len(os.sched_getaffinity(0)))
    per_round = 4000
    rounds = []
    t0 = time.perf_counter()
    ps = None
    for r in range(64):
        try:
            ps, st = mtgp.search_params(44497, id=1, seed=44497 + r, max_draws=per_round, threads=threads)
        except mtgp.MTGPError:
            rounds.append({"round": r, "found": False})
            log(f"param_search_44497: round {r} ({per_round} draws) found none, "
                f"{time.perf_counter() - t0:.0f} s")
            continue
        rounds.append({"round": r, "found": True, **st})
        log(f"param_search_44497: round {r} found a set: {st}")
        break
    res = {"threads": threads, "draws_per_round": per_round, "rounds": len(rounds),
           "seconds": round(time.perf_counter() - t0, 1), "last_round": rounds[-1]}
    if ps is None:
        return res
    res["set"] = {"M": ps.pos, "sh1": ps.sh1, "sh2": ps.sh2, "param_tbl": list(ps.param_tbl),
                  "temper_tbl": list(ps.temper_tbl)}
    for name, tempered in (("tempered", True), ("untempered", False)):
        t1 = time.perf_counter()
        k, delta = mtgp.equidistribution(ps, tempered=tempered)
        res[name] = {"delta": delta, "k_min": min(k), "k": list(k), "seconds": round(time.perf_counter() - t1, 2)}
        log(f"param_search_44497: {name} delta {delta}")
    return res


def single_stream(torch, I, mtgp, ctx):
    """One generator, 2^20 uint32 per eager call: as one workgroup (the
    recursion's rounds in sequence), and split into jump-ahead segments (the
    first split call finds the orbit's annihilator and the jump polynomials;
    the timed calls reuse them)."""
    (ps,), n = I.single_stream()
    g = mtgp.Generator(ps, 1234)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    ms = timed_ms(torch, lambda: g.generate(n, I.KIND_U32, out=out))
    g.set_split(16)
    t0 = time.perf_counter()
    g.generate(n, I.KIND_U32, out=out)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    ms_split = timed_ms(torch, lambda: g.generate(n, I.KIND_U32, out=out))
    g.close()
    return {"M": ps.pos, "numbers": n, "ms": round(ms, 4), "G_numbers_s": round(n / ms / 1e6, 3),
            "split_16_rounds": {"ms": round(ms_split, 4), "G_numbers_s": round(n / ms_split / 1e6, 3),
                                "first_call_s": round(first_s, 3)}}


def serving(torch, I, mtgp, ctx):
    """65536 resident MTGP-11213 states served by the library's request loop
    (mtgp_server_*: native admission and tick building; Python only releases
    arrivals on time and collects completions). Capacity: the completion
    rate of an open-loop burst offered well above it. Sweep: open-loop
    Poisson arrivals at fractions of that capacity, each point at least 2 s
    and 10^4 requests, log-normal sizes (median 2^16, sigma 1.5, clipped to
    [2^10, 2^26]): p50/p99 latency, sustained requests/s and numbers/s (and
    their share of 8 TB/s); the knee is the first load whose p99 is at least
    5x the p99 at load 0.1 (the sweep stops one point after it)."""
    from paper_1005_4973_amd import serve
    G = 65536
    params = I.serving_params(G)
    batch = mtgp.Batch(params, I.state_seeds(G))
    arena, chunk = 8 << 30, 1 << 18

    def native(trace, realtime=True):
        srv = serve.NativeServer(batch, arena_bytes=arena, chunk=chunk, depth=2)
        st = srv.run(trace, realtime=realtime)
        srv.close()
        return st

    def point(load, st, lam, num):
        return {"load": load, "offered_req_per_s": round(lam, 1), "requests": num, "completed": st.completed,
                "wall_s": round(st.wall_s, 3), "req_per_s": round(st.completed / st.wall_s, 1),
                "numbers_per_s": round(st.numbers / st.wall_s, 1),
                "frac_of_8TBs": round(4 * st.numbers / st.wall_s / 1e12 / 8.0, 4),
                "p50_ms": round(float(st.percentile(50)) * 1e3, 3), "p99_ms": round(float(st.percentile(99)) * 1e3, 3)}

    native(I.serving_trace_arrays(2000, 1e5, G, seed=5000), True)        # warm-up
    # capacity: an open-loop burst offered at 4M requests/s for 0.5 s
    burst = I.serving_trace_arrays(2_000_000, 4e6, G, seed=5001)
    st = native(burst, True)
    cap = st.completed / st.wall_s
    log(f"serving capacity estimate: {cap:.0f} requests/s ({st.numbers / st.wall_s / 1e9:.1f} G numbers/s)")
    points = []
    after_knee = 0
    for frac in (0.1, 0.25, 0.5, 0.75, 1.0, 1.15, 1.3, 1.5, 1.75, 2.0):
        lam = frac * cap
        num = int(max(10_000, lam * 2.0))
        trace = I.serving_trace_arrays(num, lam, G, seed=6000 + int(frac * 100))
        points.append(point(frac, native(trace, True), lam, num))
        log(f"serving load {frac}: {points[-1]}")
        if points[-1]["p99_ms"] >= 5 * points[0]["p99_ms"]:
            after_knee += 1
            if after_knee == 2:
                break   # past the knee: further points only queue longer
    base = points[0]["p99_ms"]
    knee = next((p["load"] for p in points if p["p99_ms"] >= 5 * base), None)
    at = next((p for p in points if p["load"] == knee), None)
    batch.close()
    torch.cuda.empty_cache()
    return {"generators": G, "chunk": chunk, "arena_GiB": arena >> 30, "sigma": 1.5, "loop": "native",
            "capacity_req_per_s": round(cap, 1), "points": points,
            "knee": {"load": knee, "p99_ms": at["p99_ms"] if at else None,
                     "sustained_numbers_per_s": at["numbers_per_s"] if at else None,
                     "frac_of_8TBs": at["frac_of_8TBs"] if at else None,
                     "rule": "first load with p99 >= 5 x p99 at load 0.1"},
            "split_ticks": "off (mtgp_server_set_split refuses them for now)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the generators are independent and need no "
              f"collective; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1005_4973_amd import inputs as I
    from paper_1005_4973_amd import mtgp

    torch.cuda.set_device(0)
    ctx = {}
    head = headline(args, torch, I, mtgp, ctx)
    ctx["head_ms"] = head["ms_per_step"]
    log(f"headline: {head['value']} G numbers/s")

    res = {
        # the workload's metric; uint32 and float32 outputs count alike (one 32-bit word each)
        "metric": "G uint32/s & % HBM write roofline, batched vs plain; p99 request latency",
        "value": head["value"],
        "unit": "G numbers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded parameter sets and states)",
        "config": head["config"],
        "roofline": head["roofline"],
    }
    if not args.no_cpu_baseline:
        # 16 threads: the host CPU share of one GPU on the benchmark machine
        # (the machine's own count is larger but shared among its GPUs)
        threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
        res["cpu_baseline"] = cpu_baseline(ctx["params"], ctx["reqs"], threads)
        log(f"cpu baseline: {res['cpu_baseline']['value']} G numbers/s")
    sections = [s for s in args.sections.split(",") if s]
    fns = {"batched_plain": batched_plain, "independent_128": independent_128, "large_states": large_states,
           "large_states_wide_m": large_states_wide_m, "normals": normals,
           "single_stream": single_stream, "serving": serving, "param_search": param_search,
           "param_search_44497": param_search_44497}
    unknown = [name for name in sections if name not in fns]
    if unknown:
        raise SystemExit(f"unknown sections: {unknown}")
    def release_headline():
        # the headline's batch and 28.6 GB output buffer serve batched_plain only
        if "batch" in ctx:
            ctx.pop("batch").close()
            ctx.pop("out", None)
            torch.cuda.empty_cache()

    for name in sections:
        if name != "batched_plain":
            release_headline()
        t0 = time.perf_counter()
        res[name] = fns[name](torch, I, mtgp, ctx)
        log(f"{name}: done in {time.perf_counter() - t0:.1f} s: {json.dumps(res[name])[:300]}")
    release_headline()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
