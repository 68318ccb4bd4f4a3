"""Throughput benchmark of the MTGP HIP path on one MI355X.

Headline step (`value`): the 128-generator workload -- 128 distinct
MTGP-11213 generators (M drawn by the paper's thread-count rule), 2^22
outputs each, generated as uint32, then float32 in [1,2), then float32 in
[0,1): three replays of HIP-graph-captured plans (one per output kind),
each writing 2 GiB. The batch's launch shape and jump-ahead split limit are
autotuned once, before the timed region. A replay first computes the start
states of each stream's segments (a raw-word prefix and the jump
correlations), then runs the persistent generation kernel: every segment's
state is loaded into LDS, the recursion rounds run with tempering and
conversion, outputs leave with nontemporal stores, and each generator's end
state is stored back.

The same JSON line also reports:
  batched_uneven  4096 generators (2:1:1 over p = 11213, 23209, 44497),
                  lengths log-uniform in [2^10, 2^24], mixed kinds: one
                  graph-captured persistent launch vs one launch per request
  large_states    256 generators at p = 23209 and at p = 44497, 2^24 uint32 each
  normals         the headline generators, 2^22 Box-Muller normals each (float32)
  param_search    host-side search for full-period parameter sets (p = 4423, 11213) and
                  the dimension of equidistribution k(v), Delta of one found set
  single_stream   one MTGP-11213 generator, 2^20 uint32 per eager call, unsplit
                  and split into jump-ahead segments
  serving         65536 resident MTGP-11213 states behind the library's native
                  request loop, Poisson arrivals at a swept fraction of the
                  measured saturation rate, log-normal sizes
                  (median 2^16, sigma 1.5, clipped to [2^10, 2^26]):
                  p50/p99 latency and sustained numbers/s
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
SECTIONS = ("batched_uneven", "large_states", "large_states_wide_m", "normals", "single_stream", "serving",
            "param_search")


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


def cpu_baseline(params, n_per_gen, kinds, threads, reps=30):
    """The oracle on the host cores: one generator and kind per task, each
    task producing `reps` chunks of the headline's per-generator length (the
    workload's generators, kinds and lengths, about 10 s of wall time on 16
    cores); plus single-core rates for the three periods."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_1005_4973_amd import inputs as I

    tasks = [(g, k) for g in range(len(params)) for k in kinds]

    def run(task):
        g, k = task
        st = O.seed_state(I.STATE_SEED_BASE + g, params[g].mexp)
        for _ in range(reps):
            O.generate(params[g], st, n_per_gen, k)
        return reps * n_per_gen

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        total = sum(ex.map(run, tasks))
    dt = time.perf_counter() - t0
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
            "sample": f"{len(params)} generators x {len(kinds)} kinds x {reps} chunks of {n_per_gen} outputs "
                      f"({total} numbers, {dt:.2f} s wall on {threads} threads)",
            "single_core_M_numbers_s": single,
            "matrix_form_python": {"numbers_s": round(m / py_s, 1), "sample": f"{m} outputs of the single stream",
                                   "single_stream_s": round(n1 / (m / py_s), 1)}}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mtgp_kernel_headline_128x4M_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1005_4973_amd", "csrc", f) for f in ("mtgp_kernels.hip", "mtgp_internal.h")]


def measured_traffic(tuning):
    """HBM bytes per launch of the headline generation kernel from the committed
    counter summary, or None when the kernel sources or the tuned configuration
    differ from those the counters were taken with."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("kernel_source_sha256_16:", "traffic_bytes_per_launch:", "tuning:")))
    if fields.get("kernel_source_sha256_16", "").split()[0:1] != [h.hexdigest()[:16]]:
        return None
    # the split limit sets the segments whose start states the kernel reads;
    # the launch shape changes no byte the kernel moves
    recorded = dict(kv.split("=") for kv in fields.get("tuning", "").split())
    if recorded.get("split_rounds") != str(tuning["split_rounds"]):
        return None
    return int(fields["traffic_bytes_per_launch"].strip())


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
# headline: 128 independent generators
# ---------------------------------------------------------------------------

def headline(args, torch, I, mtgp):
    params, n = I.independent_128()
    G = len(params)
    kinds = (I.KIND_U32, I.KIND_F12, I.KIND_F01)
    batch = mtgp.Batch(params, I.state_seeds(G))
    out = torch.empty(G * n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    reqs = {k: [(g, k, n, out.data_ptr() + 4 * g * n) for g in range(G)] for k in kinds}
    # launch shape and jump-ahead split limit, tuned on the uint32 requests
    # (outputs are identical under every choice; states are left untouched)
    tuning = batch.autotune(reqs[I.KIND_U32], reps=3, stream=stream)
    log(f"autotune: {tuning}")
    plans = [batch.plan(reqs[k]) for k in kinds]

    for _ in range(args.warmup):
        for p in plans:
            p.launch(stream)
    torch.cuda.synchronize()

    # each launch as its two phases, with events around the generation phase:
    # segment start states (raw prefix + jump kernels), then the persistent
    # generation kernel, the dominant one
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps * len(kinds))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    for _ in range(args.steps):
        for p in plans:
            ev[i][0].record(stream)
            p.launch_phase(mtgp.PHASE_PREPARE, stream)
            ev[i][1].record(stream)
            p.launch_phase(mtgp.PHASE_GENERATE, stream)
            ev[i][2].record(stream)
            i += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # store-only ceiling: a torch fill of the same 2 GiB buffer
    fill_ms = timed_ms(torch, lambda: out.fill_(7))
    store_gbs = 4 * G * n / fill_ms / 1e6

    numbers_per_step = G * n * len(kinds)
    gen_ms = [b.elapsed_time(c) for a, b, c in ev]
    prep_ms = [a.elapsed_time(b) for a, b, c in ev]
    avg_gen_s = sum(gen_ms) / len(gen_ms) / 1e3
    N = 351
    # algorithmic bytes of one launch: outputs + state in and out + parameter record
    alg_bytes = G * (4 * n + 8 * N + 256)
    achieved = alg_bytes / avg_gen_s / 1e9
    for p in plans:
        p.close()
    batch.close()
    del out
    torch.cuda.empty_cache()
    mode = tuning["mode"]
    kernel = "mtgp_kernel<{}, {}>".format("true" if mode >= 0 and mode & 1 else "false",
                                          "true" if mode >= 0 and mode & 4 else "false")
    return params, n, kinds, tuning, {
        "value": round(numbers_per_step * args.steps / dt / 1e9, 3),
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(tuning),
                     "kernel": kernel + " (persistent generation over jump-ahead segments)",
                     "avg_launch_ms": round(avg_gen_s * 1e3, 4),
                     "avg_prepare_ms": round(sum(prep_ms) / len(prep_ms), 4),
                     "alg_bytes_per_launch": alg_bytes,
                     "store_ceiling_GBs": round(store_gbs, 1),
                     "frac_of_store_ceiling": round(achieved / store_gbs, 4)},
    }


# ---------------------------------------------------------------------------
# extra sections
# ---------------------------------------------------------------------------

def batched_uneven(torch, I, mtgp):
    params, reqs = I.batched_uneven()
    G = len(params)
    tot = sum(r.n for r in reqs)
    batch = mtgp.Batch(params, I.state_seeds(G))
    out = torch.empty(tot, dtype=torch.int32, device="cuda")
    base = out.data_ptr()
    rq = [(r.gen, r.kind, r.n, base + 4 * r.offset) for r in reqs]
    t0 = time.perf_counter()
    tuning = batch.autotune(rq, reps=2)
    tune_s = time.perf_counter() - t0
    plan = batch.plan(rq)
    ms_b = timed_ms(torch, lambda: plan.launch())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.generate_plain(rq)
    torch.cuda.synchronize()
    ms_p = (time.perf_counter() - t0) * 1e3
    plan.close()
    # critical path: the segment with the most rounds under the tuned shape and
    # split limit, timed alone (same shape, no split, one workgroup)
    r_max, crit = 0, None
    for r in reqs:
        ps = params[r.gen]
        W = round_width(state_words(ps.mexp), ps.pos, tuning)
        rounds = -(-r.n // W)
        S = -(-rounds // tuning["split_rounds"]) if tuning["split_rounds"] else 1
        J = -(-r.n // S)
        if -(-J // W) > r_max:
            r_max, crit = -(-J // W), (r, J)
    batch.set_split(0)
    (r, J) = crit
    p1 = batch.plan([(r.gen, r.kind, J, base + 4 * r.offset)])
    ms_c = timed_ms(torch, lambda: p1.launch())
    p1.close()
    batch.close()
    del out
    torch.cuda.empty_cache()
    Ns = {11213: 351, 23209: 726, 44497: 1391}
    alg = sum(4 * r.n + 8 * Ns[params[r.gen].mexp] + 256 for r in reqs)
    return {"generators": G, "numbers": tot,
            "batched": {"ms": round(ms_b, 3), "G_numbers_s": round(tot / ms_b / 1e6, 2), **roof(alg, ms_b / 1e3),
                        "autotuned": tuning, "autotune_s": round(tune_s, 1)},
            "critical_path": {"segment_rounds": r_max, "mexp": params[crit[0].gen].mexp, "segment_outputs": crit[1],
                              "alone_ms": round(ms_c, 3), "makespan_over_bound": round(ms_b / ms_c, 2)},
            "plain_one_launch_per_request": {"ms": round(ms_p, 1), "G_numbers_s": round(tot / ms_p / 1e6, 3)},
            "speedup_batched_vs_plain": round(ms_p / ms_b, 1)}


def state_words(mexp):
    return (mexp + 31) // 32


def round_width(N, M, tuning):
    """Steps a round of this generator computes under a tuned launch shape:
    W = min(N - M, lanes * s), s the largest steps per lane allowed by the
    shape with lanes * s <= N - M (the library's own rule)."""
    mode = tuning["mode"]
    if mode >= 0 and (mode & 3) == 2:
        return 64   # chunked form: a round is one chunk of 64 steps
    if mode < 0:
        wave, threads, cap = False, 256, 4
    else:
        wave, threads, cap = bool(mode & 1), tuning["threads"], tuning["spl"]
    lanes = 64 if wave else threads
    cands = (16, 12, 8, 6, 4, 2, 1) if wave else (4, 2, 1)
    s = next((c for c in cands if c <= cap and lanes * c <= N - M), 1)
    return min(N - M, lanes * s)


def large_states(torch, I, mtgp):
    res = {}
    for mexp, N in ((23209, 726), (44497, 1391)):
        params, n = I.large_states(mexp)
        G = len(params)
        batch = mtgp.Batch(params, I.state_seeds(G))
        out = torch.empty(G * n, dtype=torch.int32, device="cuda")
        rq = [(g, 0, n, out.data_ptr() + 4 * g * n) for g in range(G)]
        t0 = time.perf_counter()
        tuning = batch.autotune(rq, reps=2)
        tune_s = time.perf_counter() - t0
        plan = batch.plan(rq)
        ms = timed_ms(torch, lambda: plan.launch())
        plan.close()
        batch.close()
        del out
        torch.cuda.empty_cache()
        alg = G * (4 * n + 8 * N + 256)
        res[f"p{mexp}"] = {"generators": G, "numbers": G * n, "ms": round(ms, 3),
                           "G_numbers_s": round(G * n / ms / 1e6, 2), **roof(alg, ms / 1e3),
                           "autotuned": tuning, "autotune_s": round(tune_s, 1)}
    return res


def large_states_wide_m(torch, I, mtgp):
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
    ms = timed_ms(torch, lambda: plan.launch(), reps=5, warmup=1)
    plan.close()
    widths = [round_width(N, ps.pos, tuning) for ps in params]
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


def normals(torch, I, mtgp):
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


def param_search(torch, I, mtgp):
    """Host-side recursion-parameter search (section 5): full-period sets with
    an ID embedded, seeded so the draw counts are fixed; the paper's own
    search took 338 s per MTGP-11213 set on average (context only)."""
    threads = min(16, len(os.sched_getaffinity(0)))
    runs = []
    found = {}
    for mexp, ident in ((4423, 1), (11213, 1), (11213, 4)):
        ps, st = mtgp.search_params(mexp, id=ident, seed=mexp, threads=threads)
        runs.append({"mexp": mexp, "id": ident, "draws": st["draws"], "seconds": st["seconds"]})
        found[(mexp, ident)] = ps
    # dimension of equidistribution (section 3.4) of a found set, tempered and
    # not: one core, host only
    ps = found[(11213, 1)]
    equi = {"mexp": 11213, "id": 1}
    for name, tempered in (("tempered", True), ("untempered", False)):
        t0 = time.perf_counter()
        k, delta = mtgp.equidistribution(ps, tempered=tempered)
        equi[name] = {"delta": delta, "k_min": min(k), "seconds": round(time.perf_counter() - t0, 2)}
    return {"threads": threads, "runs": runs, "equidistribution": equi}


def single_stream(torch, I, mtgp):
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


def serving(torch, I, mtgp):
    """65536 resident MTGP-11213 states served by the library's request loop
    (mtgp_server_*, native admission and tick building; Python only feeds
    arrivals): saturation rate with all requests available at once, then
    Poisson arrivals at fractions of it. One point with the Python loop
    (serve.Server) is kept for comparison."""
    from paper_1005_4973_amd import serve
    G = 65536
    params = I.serving_params(G)
    batch = mtgp.Batch(params, I.state_seeds(G))
    arena, chunk = 8 << 30, 1 << 18

    def native(trace, realtime):
        srv = serve.NativeServer(batch, arena_bytes=arena, chunk=chunk, depth=2)
        st = srv.run(trace, realtime=realtime)
        srv.close()
        return st

    def point(load, st, lam=None, num=None):
        d = {"load": load, "req_per_s": round(lam if lam is not None else st.completed / st.wall_s, 1),
             "completed": st.completed, "numbers_per_s": round(st.numbers / st.wall_s, 1),
             "p50_ms": round(st.percentile(50) * 1e3, 3), "p99_ms": round(st.percentile(99) * 1e3, 3)}
        if num is not None:
            d["requests"] = num
        return d

    sat_trace = I.serving_trace(20000, rate_per_s=1.0, num_gens=G, seed=5001)
    native(sat_trace[:500], False)          # warm-up
    st = native(sat_trace, False)
    sat_rate = st.completed / st.wall_s
    points = [point("saturation", st)]
    for frac in (0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2):
        lam = frac * sat_rate
        num = int(min(40000, max(500, lam * 1.5)))
        trace = I.serving_trace(num, rate_per_s=lam, num_gens=G, seed=6000 + int(frac * 100))
        s = native(trace, True)
        points.append(point(frac, s, lam, num))
        log(f"serving load {frac}: {points[-1]}")
    # the Python loop at the rate the native loop sustained at 0.5 load, for comparison
    lam = 0.5 * sat_rate
    trace = I.serving_trace(int(min(12000, max(500, lam * 1.5))), rate_per_s=lam, num_gens=G, seed=6050)
    srv = serve.Server(serve.GpuExecutor(batch), mem_budget_bytes=arena, chunk=chunk, depth=2, keep_outputs=False)
    py = point(0.5, srv.run(trace, realtime=True), lam, len(trace))
    batch.close()
    torch.cuda.empty_cache()
    return {"generators": G, "chunk": chunk, "arena_GiB": arena >> 30, "sigma": 1.5, "loop": "native",
            "points": points, "python_loop_at_0.5": py}


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
    params, n, kinds, tuning, head = headline(args, torch, I, mtgp)
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
        "config": {"workload": "128 independent MTGP-11213 generators (distinct seeded parameter sets, "
                               "M in [2,95]), 2^22 outputs each as uint32, float32 [1,2) and float32 [0,1); "
                               "one graph-captured plan per output kind (jump-ahead segment states, then "
                               "persistent generation)",
                   "generators": 128, "mexp": 11213, "outputs_per_generator": n,
                   "kinds": ["uint32", "float32_1to2", "float32_0to1"], "autotuned": tuning},
        "roofline": head["roofline"],
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
        res["cpu_baseline"] = cpu_baseline(params, n, kinds, threads)
        log(f"cpu baseline: {res['cpu_baseline']['value']} G numbers/s")
    sections = [s for s in args.sections.split(",") if s]
    fns = {"batched_uneven": batched_uneven, "large_states": large_states,
           "large_states_wide_m": large_states_wide_m, "normals": normals,
           "single_stream": single_stream, "serving": serving, "param_search": param_search}
    unknown = [name for name in sections if name not in fns]
    if unknown:
        raise SystemExit(f"unknown sections: {unknown}")
    for name in sections:
        t0 = time.perf_counter()
        res[name] = fns[name](torch, I, mtgp)
        log(f"{name}: done in {time.perf_counter() - t0:.1f} s: {json.dumps(res[name])[:300]}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
