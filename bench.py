"""Throughput benchmark of the MTGP HIP path on one MI355X.

One step = the whole generation path for the 128-generator workload: 128
distinct MTGP-11213 generators (paper M rule), 2^22 outputs each, generated
as uint32, then float32 in [1,2), then float32 in [0,1) -- one persistent
batched launch per output kind, each writing 2 GiB. Every launch loads each
state into LDS, runs the recursion rounds with tempering and conversion,
stores outputs with nontemporal writes, and stores the states back.

Prints one JSON line. `value` is numbers/s (all kinds count) with the inputs
(states, parameters) resident in HBM when the timed region starts.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (default: host cores, max 16)")
    return ap.parse_args()


def cpu_baseline(params, n_per_gen, kinds, threads):
    """The oracle on the host cores: one generator per task, a bounded sample."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_1005_4973_amd import inputs as I

    # about 15 s of single-core oracle work: every generator, every kind,
    # three times the per-generator length of one step
    sample_gens = len(params)
    n = 3 * n_per_gen
    tasks = [(g, k) for g in range(sample_gens) for k in kinds]

    def run(task):
        g, k = task
        st = O.seed_state(I.STATE_SEED_BASE + g, params[g].mexp)
        O.generate(params[g], st, n, k)
        return n

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        total = sum(ex.map(run, tasks))
    dt = time.perf_counter() - t0
    return {"value": total / dt / 1e9, "unit": "G numbers/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample_gens} generators x {n} outputs x {len(kinds)} kinds "
                      f"({total} numbers, {dt:.2f} s wall)"}


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
    params, n = I.independent_128()
    G = len(params)
    kinds = (I.KIND_U32, I.KIND_F12, I.KIND_F01)
    batch = mtgp.Batch(params, I.state_seeds(G))
    out = torch.empty(G * n, dtype=torch.int32, device="cuda")
    reqs = [[(g, k, n, out.data_ptr() + 4 * g * n) for g in range(G)] for k in kinds]
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        for r in reqs:
            batch.generate(r, stream)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps * len(kinds))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    for _ in range(args.steps):
        for r in reqs:
            ev[i][0].record(stream)
            batch.generate(r, stream)
            ev[i][1].record(stream)
            i += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    numbers_per_step = G * n * len(kinds)
    value = numbers_per_step * args.steps / dt
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    avg_launch_s = sum(launch_ms) / len(launch_ms) / 1e3
    N = 351
    alg_bytes = sum(4 * n + 8 * N + 256 for _ in range(G))   # outputs + state in/out + parameters
    achieved = alg_bytes / avg_launch_s / 1e9

    res = {
        "metric": "G numbers/s (uint32 and float32 outputs) and % of HBM write roofline",
        "value": round(value / 1e9, 3),
        "unit": "G numbers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded parameter sets and states)",
        "config": {"workload": "128 independent MTGP-11213 generators (distinct seeded parameter sets, "
                               "M in [2,95]), 2^22 outputs each as uint32, float32 [1,2) and float32 [0,1); "
                               "one persistent batched launch per output kind",
                   "generators": G, "mexp": 11213, "outputs_per_generator": n,
                   "kinds": ["uint32", "float32_1to2", "float32_0to1"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "mtgp_generate_kernel", "avg_launch_ms": round(avg_launch_s * 1e3, 4)},
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
        res["cpu_baseline"] = cpu_baseline(params, n, kinds, threads)
    batch.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
