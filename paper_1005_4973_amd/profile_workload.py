"""Workload driver for hardware-counter runs (rocprofv3 --pmc).

Runs, in order:
  1. a device-to-device copy of exactly 1 GiB (torch), whose FETCH_SIZE and
     WRITE_SIZE readings calibrate the counters (1 GiB read, 1 GiB written);
  2. one workload as bench.py times it, in a given configuration (split
     limit and launch shape) or autotuned on its requests (the chosen
     configuration is printed); the plan is replayed twelve times back to
     back, each replay as its two phases (prepare: raw prefix and jump
     kernels; generate: the persistent generation kernel), as the benchmark
     queues its replays. The last replays are the warm ones to read (the
     first run cold); counters of the last replay are the ones to read.
     Workloads:
       batched_uneven   4096 generators (11213:23209:44497 = 2:1:1), lengths
                        log-uniform in [2^10, 2^24], mixed kinds (the headline)
       independent_128  128 MTGP-11213 generators, 2^22 uint32 outputs each
       large_23209      256 MTGP-23209 generators, 2^24 uint32 outputs each
       large_44497      256 MTGP-44497 generators, 2^24 uint32 outputs each

  3. with --probe, the store-only probe (libmtgp_probe.so) over the plan's
     work items: the write ceiling of the same output layout.

Example (a configuration bench.py's autotuner picks for the headline):
  rocprofv3 --pmc FETCH_SIZE -d out -o fetch --output-format csv -- \
      python3 paper_1005_4973_amd/profile_workload.py --workload batched_uneven --split 6174 --shape 0,256,2
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30


REPLAYS = 12


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batched_uneven",
                    choices=("batched_uneven", "independent_128", "large_23209", "large_44497"))
    ap.add_argument("--split", type=int, default=None, help="split limit in rounds (default: autotune)")
    ap.add_argument("--shape", default="auto", help="'auto' or mode,threads,spl (with --split)")
    ap.add_argument("--probe", action="store_true", help="also time the store-only probe on the plan's items")
    args = ap.parse_args()
    import torch
    from paper_1005_4973_amd import inputs as I
    from paper_1005_4973_amd import mtgp

    torch.cuda.set_device(0)
    src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    if args.workload == "batched_uneven":
        params, reqs = I.batched_uneven()
        G = len(params)
        tot = sum(r.n for r in reqs)
        out = torch.empty(tot, dtype=torch.int32, device="cuda")
        rq = [(r.gen, r.kind, r.n, out.data_ptr() + 4 * r.offset) for r in reqs]
    else:
        params, n = I.independent_128() if args.workload == "independent_128" else \
            I.large_states(int(args.workload.split("_")[1]))
        G = len(params)
        out = torch.empty(G * n, dtype=torch.int32, device="cuda")
        rq = [(g, I.KIND_U32, n, out.data_ptr() + 4 * g * n) for g in range(G)]
    batch = mtgp.Batch(params, I.state_seeds(G))
    if args.split is None:
        print(f"autotune: {batch.autotune(rq, reps=2)}", flush=True)
    else:
        batch.set_split(args.split)
        if args.shape != "auto":
            mode, threads, spl = (int(v) for v in args.shape.split(","))
            batch.set_launch(mode, threads, spl, 0, 0)
        print(f"configuration: workload {args.workload}, split {args.split}, shape {args.shape}", flush=True)
    plan = batch.plan(rq)
    d = plan.describe()
    # the lines a counter summary records: what the counted launch was
    print("split_rounds: {}".format(args.split if args.split is not None else "autotuned (see above)"), flush=True)
    print("launch: " + " ".join(f"{k}={d[k]}" for k in ("mode", "threads", "spl", "lds_words", "grid")), flush=True)
    print(f"work items: {d['items']}, jumps: {d['jumps']}", flush=True)
    for _ in range(REPLAYS):
        plan.launch_phase(mtgp.PHASE_PREPARE)
        plan.launch_phase(mtgp.PHASE_GENERATE)
    torch.cuda.synchronize()
    if args.probe:
        # the store-only probe over the same work items in queue order, on as
        # many wavefronts as the launch runs items at once (one warm-up and
        # three timed launches of store_probe_kernel<1, 0>)
        from paper_1005_4973_amd import probe
        outs, ns = plan.items()
        waves = d["grid"] * (d["threads"] // 64 if d["mode"] & 3 else 1)
        ms = probe.store_ms(outs, ns, waves, 1, False, reps=3)
        print(f"store probe: {waves} wavefronts, {ms:.4f} ms, {4 * int(ns.sum()) / ms / 1e6:.1f} GB/s", flush=True)
    plan.close()
    batch.close()
    print("profile workload done", flush=True)


if __name__ == "__main__":
    main()
