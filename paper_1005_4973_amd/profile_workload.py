"""Workload driver for hardware-counter runs (rocprofv3 --pmc).

Runs, in order:
  1. a device-to-device copy of exactly 1 GiB (torch), whose FETCH_SIZE and
     WRITE_SIZE readings calibrate the counters (1 GiB read, 1 GiB written);
  2. the headline workload as bench.py times it: 128 MTGP-11213 generators
     (paper M rule), 2^22 uint32 outputs each; the batch is autotuned on
     these requests (the chosen configuration is printed), or set to the
     configuration given with --split and --shape, then the plan is replayed
     three times as its two phases (prepare: raw prefix and jump kernels;
     generate: the persistent generation kernel). Counters of the last replay
     are the ones to read.

Example (the configuration bench.py's autotuner picks for this workload):
  rocprofv3 --pmc FETCH_SIZE -d out -o fetch --output-format csv -- \
      python paper_1005_4973_amd/profile_workload.py --split 2048 --shape auto
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--split", type=int, default=None, help="split limit in rounds (default: autotune)")
    ap.add_argument("--shape", default="auto", help="'auto' or mode,threads,spl (with --split)")
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

    params, n = I.independent_128()
    G = len(params)
    batch = mtgp.Batch(params, I.state_seeds(G))
    out = torch.empty(G * n, dtype=torch.int32, device="cuda")
    reqs = [(g, I.KIND_U32, n, out.data_ptr() + 4 * g * n) for g in range(G)]
    if args.split is None:
        print(f"autotune: {batch.autotune(reqs, reps=3)}", flush=True)
    else:
        batch.set_split(args.split)
        if args.shape != "auto":
            mode, threads, spl = (int(v) for v in args.shape.split(","))
            batch.set_launch(mode, threads, spl, 0, 0)
        print(f"configuration: split {args.split}, shape {args.shape}", flush=True)
    plan = batch.plan(reqs)
    for _ in range(3):
        plan.launch_phase(mtgp.PHASE_PREPARE)
        plan.launch_phase(mtgp.PHASE_GENERATE)
        torch.cuda.synchronize()
    plan.close()
    batch.close()
    print("profile workload done", flush=True)


if __name__ == "__main__":
    main()
