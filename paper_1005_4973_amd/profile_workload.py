"""Workload driver for hardware-counter runs (rocprofv3 --pmc).

Runs, in order:
  1. a device-to-device copy of exactly 1 GiB (torch), whose FETCH_SIZE and
     WRITE_SIZE readings calibrate the counters (1 GiB read, 1 GiB written);
  2. one launch of the headline workload: 128 MTGP-11213 generators
     (paper M rule), 2^22 uint32 outputs each, as a replay of the
     graph-captured plan bench.py times (after one warm-up replay).

Example:
  rocprofv3 --pmc FETCH_SIZE -d out -o fetch --output-format csv -- \
      python paper_1005_4973_amd/profile_workload.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30


def main():
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
    plan = batch.plan([(g, I.KIND_U32, n, out.data_ptr() + 4 * g * n) for g in range(G)])
    plan.launch()
    torch.cuda.synchronize()
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    batch.close()
    print("profile workload done", flush=True)


if __name__ == "__main__":
    main()
