"""Workload driver for a kernel trace of the request loop (rocprofv3
--kernel-trace --stats).

The serving configuration bench.py measures: 65536 resident MTGP-11213
states, an 8 GiB output arena, chunks of 2^18 outputs, two ticks in flight.
After a warm-up of 2000 requests it offers one open-loop burst (log-normal
sizes, median 2^16, sigma 1.5, clipped to [2^10, 2^26]) well above capacity
and prints the requests, outputs and wall time of the burst, so that the
trace's tick launches can be set against them: their count, their durations
and the share of the burst's wall time the device spends in them.

Example:
  rocprofv3 --kernel-trace --stats -d out -o serve --output-format csv -- \\
      python3 paper_1005_4973_amd/profile_serving.py --requests 400000
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=400_000)
    ap.add_argument("--rate", type=float, default=4e6, help="offered requests/s of the burst")
    args = ap.parse_args()
    import torch
    from paper_1005_4973_amd import inputs as I
    from paper_1005_4973_amd import mtgp, serve

    torch.cuda.set_device(0)
    G = 65536
    batch = mtgp.Batch(I.serving_params(G), I.state_seeds(G))

    def native(trace):
        srv = serve.NativeServer(batch, arena_bytes=8 << 30, chunk=1 << 18, depth=2)
        st = srv.run(trace, realtime=True)
        srv.close()
        return st

    st = native(I.serving_trace_arrays(2000, 1e5, G, seed=5000))
    print(f"warm-up: {st.completed} requests", flush=True)
    st = native(I.serving_trace_arrays(args.requests, args.rate, G, seed=5001))
    print(f"burst: {st.completed} requests, {st.numbers} outputs, wall {st.wall_s:.4f} s, "
          f"{st.completed / st.wall_s:.0f} requests/s, {st.numbers / st.wall_s / 1e9:.1f} G outputs/s, "
          f"p50 {st.percentile(50) * 1e3:.2f} ms, p99 {st.percentile(99) * 1e3:.2f} ms", flush=True)
    batch.close()


if __name__ == "__main__":
    main()
