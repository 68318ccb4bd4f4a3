"""Continuous-batching request loop over resident MTGP states.

Requests (generator, kind, n) arrive over time. The server keeps every
generator state resident in HBM (one mtgp batch), admits requests in arrival
order while their output footprint (4n bytes) fits a memory budget, and runs
ticks: each tick advances every admitted request by up to `chunk` outputs in
one persistent batched launch, so small requests finish while large ones are
still streaming and requests that arrive mid-run join at the next tick.
Requests for one generator are served strictly in arrival order (one chunk
per tick, from the oldest unfinished request of that generator), so each
result is exactly the stream segment it would get alone.

Up to `depth` ticks are queued on the device at once (stream order keeps
consecutive chunks of one generator in sequence); completion is detected with
events and a request's latency is its completion time minus its arrival time.

The executor interface (launch / ready / wait) lets tests drive the same
scheduler with a CPU executor. NativeServer runs the same policy in the
library (mtgp_server_*), with the request bookkeeping, admission and tick
building in C++; Python only feeds arrivals and collects completions.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple


@dataclass
class Request:
    rid: int
    gen: int
    kind: int
    n: int
    arrival: float                  # seconds, on the server clock
    out: object = None              # output buffer (executor-specific)
    done: int = 0                   # outputs already scheduled
    finished: int = 0               # outputs completed on the device
    t_admit: float = math.nan
    t_done: float = math.nan
    rejected: bool = False

    @property
    def nbytes(self) -> int:
        return 4 * self.n


class Executor:
    """Runs one tick: a list of (gen, kind, n, out, offset) chunks."""

    def alloc(self, req: Request):
        raise NotImplementedError

    def free(self, req: Request):
        pass

    def launch(self, chunks: List[Tuple[int, int, int, object, int]]):
        raise NotImplementedError

    def ready(self, handle) -> bool:
        raise NotImplementedError

    def wait(self, handle):
        raise NotImplementedError


class GpuExecutor(Executor):
    """Chunks go to one mtgp batch launch on a dedicated stream; an event per tick."""

    def __init__(self, batch, stream=None):
        import torch
        self.torch = torch
        self.batch = batch
        self.stream = stream if stream is not None else torch.cuda.Stream()

    def alloc(self, req: Request):
        t = self.torch
        dtype = t.int32 if req.kind == 0 else t.float32
        with t.cuda.stream(self.stream):
            req.out = t.empty(req.n, dtype=dtype, device="cuda")

    def free(self, req: Request):
        pass   # the caller owns req.out; torch frees it when dropped

    def launch(self, chunks):
        import numpy as np
        t = self.torch
        k = len(chunks)
        gens = np.fromiter((c[0] for c in chunks), dtype=np.uint32, count=k)
        kinds = np.fromiter((c[1] for c in chunks), dtype=np.uint32, count=k)
        ns = np.fromiter((c[2] for c in chunks), dtype=np.uint64, count=k)
        ptrs = np.fromiter((c[3].data_ptr() + 4 * c[4] for c in chunks), dtype=np.uint64, count=k)
        self.batch.generate_arrays(gens, kinds, ns, ptrs, self.stream)
        ev = t.cuda.Event()
        ev.record(self.stream)
        return ev

    def ready(self, handle) -> bool:
        return handle.query()

    def wait(self, handle):
        handle.synchronize()


@dataclass
class ServeStats:
    offered_rate: float
    completed: int
    rejected: int
    numbers: int
    wall_s: float
    latencies: List[float] = field(default_factory=list)

    def percentile(self, q: float) -> float:
        if not self.latencies:
            return math.nan
        xs = sorted(self.latencies)
        k = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
        return xs[k]

    def as_dict(self):
        return {"offered_req_per_s": self.offered_rate, "completed": self.completed,
                "rejected": self.rejected, "numbers": self.numbers, "wall_s": round(self.wall_s, 4),
                "numbers_per_s": self.numbers / self.wall_s if self.wall_s > 0 else math.nan,
                "p50_ms": self.percentile(50) * 1e3, "p99_ms": self.percentile(99) * 1e3}


class Server:
    def __init__(self, executor: Executor, mem_budget_bytes: int = 8 << 30, chunk: int = 1 << 18,
                 depth: int = 2, max_requests_per_tick: int = 1 << 16,
                 clock: Callable[[], float] = time.perf_counter, keep_outputs: bool = True):
        self.ex = executor
        self.keep_outputs = keep_outputs
        self.budget = mem_budget_bytes
        self.chunk = chunk
        self.depth = depth
        self.max_per_tick = max_requests_per_tick
        self.clock = clock
        self.waiting: Deque[Request] = collections.deque()     # arrived, not admitted (FIFO)
        self.active: Dict[int, Deque[Request]] = {}            # gen -> admitted, unfinished (FIFO)
        self.inflight: Deque[Tuple[object, List[Tuple[Request, int]]]] = collections.deque()
        self.in_use = 0
        self.unscheduled = 0        # outputs admitted but not yet put in a tick
        self.completed: List[Request] = []
        self.rejected: List[Request] = []

    # -- admission -----------------------------------------------------------
    def submit(self, req: Request):
        if req.nbytes > self.budget:
            req.rejected = True
            self.rejected.append(req)
            return
        self.waiting.append(req)

    def _admit(self, now: float):
        while self.waiting and self.in_use + self.waiting[0].nbytes <= self.budget:
            r = self.waiting.popleft()
            self.ex.alloc(r)
            r.t_admit = now
            self.in_use += r.nbytes
            self.unscheduled += r.n
            self.active.setdefault(r.gen, collections.deque()).append(r)

    # -- ticks ---------------------------------------------------------------
    def _build_tick(self) -> List[Tuple[Request, int]]:
        picks = []
        for gen, q in self.active.items():
            # oldest request of this generator with work left to schedule
            for r in q:
                if r.done < r.n:
                    k = min(self.chunk, r.n - r.done)
                    picks.append((r, k))
                    break
            if len(picks) >= self.max_per_tick:
                break
        return picks

    def _launch(self, picks):
        chunks = [(r.gen, r.kind, k, r.out, r.done) for (r, k) in picks]
        handle = self.ex.launch(chunks)       # nothing is committed if this raises
        for r, k in picks:
            r.done += k
            self.unscheduled -= k
        self.inflight.append((handle, picks))

    def _retire(self, handle_picks, now: float):
        _, picks = handle_picks
        for r, k in picks:
            r.finished += k
            if r.finished == r.n:
                r.t_done = now
                self.in_use -= r.nbytes
                q = self.active[r.gen]
                q.remove(r)
                if not q:
                    del self.active[r.gen]
                self.ex.free(r)
                if not self.keep_outputs:
                    r.out = None
                self.completed.append(r)

    def _pending_work(self) -> bool:
        return self.unscheduled > 0

    def step(self, now: float):
        """Retire finished ticks, admit arrivals, and queue ticks up to `depth`."""
        while self.inflight and self.ex.ready(self.inflight[0][0]):
            self._retire(self.inflight.popleft(), now)
        self._admit(now)
        while len(self.inflight) < self.depth and self._pending_work():
            self._launch(self._build_tick())

    def drain(self):
        while self.inflight:
            h = self.inflight[0][0]
            self.ex.wait(h)
            self._retire(self.inflight.popleft(), self.clock())

    # -- trace driver --------------------------------------------------------
    def run(self, trace: Sequence[Tuple[float, int, int, int]], realtime: bool = True,
            poll_s: float = 20e-6) -> ServeStats:
        """trace: (arrival_s, gen, n, kind) sorted by arrival. With realtime,
        requests are released when the wall clock reaches their arrival time;
        otherwise all are available at once (saturation)."""
        t0 = self.clock()
        reqs = [Request(i, g, k, n, a if realtime else 0.0) for i, (a, g, n, k) in enumerate(trace)]
        i = 0
        while i < len(reqs) or self.waiting or self.active or self.inflight:
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            self.step(now)
            if self.inflight and not self.ex.ready(self.inflight[0][0]):
                # nothing to retire yet; wait for the next arrival or a short poll
                nxt = reqs[i].arrival - now if i < len(reqs) else poll_s
                if nxt > 0:
                    time.sleep(min(poll_s, nxt))
            elif not self.inflight and i < len(reqs) and not self.waiting:
                dt = reqs[i].arrival - (self.clock() - t0)
                if dt > 0:
                    time.sleep(dt)
            elif not self.inflight and not self.active and i >= len(reqs) and self.waiting:
                # a request larger than the free budget with nothing in flight cannot happen
                # (submit rejects requests above the whole budget); admit on the next step
                pass
        self.drain()
        wall = self.clock() - t0
        done = [r for r in reqs if not r.rejected and not math.isnan(r.t_done)]
        lat = [r.t_done - r.arrival for r in done]
        span = trace[-1][0] if (realtime and trace) else 0.0
        rate = len(trace) / span if span > 0 else math.inf
        return ServeStats(rate, len(done), len(self.rejected), sum(r.n for r in done), wall, lat)


SERVER_REQUEST_DTYPE = [("rid", "<u8"), ("gen", "<u4"), ("kind", "<u4"), ("n", "<u8")]
COMPLETION_DTYPE = [("rid", "<u8"), ("offset", "<u8"), ("n", "<u8")]


class NativeServer:
    """The library's request loop (mtgp_server_*) over a batch, with a device
    output arena of `arena_bytes` (the admission budget)."""

    def __init__(self, batch, arena_bytes: int = 8 << 30, chunk: int = 1 << 18, depth: int = 2,
                 stream=None, max_report: int = 1 << 16, split=None):
        """split: None, or (min_outputs, max_segments, seg_chunks, slots) for
        mtgp_server_set_split (jump-ahead segments for long requests on
        generators prepared with Batch.prepare_split)."""
        import numpy as np
        import torch
        from . import mtgp
        self.np, self.torch, self.mtgp = np, torch, mtgp
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.arena = torch.empty(arena_bytes // 4, dtype=torch.int32, device="cuda")
        L = mtgp.lib()
        self._h = L.mtgp_server_create(batch._h, self.arena.data_ptr(), arena_bytes, chunk, depth,
                                       mtgp._stream_ptr(self.stream))
        if not self._h:
            raise mtgp.MTGPError(mtgp.MTGP_EINVAL, "mtgp_server_create")
        if split is not None:
            mtgp._check(L.mtgp_server_set_split(self._h, *[int(v) for v in split]), "mtgp_server_set_split")
        self._done = np.zeros(max_report, dtype=COMPLETION_DTYPE)
        self._ndone = __import__("ctypes").c_uint32(0)

    def submit(self, reqs):
        """reqs: numpy array of SERVER_REQUEST_DTYPE, in arrival order."""
        if len(reqs):
            self.mtgp._check(self.mtgp.lib().mtgp_server_submit(self._h, reqs.ctypes.data, len(reqs)),
                             "mtgp_server_submit")

    def poll(self):
        """One scheduling step; returns completions (numpy COMPLETION_DTYPE)."""
        import ctypes
        L = self.mtgp.lib()
        ptr = self._done.ctypes.data_as(ctypes.POINTER(self.mtgp.CompletionC))
        self.mtgp._check(L.mtgp_server_poll(self._h, ptr, len(self._done), ctypes.byref(self._ndone)),
                         "mtgp_server_poll")
        return self._done[: self._ndone.value].copy()

    def release(self, rids):
        rids = self.np.ascontiguousarray(rids, dtype=self.np.uint64)
        if len(rids):
            self.mtgp._check(self.mtgp.lib().mtgp_server_release(self._h, rids.ctypes.data, len(rids)),
                             "mtgp_server_release")

    def output(self, offset: int, n: int):
        """A completed request's outputs: a view of the arena (valid until released)."""
        return self.arena[offset // 4: offset // 4 + n]

    def pending(self):
        """(waiting, active, in-flight ticks) inside the library's loop."""
        import ctypes
        w, a, f = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint32(0)
        self.mtgp._check(self.mtgp.lib().mtgp_server_pending(self._h, ctypes.byref(w), ctypes.byref(a),
                                                            ctypes.byref(f)), "mtgp_server_pending")
        return w.value, a.value, f.value

    def run(self, trace: Sequence[Tuple[float, int, int, int]], realtime: bool = True, keep: bool = False,
            on_complete: Optional[Callable[[int, object], None]] = None, poll_s: float = 20e-6,
            clock: Callable[[], float] = time.perf_counter) -> ServeStats:
        """Like Server.run. Each completed request's outputs are handed to
        on_complete(rid, arena view) if given, then released, unless keep (then
        self.kept maps rid -> (offset, n) and the caller releases them; a trace
        whose kept outputs outgrow the arena raises instead of waiting)."""
        np = self.np
        if isinstance(trace, tuple) and len(trace) == 4 and hasattr(trace[0], "shape"):
            t_in, g_in, n_in, k_in = trace          # arrays (inputs.serving_trace_arrays)
        else:
            t_in = [t[0] for t in trace]
            g_in = [t[1] for t in trace]
            n_in = [t[2] for t in trace]
            k_in = [t[3] for t in trace]
        count = len(t_in)
        arrival = np.asarray(t_in, dtype=np.float64) if realtime else np.zeros(count)
        reqs = np.zeros(count, dtype=SERVER_REQUEST_DTYPE)
        reqs["rid"] = np.arange(count)
        reqs["gen"] = g_in
        reqs["n"] = n_in
        reqs["kind"] = k_in
        t_done = np.full(count, np.nan)
        self.kept = {}
        # the loop calls the library directly with pointers taken once (no
        # per-call slicing, pointer objects or copies of the completions)
        import ctypes
        L = self.mtgp.lib()
        submit_fn, poll_fn, release_fn = L.mtgp_server_submit, L.mtgp_server_poll, L.mtgp_server_release
        h = self._h
        base = reqs.ctypes.data
        size = reqs.dtype.itemsize
        done_arr = self._done
        done_ptr = done_arr.ctypes.data_as(ctypes.POINTER(self.mtgp.CompletionC))
        cap = len(done_arr)
        ndone = ctypes.c_uint32(0)
        ndone_ref = ctypes.byref(ndone)
        rel = np.zeros(cap, dtype=np.uint64)
        rel_ptr = rel.ctypes.data
        check = self.mtgp._check
        t0 = clock()
        i = 0
        outstanding = 0
        while i < count or outstanding > 0:
            now = clock() - t0
            j = int(np.searchsorted(arrival, now, side="right")) if realtime else count
            if j > i:
                check(submit_fn(h, base + i * size, j - i), "mtgp_server_submit")
                outstanding += j - i
                i = j
            check(poll_fn(h, done_ptr, cap, ndone_ref), "mtgp_server_poll")
            nd = ndone.value
            if nd:
                done = done_arr[:nd]
                rid = done["rid"]
                t_done[rid] = clock() - t0
                outstanding -= nd
                if on_complete is not None:
                    for c in done:
                        on_complete(int(c["rid"]), self.output(int(c["offset"]), int(c["n"])))
                if keep:
                    for c in done:
                        self.kept[int(c["rid"])] = (int(c["offset"]), int(c["n"]))
                else:
                    rel[:nd] = rid
                    check(release_fn(h, rel_ptr, nd), "mtgp_server_release")
            elif outstanding > 0:
                if keep:
                    waiting, active, inflight = self.pending()
                    if waiting and not active and not inflight:
                        raise RuntimeError("the arena is full of kept outputs: release some or use a larger arena")
                time.sleep(poll_s)                            # work on the device: poll again shortly
            elif i < count:
                time.sleep(max(0.0, arrival[i] - (clock() - t0)))   # idle until the next arrival
        wall = clock() - t0
        ok = ~np.isnan(t_done)
        lat = list((t_done - arrival)[ok])
        span = float(arrival[-1]) if (realtime and count) else 0.0
        rate = count / span if span > 0 else math.inf
        return ServeStats(rate, int(ok.sum()), 0, int(reqs["n"][ok].sum()), wall, lat)

    def close(self):
        if getattr(self, "_h", None):
            self.mtgp.lib().mtgp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

