"""Python binding of libmtgp.so (include/mtgp.h): argument marshalling only.

Every generation step runs in the HIP kernels of libmtgp.so; this module only
passes torch tensor pointers and torch streams through the C ABI. It raises
if the library has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, NamedTuple, Optional, Sequence

import torch  # loads torch's HIP runtime first, so the library shares it

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmtgp.so")

MTGP_OK = 0
MTGP_EINVAL = -1
MTGP_ENOMEM = -2
MTGP_EDEVICE = -3

PHASE_ALL = 0
PHASE_PREPARE = 1
PHASE_GENERATE = 2

MODE_GROUP = 0
MODE_WAVE = 1
MODE_REC_BASIS = 4   # flag: recursion table from its F2 basis in registers (not an LDS lookup)

KIND_UINT32 = 0
KIND_FLOAT32_1TO2 = 1
KIND_FLOAT32_0TO1 = 2
KIND_NORMAL_FLOAT32 = 3   # Box-Muller on pairs of float [1,2) outputs; n even


class MTGPError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class ParamSetC(ctypes.Structure):
    _fields_ = [("mexp", ctypes.c_uint32), ("pos", ctypes.c_uint32),
                ("sh1", ctypes.c_uint32), ("sh2", ctypes.c_uint32),
                ("param_tbl", ctypes.c_uint32 * 16), ("temper_tbl", ctypes.c_uint32 * 16)]


class SearchStatsC(ctypes.Structure):
    _fields_ = [("draws", ctypes.c_uint64), ("evaluated", ctypes.c_uint64), ("full_degree", ctypes.c_uint64),
                ("sieve_passed", ctypes.c_uint64), ("seconds", ctypes.c_double)]


class ServerRequestC(ctypes.Structure):
    _fields_ = [("rid", ctypes.c_uint64), ("gen", ctypes.c_uint32), ("kind", ctypes.c_uint32), ("n", ctypes.c_uint64)]


class CompletionC(ctypes.Structure):
    _fields_ = [("rid", ctypes.c_uint64), ("offset", ctypes.c_uint64), ("n", ctypes.c_uint64)]


class TuningC(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("threads", ctypes.c_int), ("spl", ctypes.c_int),
                ("split_rounds", ctypes.c_uint32), ("ms", ctypes.c_float), ("trials", ctypes.c_uint32)]


class PlanInfoC(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("threads", ctypes.c_uint32), ("spl", ctypes.c_uint32),
                ("lds_words", ctypes.c_uint32), ("grid", ctypes.c_uint32), ("items", ctypes.c_uint32),
                ("jumps", ctypes.c_uint32)]


class RequestC(ctypes.Structure):
    _fields_ = [("gen", ctypes.c_uint32), ("kind", ctypes.c_uint32),
                ("n", ctypes.c_uint64), ("out", ctypes.c_void_p)]


def _request_dtype():
    import numpy as np
    return np.dtype({"names": ["gen", "kind", "n", "out"],
                     "formats": [np.uint32, np.uint32, np.uint64, np.uint64],
                     "offsets": [RequestC.gen.offset, RequestC.kind.offset, RequestC.n.offset, RequestC.out.offset],
                     "itemsize": ctypes.sizeof(RequestC)})


REQUEST_DTYPE = _request_dtype()

# Every symbol the header declares, with its ctypes signature.
_SIGNATURES = {
    "mtgp_state_words": (ctypes.c_uint32, [ctypes.c_uint32]),
    "mtgp_create": (ctypes.c_void_p, [ctypes.POINTER(ParamSetC), ctypes.c_uint32]),
    "mtgp_generate_uint32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "mtgp_generate_float32_1to2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "mtgp_generate_float32_0to1": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "mtgp_generate_normal_float32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "mtgp_destroy": (None, [ctypes.c_void_p]),
    "mtgp_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "mtgp_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "mtgp_batch_create": (ctypes.c_void_p, [ctypes.POINTER(ParamSetC), ctypes.c_void_p, ctypes.c_uint32]),
    "mtgp_batch_generate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RequestC), ctypes.c_uint32, ctypes.c_void_p]),
    "mtgp_batch_generate_plain": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RequestC), ctypes.c_uint32, ctypes.c_void_p]),
    "mtgp_batch_generate_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RequestC), ctypes.c_uint32,
                                                  ctypes.c_void_p]),
    "mtgp_batch_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "mtgp_batch_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64]),
    "mtgp_batch_size": (ctypes.c_uint32, [ctypes.c_void_p]),
    "mtgp_batch_destroy": (None, [ctypes.c_void_p]),
    "mtgp_batch_plan_create": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.POINTER(RequestC), ctypes.c_uint32]),
    "mtgp_plan_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mtgp_plan_launch_phase": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "mtgp_plan_describe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mtgp_batch_prepare_split": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "mtgp_server_set_split": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32]),
    "mtgp_plan_items": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "mtgp_batch_set_split": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "mtgp_set_split": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "mtgp_server_create": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                             ctypes.c_uint32, ctypes.c_void_p]),
    "mtgp_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "mtgp_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CompletionC), ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_uint32)]),
    "mtgp_server_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "mtgp_server_pending": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32)]),
    "mtgp_server_destroy": (None, [ctypes.c_void_p]),
    "mtgp_search_params": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint32, ctypes.POINTER(ParamSetC), ctypes.POINTER(SearchStatsC)]),
    "mtgp_equidistribution": (ctypes.c_int, [ctypes.POINTER(ParamSetC), ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
    "mtgp_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RequestC), ctypes.c_uint32, ctypes.c_void_p,
                                           ctypes.c_uint32, ctypes.POINTER(TuningC)]),
    "mtgp_plan_destroy": (None, [ctypes.c_void_p]),
    "mtgp_batch_set_launch": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_int] * 5),
    "mtgp_set_launch": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_int] * 4),
    "mtgp_last_error": (ctypes.c_int, []),
    "mtgp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1005_4973_amd/build.py "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().mtgp_strerror(code).decode()
    except RuntimeError:
        return str(code)


def state_words(mexp: int) -> int:
    return int(lib().mtgp_state_words(mexp))


class FoundParams(NamedTuple):
    """A parameter set from search_params (same fields as the parameter sets
    the other calls take)."""
    mexp: int
    pos: int
    sh1: int
    sh2: int
    param_tbl: tuple
    temper_tbl: tuple


def search_params(mexp: int, id: int = 0, seed: int = 1, max_draws: int = 1 << 20, threads: int = 0):
    """Recursion-parameter search of period 2^mexp - 1 with `id` embedded
    (mtgp_search_params; host only). Returns (FoundParams, stats dict)."""
    p = ParamSetC()
    st = SearchStatsC()
    rc = lib().mtgp_search_params(mexp, id & 0xFFFFFFFF, seed, max_draws, threads, ctypes.byref(p), ctypes.byref(st))
    _check(rc, "mtgp_search_params")
    stats = {"draws": st.draws, "evaluated": st.evaluated, "full_degree": st.full_degree,
             "sieve_passed": st.sieve_passed, "seconds": round(st.seconds, 3)}
    return FoundParams(p.mexp, p.pos, p.sh1, p.sh2, tuple(p.param_tbl), tuple(p.temper_tbl)), stats


def equidistribution(ps, tempered: bool = True, vmax: int = 32):
    """Dimensions of equidistribution k(1) .. k(vmax) (section 3.4) of a
    full-period parameter set, and the total dimension defect over them
    (mtgp_equidistribution; host only). Returns (list of k(v), delta)."""
    k = (ctypes.c_uint32 * vmax)()
    d = ctypes.c_uint32()
    rc = lib().mtgp_equidistribution(ctypes.byref(_param_c(ps)), 1 if tempered else 0, vmax, k, ctypes.byref(d))
    _check(rc, "mtgp_equidistribution")
    return list(k), int(d.value)


def _param_c(ps) -> ParamSetC:
    p = ParamSetC()
    p.mexp, p.pos, p.sh1, p.sh2 = ps.mexp, ps.pos, ps.sh1, ps.sh2
    for i in range(16):
        p.param_tbl[i] = ps.param_tbl[i]
        p.temper_tbl[i] = ps.temper_tbl[i]
    return p


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc: int, what: str):
    if rc != MTGP_OK:
        raise MTGPError(rc, what)


_DTYPE = {KIND_UINT32: torch.int32, KIND_FLOAT32_1TO2: torch.float32, KIND_FLOAT32_0TO1: torch.float32,
          KIND_NORMAL_FLOAT32: torch.float32}
_GEN_FN = {KIND_UINT32: "mtgp_generate_uint32", KIND_FLOAT32_1TO2: "mtgp_generate_float32_1to2",
           KIND_FLOAT32_0TO1: "mtgp_generate_float32_0to1", KIND_NORMAL_FLOAT32: "mtgp_generate_normal_float32"}


def _out_tensor(n: int, kind: int, out: Optional[torch.Tensor], device) -> torch.Tensor:
    if out is None:
        return torch.empty(n, dtype=_DTYPE[kind], device=device)
    if not out.is_cuda or out.element_size() != 4 or not out.is_contiguous() or out.numel() < n:
        raise ValueError("out must be a contiguous 4-byte CUDA tensor with at least n elements")
    return out


class Generator:
    """One MTGP generator (mtgp_create). Outputs land in torch tensors."""

    def __init__(self, ps, seed: int):
        self.ps = ps
        self._h = lib().mtgp_create(ctypes.byref(_param_c(ps)), seed & 0xFFFFFFFF)
        if not self._h:
            raise MTGPError(lib().mtgp_last_error(), "mtgp_create")
        self.nwords = state_words(ps.mexp)

    def generate(self, n: int, kind: int = KIND_UINT32, out: Optional[torch.Tensor] = None,
                 stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        out = _out_tensor(n, kind, out, "cuda")
        rc = getattr(lib(), _GEN_FN[kind])(self._h, n, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
        _check(rc, _GEN_FN[kind])
        return out[:n] if out.numel() != n else out

    def generate_uint32(self, n, out=None, stream=None):
        return self.generate(n, KIND_UINT32, out, stream)

    def generate_float32_1to2(self, n, out=None, stream=None):
        return self.generate(n, KIND_FLOAT32_1TO2, out, stream)

    def generate_float32_0to1(self, n, out=None, stream=None):
        return self.generate(n, KIND_FLOAT32_0TO1, out, stream)

    def generate_normal_float32(self, n, out=None, stream=None):
        return self.generate(n, KIND_NORMAL_FLOAT32, out, stream)

    def set_split(self, max_rounds: int):
        """Split calls longer than max_rounds rounds into jump-ahead segments (0: off)."""
        _check(lib().mtgp_set_split(self._h, max_rounds), "mtgp_set_split")

    def set_launch(self, mode: int = -1, threads: int = 0, spl: int = 1, lds_words: int = 0):
        """Override the launch shape (mode -1 restores the automatic choice)."""
        _check(lib().mtgp_set_launch(self._h, mode, threads, spl, lds_words), "mtgp_set_launch")

    def get_state(self):
        import numpy as np
        words = np.zeros(self.nwords, dtype=np.uint32)
        consumed = ctypes.c_uint64(0)
        _check(lib().mtgp_get_state(self._h, words.ctypes.data, ctypes.byref(consumed)), "mtgp_get_state")
        return words, consumed.value

    def set_state(self, words, consumed: int = 0):
        import numpy as np
        w = np.ascontiguousarray(np.asarray(words, dtype=np.uint32))
        if w.size != self.nwords:
            raise ValueError("state must have N words")
        _check(lib().mtgp_set_state(self._h, w.ctypes.data, consumed), "mtgp_set_state")

    def close(self):
        if getattr(self, "_h", None):
            lib().mtgp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many resident generators (mtgp_batch_create); one persistent launch per call."""

    def __init__(self, params: Sequence, seeds: Sequence[int]):
        import numpy as np
        if len(params) != len(seeds) or len(params) == 0:
            raise ValueError("params and seeds must be non-empty and of equal length")
        arr = (ParamSetC * len(params))(*[_param_c(p) for p in params])
        sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint32))
        self._h = lib().mtgp_batch_create(arr, sd.ctypes.data, len(params))
        if not self._h:
            raise MTGPError(lib().mtgp_last_error(), "mtgp_batch_create")
        self.params = list(params)
        self.count = len(params)

    @staticmethod
    def _reqs(requests: Iterable):
        """Requests as the C array, its length and the output tensors it points
        into. A tensor output is checked like Generator.generate's (a contiguous
        4-byte CUDA tensor on the current device with at least n elements); an
        integer output is a device address that the caller vouches for: at
        least 4 n bytes, 4-byte aligned, alive until the work has run."""
        reqs = list(requests)
        arr = (RequestC * max(1, len(reqs)))()
        tensors = []
        for i, (gen, kind, n, out) in enumerate(reqs):
            if isinstance(out, torch.Tensor):
                _out_tensor(n, kind, out, "cuda")
                if out.device.index != torch.cuda.current_device():
                    raise ValueError("out must be on the current CUDA device")
                ptr = out.data_ptr()
                tensors.append(out)
            else:
                ptr = int(out)
            arr[i].gen, arr[i].kind, arr[i].n, arr[i].out = gen, kind, n, ptr
        return arr, len(reqs), tensors

    def generate(self, requests: Iterable, stream: Optional[torch.cuda.Stream] = None):
        """requests: iterable of (gen, kind, n, out tensor or device address). With a split
        limit set, a call holding a longer request runs as jump-ahead segments. The call is
        stream-ordered: the output tensors must outlive the work (hold them, or use them on
        the same stream, until it has run)."""
        arr, k, _ = self._reqs(requests)
        _check(lib().mtgp_batch_generate(self._h, arr, k, _stream_ptr(stream)), "mtgp_batch_generate")

    def generate_arrays(self, gens, kinds, ns, ptrs, stream: Optional[torch.cuda.Stream] = None):
        """Same as generate, with the requests as equal-length integer arrays
        (generator, kind, n, output device address): no per-request Python work.
        The addresses are the caller's responsibility, as integer outputs of
        generate are (at least 4 n bytes each, 4-byte aligned, alive until the
        work has run); the library checks alignment and nothing else about them."""
        import numpy as np
        k = len(gens)
        arr = np.zeros(k, dtype=REQUEST_DTYPE)
        arr["gen"] = gens
        arr["kind"] = kinds
        arr["n"] = ns
        arr["out"] = ptrs
        rc = lib().mtgp_batch_generate(self._h, ctypes.cast(arr.ctypes.data, ctypes.POINTER(RequestC)), k,
                                       _stream_ptr(stream))
        _check(rc, "mtgp_batch_generate")

    def generate_static(self, requests: Iterable, stream: Optional[torch.cuda.Stream] = None):
        """mtgp_batch_generate_static: the same call without jump-ahead and without
        allocation (work items in the library's fixed per-GPU scratch)."""
        arr, k, _ = self._reqs(requests)
        _check(lib().mtgp_batch_generate_static(self._h, arr, k, _stream_ptr(stream)), "mtgp_batch_generate_static")

    def generate_plain(self, requests: Iterable, stream: Optional[torch.cuda.Stream] = None):
        arr, k, _ = self._reqs(requests)
        _check(lib().mtgp_batch_generate_plain(self._h, arr, k, _stream_ptr(stream)), "mtgp_batch_generate_plain")

    def set_split(self, max_rounds: int):
        """Split requests longer than max_rounds rounds into jump-ahead segments (0: off), in plans
        and in eager generate calls (such a call runs as a one-off plan)."""
        _check(lib().mtgp_batch_set_split(self._h, max_rounds), "mtgp_batch_set_split")

    def autotune(self, requests: Iterable, reps: int = 5, stream: Optional[torch.cuda.Stream] = None) -> dict:
        """Time candidate launch shapes and split limits on these requests and keep
        the fastest (mtgp_batch_autotune); streams are left where they were."""
        arr, k, _ = Batch._reqs(requests)
        t = TuningC()
        _check(lib().mtgp_batch_autotune(self._h, arr, k, _stream_ptr(stream), reps, ctypes.byref(t)),
               "mtgp_batch_autotune")
        return {"mode": t.mode, "threads": t.threads, "spl": t.spl, "split_rounds": t.split_rounds,
                "ms": round(t.ms, 4), "trials": t.trials}

    def plan(self, requests: Iterable) -> "Plan":
        """Capture the persistent launch for a fixed request list (see Plan)."""
        return Plan(self, requests)

    def set_launch(self, mode: int = -1, threads: int = 0, spl: int = 1, lds_words: int = 0, grid: int = 0):
        """Override the persistent launch shape (mode -1 restores the automatic choice)."""
        _check(lib().mtgp_batch_set_launch(self._h, mode, threads, spl, lds_words, grid), "mtgp_batch_set_launch")

    def prepare_split(self, gens):
        """Find and cache the orbit annihilators jump-ahead needs for these
        generators (mtgp_batch_prepare_split; synchronous, threaded)."""
        import numpy as np
        g = np.ascontiguousarray(np.asarray(list(gens), dtype=np.uint32))
        _check(lib().mtgp_batch_prepare_split(self._h, g.ctypes.data if g.size else None, g.size),
               "mtgp_batch_prepare_split")

    def get_state(self, gen: int):
        import numpy as np
        words = np.zeros(state_words(self.params[gen].mexp), dtype=np.uint32)
        consumed = ctypes.c_uint64(0)
        _check(lib().mtgp_batch_get_state(self._h, gen, words.ctypes.data, ctypes.byref(consumed)),
               "mtgp_batch_get_state")
        return words, consumed.value

    def set_state(self, gen: int, words, consumed: int = 0):
        import numpy as np
        w = np.ascontiguousarray(np.asarray(words, dtype=np.uint32))
        _check(lib().mtgp_batch_set_state(self._h, gen, w.ctypes.data, consumed), "mtgp_batch_set_state")

    def close(self):
        if getattr(self, "_h", None):
            lib().mtgp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A fixed request list whose persistent launch is captured in a HIP graph
    (mtgp_batch_plan_create); each launch() continues every listed stream.
    Every replay writes the listed outputs: the plan holds its output tensors
    for its lifetime (integer addresses stay the caller's to keep valid)."""

    def __init__(self, batch: Batch, requests: Iterable):
        arr, k, self._outs = Batch._reqs(requests)
        self.batch = batch
        self._h = lib().mtgp_batch_plan_create(batch._h, arr, k)
        if not self._h:
            raise MTGPError(lib().mtgp_last_error(), "mtgp_batch_plan_create")

    def launch(self, stream: Optional[torch.cuda.Stream] = None):
        _check(lib().mtgp_plan_launch(self._h, _stream_ptr(stream)), "mtgp_plan_launch")

    def launch_phase(self, phase: int, stream: Optional[torch.cuda.Stream] = None):
        """PHASE_PREPARE (segment start states) or PHASE_GENERATE; a replay is
        both, in that order (mtgp_plan_launch_phase)."""
        _check(lib().mtgp_plan_launch_phase(self._h, int(phase), _stream_ptr(stream)), "mtgp_plan_launch_phase")

    def describe(self) -> dict:
        """The resolved launch of the generation kernel and the work item and
        jump counts (mtgp_plan_describe)."""
        d = PlanInfoC()
        _check(lib().mtgp_plan_describe(self._h, ctypes.byref(d)), "mtgp_plan_describe")
        return {f: getattr(d, f) for f, _ in PlanInfoC._fields_}

    def items(self):
        """(output device addresses, output counts) of the generation launch's
        work items in queue order, as uint64 arrays (mtgp_plan_items)."""
        import numpy as np
        k = self.describe()["items"]
        outs = np.zeros(max(k, 1), dtype=np.uint64)
        ns = np.zeros(max(k, 1), dtype=np.uint64)
        got = lib().mtgp_plan_items(self._h, outs.ctypes.data, ns.ctypes.data, k)
        if got < 0:
            raise MTGPError(got, "mtgp_plan_items")
        return outs[:got], ns[:got]

    def close(self):
        if getattr(self, "_h", None):
            lib().mtgp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
