"""Store-only probe (libmtgp_probe.so): the write ceiling of an output layout.

A measurement aid for the benchmark, outside the generator library: it times
a kernel that only stores, filling the same output ranges in the same queue
order as a plan's generation launch, with one 4-byte store per lane (the
generation kernels' pattern) or wider ones.
"""
import ctypes
import os

import numpy as np

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmtgp_probe.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_PATH):
            raise RuntimeError(f"{_PATH} is not built: run paper_1005_4973_amd/build.py")
        import torch  # noqa: F401  (same HIP runtime as the rest)
        _lib = ctypes.CDLL(_PATH)
        _lib.mtgp_probe_store_ms.restype = ctypes.c_int
        _lib.mtgp_probe_store_ms.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p,
                                             ctypes.c_void_p]
    return _lib


def store_ms(outs, ns, waves, width=1, nontemporal=False, reps=3, stream=None):
    """Average ms of `reps` store-only launches of `waves` wavefronts over the
    ranges (outs[i], ns[i] words), after one warm-up launch."""
    o = np.ascontiguousarray(np.asarray(outs, dtype=np.uint64))
    n = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64))
    if o.shape != n.shape or o.size == 0:
        raise ValueError("outs and ns must be non-empty and of equal length")
    ms = ctypes.c_float(0.0)
    sp = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    rc = lib().mtgp_probe_store_ms(o.ctypes.data, n.ctypes.data, o.size, waves, width, int(nontemporal), reps, sp,
                                   ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"mtgp_probe_store_ms failed ({rc})")
    return ms.value
