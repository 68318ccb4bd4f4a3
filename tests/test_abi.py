"""The C-ABI library builds, loads and exports every symbol include/mtgp.h
declares (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mtgp.h")
LIB = os.path.join(ROOT, "paper_1005_4973_amd", "libmtgp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mtgp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mtgp_create", "mtgp_generate_uint32", "mtgp_generate_float32_1to2",
                 "mtgp_generate_float32_0to1", "mtgp_destroy", "mtgp_batch_generate"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1005_4973_amd import build
        build.build()
    import torch  # noqa: F401  (same HIP runtime as the binding uses)
    L = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_signatures_cover_header():
    from paper_1005_4973_amd import mtgp
    assert sorted(mtgp._SIGNATURES) == declared_functions()


def test_host_only_calls():
    """Calls that touch no device: state-size query, error strings, NULL-safe destroy."""
    from paper_1005_4973_amd import mtgp
    L = mtgp.lib()
    assert L.mtgp_state_words(11213) == 351
    assert L.mtgp_state_words(23209) == 726
    assert L.mtgp_state_words(44497) == 1391
    assert L.mtgp_state_words(64) == 0
    assert L.mtgp_strerror(-1) == b"invalid argument or parameter set"
    L.mtgp_destroy(None)
    L.mtgp_batch_destroy(None)
    L.mtgp_plan_destroy(None)
    # NULL handles are rejected before any device work
    assert L.mtgp_plan_launch_phase(None, mtgp.PHASE_GENERATE, None) == mtgp.MTGP_EINVAL
    assert L.mtgp_batch_autotune(None, None, 1, None, 3, None) == mtgp.MTGP_EINVAL
    assert L.mtgp_batch_set_split(None, 8) == mtgp.MTGP_EINVAL
    # the request loop: bad creation arguments give NULL, NULL handles EINVAL
    assert L.mtgp_server_create(None, None, 1 << 20, 1 << 10, 2, None) is None
    assert L.mtgp_server_submit(None, None, 1) == mtgp.MTGP_EINVAL
    assert L.mtgp_server_poll(None, None, 0, None) == mtgp.MTGP_EINVAL
    assert L.mtgp_server_release(None, None, 1) == mtgp.MTGP_EINVAL
    assert L.mtgp_server_pending(None, None, None, None) == mtgp.MTGP_EINVAL
    L.mtgp_server_destroy(None)
    # host-only analyses reject NULL outputs
    assert L.mtgp_search_params(11213, 1, 1, 10, 1, None, None) == mtgp.MTGP_EINVAL
    assert L.mtgp_equidistribution(None, 1, 32, None, None) == mtgp.MTGP_EINVAL


def test_create_rejects_bad_parameters_before_touching_the_device():
    from paper_1005_4973_amd import inputs as I
    from paper_1005_4973_amd import mtgp
    ps = I.single_stream()[0][0]
    bad = [
        I.ParamSet(ps.mexp, 1, ps.sh1, ps.sh2, ps.param_tbl, ps.temper_tbl),          # M < 2
        I.ParamSet(ps.mexp, 351, ps.sh1, ps.sh2, ps.param_tbl, ps.temper_tbl),        # M > N-1
        I.ParamSet(ps.mexp, ps.pos, 32, ps.sh2, ps.param_tbl, ps.temper_tbl),         # shift > 31
        I.ParamSet(64, 2, 1, 1, ps.param_tbl, ps.temper_tbl),                         # N < 3
        I.ParamSet(ps.mexp, ps.pos, ps.sh1, ps.sh2, (1,) + ps.param_tbl[1:], ps.temper_tbl),  # tbl[0] != 0
        I.ParamSet(ps.mexp, ps.pos, ps.sh1, ps.sh2, ps.param_tbl,
                   ps.temper_tbl[:5] + (ps.temper_tbl[5] ^ 1,) + ps.temper_tbl[6:]),  # not linear
    ]
    for b in bad:
        with pytest.raises(mtgp.MTGPError) as e:
            mtgp.Generator(b, 1)
        assert e.value.code == mtgp.MTGP_EINVAL


def test_request_tensors_are_checked_before_the_call():
    """Batch requests with tensor outputs get the same checks as a single
    generator's output (CUDA, contiguous, 4-byte elements, at least n of
    them): a bad tensor is refused in Python, before any pointer reaches the
    library; integer addresses pass through unchecked (the caller's)."""
    import torch
    from paper_1005_4973_amd import mtgp
    host = torch.empty(100, dtype=torch.int32)
    for bad in (host, host.to(torch.int16), host[::2]):
        with pytest.raises(ValueError):
            mtgp.Batch._reqs([(0, mtgp.KIND_UINT32, 10, bad)])
    arr, k, tensors = mtgp.Batch._reqs([(0, mtgp.KIND_UINT32, 10, 0x1000), (1, mtgp.KIND_FLOAT32_0TO1, 0, 0x2000)])
    assert k == 2 and tensors == [] and arr[0].out == 0x1000 and arr[1].n == 0
