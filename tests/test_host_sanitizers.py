"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's device-free C++ sources (F2 polynomial arithmetic, the
parameter search, the dimension of equidistribution), the request loop over a
stand-in device (with and without split ticks), and the C oracle are
built with g++/gcc, -fsanitize=address,undefined and no recovery, and run
their self-tests (tests/host/*): any leak, out-of-bounds access, overflow of
a signed type or other undefined behaviour ends the run with an error.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1005_4973_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def build_and_run(tmp_path, compiler, sources, extra, expect):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not found")
    exe = str(tmp_path / "selftest")
    cmd = [compiler] + SAN + extra + ["-o", exe] + sources + ["-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0 and expect in run.stdout, run.stdout[-4000:] + run.stderr[-4000:]


def test_library_host_code_under_sanitizers(tmp_path):
    srcs = [os.path.join(ROOT, "tests", "host", "host_selftest.cpp")] + \
        [os.path.join(CSRC, f) for f in ("mtgp_f2.cpp", "mtgp_dc.cpp", "mtgp_equidist.cpp")]
    build_and_run(tmp_path, "g++", srcs, ["-std=c++17", "-I", os.path.join(ROOT, "include")], "host selftest ok")


def test_request_loop_under_sanitizers(tmp_path):
    """The request loop's host logic over a stand-in device (tests/host/mockhip)."""
    srcs = [os.path.join(ROOT, "tests", "host", "serve_selftest.cpp"),
            os.path.join(CSRC, "mtgp_serve.cpp"), os.path.join(CSRC, "mtgp_f2.cpp")]
    build_and_run(tmp_path, "g++", srcs, ["-std=c++17", "-I", os.path.join(ROOT, "tests", "host", "mockhip"),
                                          "-I", os.path.join(ROOT, "include"), "-I", CSRC], "serve selftest ok")


def test_split_ticks_under_sanitizers(tmp_path):
    """The request loop's split ticks (refused by the library, built here with
    MTGP_SERVE_SPLIT_TICKS=1) over the stand-in device: coverage, order,
    segment flags and staging-ring disjointness."""
    srcs = [os.path.join(ROOT, "tests", "host", "split_selftest.cpp"),
            os.path.join(CSRC, "mtgp_serve.cpp"), os.path.join(CSRC, "mtgp_f2.cpp")]
    build_and_run(tmp_path, "g++", srcs, ["-std=c++17", "-DMTGP_SERVE_SPLIT_TICKS=1",
                                          "-I", os.path.join(ROOT, "tests", "host", "mockhip"),
                                          "-I", os.path.join(ROOT, "include"), "-I", CSRC], "split selftest ok")


def test_oracle_under_sanitizers(tmp_path):
    srcs = [os.path.join(ROOT, "tests", "host", "oracle_selftest.c"),
            os.path.join(ROOT, "oracle", "mtgp_oracle.c"), os.path.join(ROOT, "oracle", "f2.c")]
    build_and_run(tmp_path, "gcc", srcs, ["-std=c11", "-fno-fast-math"], "oracle selftest ok")
