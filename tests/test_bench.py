"""Host logic of bench.py (CPU): the round width it assumes for a tuned
launch shape (the library's rule: the largest allowed steps per lane s with
lanes * s <= N - M), and the rule that reports counted HBM traffic only while
the kernel sources and the split limit match those of the counter run."""
import hashlib
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    argv = sys.argv
    sys.argv = ["bench.py"]
    try:
        import bench as b
    finally:
        sys.argv = argv
    return b


@pytest.mark.parametrize("N,M,launch,W", [
    (351, 78, {"mode": 0, "threads": 256, "spl": 4}, 256),       # 256 lanes, one step
    (1391, 100, {"mode": 0, "threads": 256, "spl": 4}, 1024),    # 256 lanes x 4 steps
    (726, 6, {"mode": 0, "threads": 256, "spl": 4}, 512),        # 256 x 2 (4 would exceed N - M)
    (726, 720, {"mode": 0, "threads": 256, "spl": 4}, 6),        # narrower than the workgroup
    (351, 78, {"mode": 4, "threads": 512, "spl": 1}, 273),       # 512 lanes: W = N - M
    (351, 78, {"mode": 1, "threads": 256, "spl": 8}, 256),       # wavefront form: 64 x 4
    (1391, 2, {"mode": 5, "threads": 256, "spl": 16}, 1024),     # 64 x 16, basis flag ignored
    (351, 78, {"mode": 2, "threads": 256, "spl": 2}, 64),        # chunked form: a round is a chunk
    (1391, 300, {"mode": 2, "threads": 64, "spl": 1}, 64),
])
def test_round_width(bench, N, M, launch, W):
    assert bench.round_width(N, M, launch) == W
    with pytest.raises(ValueError):
        bench.round_width(N, M, {"mode": -1, "threads": 0, "spl": 0})


LAUNCH = {"mode": 2, "threads": 64, "spl": 2, "lds_words": 2048, "grid": 2048}


def _digest(bench):
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _profile(tmp_path, hash16, split, launch):
    p = tmp_path / f"prof_{hash16}_{split}_{launch['grid']}.md"
    p.write_text(f"# t\n\nkernel_source_sha256_16: {hash16}  (sources)\nsplit_rounds: {split}\n"
                 f"launch: {' '.join(f'{k}={launch[k]}' for k in ('mode', 'threads', 'spl', 'lds_words', 'grid'))}\n"
                 f"traffic_bytes_per_launch: 123456\n")
    return str(p)


def test_traffic_reported_only_for_matching_sources_and_split(bench, tmp_path):
    d = _digest(bench)
    p = _profile(tmp_path, d, 2048, LAUNCH)
    assert bench.measured_traffic(LAUNCH, 2048, p) == 123456
    assert bench.measured_traffic(LAUNCH, 1024, p) is None
    assert bench.measured_traffic(LAUNCH, 2048, _profile(tmp_path, "0" * 16, 2048, LAUNCH)) is None
    assert bench.measured_traffic(LAUNCH, 2048, str(tmp_path / "missing.md")) is None


def test_traffic_needs_the_same_resolved_launch(bench, tmp_path):
    """A counter run taken under one launch does not stand for another: the
    shape sets the round unit the split limit counts in, and the grid and
    ring the kernel's own traffic."""
    p = _profile(tmp_path, _digest(bench), 4096, LAUNCH)
    assert bench.measured_traffic(dict(LAUNCH), 4096, p) == 123456
    for k, v in (("mode", 0), ("grid", 2304), ("lds_words", 1024), ("spl", 1), ("threads", 256)):
        assert bench.measured_traffic({**LAUNCH, k: v}, 4096, p) is None


def test_roofline_block_fractions(bench):
    ceil = {"waves": 2048, "probe_4B_plain": 6000.0, "probe_4B_nontemporal": 5800.0, "probe_16B_plain": 6100.0}
    blk = bench.roofline_block(8_000_000_000, 2.0, 2.5, LAUNCH, None, ceil)
    assert blk["achieved"] == 4000.0 and blk["frac"] == 0.5
    assert blk["end_to_end"]["frac"] == 0.4
    assert blk["frac_of_store_ceiling"] == round(4000.0 / 6000.0, 4)
    assert blk["kernel"] == "mtgp_chunk_kernel<2048, 2, 1>" and blk["launch"] == LAUNCH


def test_more_than_one_gpu_is_refused_before_any_device_work():
    """--gpus N > 1 ends with a message and a non-zero status, and without a
    GPU (this test runs on the CPU), so nothing was set up on a device first."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode != 0
    assert "one GPU only" in res.stderr and "--gpus 2" in res.stderr
    assert res.stdout == ""
