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


@pytest.mark.parametrize("N,M,tuning,W", [
    (351, 78, {"mode": -1, "threads": 0, "spl": 0}, 256),       # automatic: 256 lanes, one step
    (1391, 100, {"mode": -1, "threads": 0, "spl": 0}, 1024),    # 256 lanes x 4 steps
    (726, 6, {"mode": -1, "threads": 0, "spl": 0}, 512),        # 256 x 2 (4 would exceed N - M)
    (726, 720, {"mode": -1, "threads": 0, "spl": 0}, 6),        # narrower than the workgroup
    (351, 78, {"mode": 4, "threads": 512, "spl": 1}, 273),      # 512 lanes: W = N - M
    (351, 78, {"mode": 1, "threads": 256, "spl": 8}, 256),      # wavefront form: 64 x 4
    (1391, 2, {"mode": 5, "threads": 256, "spl": 16}, 1024),    # 64 x 16, basis flag ignored
    (351, 78, {"mode": 2, "threads": 256, "spl": 2}, 64),       # chunked form: a round is a chunk
    (1391, 300, {"mode": 2, "threads": 64, "spl": 1}, 64),
])
def test_round_width(bench, N, M, tuning, W):
    assert bench.round_width(N, M, tuning) == W


def test_traffic_reported_only_for_matching_sources_and_split(bench, tmp_path, monkeypatch):
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    digest = h.hexdigest()[:16]

    def profile(hash16, split):
        p = tmp_path / f"prof_{hash16}_{split}.md"
        p.write_text(f"# t\n\nkernel_source_sha256_16: {hash16}  (sources)\n"
                     f"tuning: split_rounds={split} mode=-1 threads=0 spl=0\ntraffic_bytes_per_launch: 123456\n")
        return str(p)

    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", profile(digest, 2048))
    assert bench.measured_traffic({"split_rounds": 2048}) == 123456
    assert bench.measured_traffic({"split_rounds": 1024}) is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", profile("0" * 16, 2048))
    assert bench.measured_traffic({"split_rounds": 2048}) is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic({"split_rounds": 2048}) is None


def test_traffic_needs_matching_launch_mode(bench, tmp_path):
    """A counter run taken under one launch mode does not stand for another:
    the round unit the split limit counts in depends on it."""
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    p = tmp_path / "prof.md"
    p.write_text(f"kernel_source_sha256_16: {h.hexdigest()[:16]}\n"
                 f"tuning: split_rounds=4096 mode=2 threads=256 spl=2\ntraffic_bytes_per_launch: 99\n")
    assert bench.measured_traffic({"split_rounds": 4096, "mode": 2}, str(p)) == 99
    assert bench.measured_traffic({"split_rounds": 4096, "mode": 0}, str(p)) is None


def test_roofline_block_fractions(bench):
    blk = bench.roofline_block(8_000_000_000, 2.0, 2.5, {"mode": 2, "threads": 256, "spl": 2}, None, 6000.0)
    assert blk["achieved"] == 4000.0 and blk["frac"] == 0.5
    assert blk["end_to_end"]["frac"] == 0.4
    assert blk["frac_of_store_ceiling"] == round(4000.0 / 6000.0, 4)
    assert "chunk" in blk["kernel"]
