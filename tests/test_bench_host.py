"""Host logic of bench.py: the algorithmic work per point that the roofline divides by,
the kernel names the counter summaries are matched on, and the rule that a traffic
figure is reported only for the kernel sources it was measured on.  CPU only."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_1709_05418_amd import synth  # noqa: E402


@pytest.mark.parametrize("K,W,H", [(10, 200, 3), (6, 64, 3), (2, 16, 4)])
def test_macs_per_point_is_the_weight_count(K, W, H):
    # every weight multiplies once per point (block 1 has no W1, R9): the MAC count is the
    # number of weight entries of the network, counted here from its layer shapes
    weights = sum(r * c for _, r, c in synth.layer_shapes(K, W, H) if c)
    assert bench.macs_per_point(K, W, H) == weights
    if (K, W, H) == (10, 200, 3):
        assert 2 * weights == 2_584_400


def test_fp8_macs_are_the_w_by_w_layers():
    K, W, H = 10, 200, 3
    sq = sum(r * c for name, r, c in synth.layer_shapes(K, W, H) if c and r == W and c == W)
    assert bench.fp8_macs_per_point(K, W, H) == sq == 840_000


@pytest.mark.parametrize("raw,short", [
    ("k_fused_reg<13, 4, false, false>", "k_fused_reg<13,4>"),
    ("k_fused_reg<13,8,true,true>", "k_fused_reg<13,8>"),
    ("k_fused_reg<13,4>", "k_fused_reg<13,4>"),
    ("k_gather<float>", "k_gather<float>"),
    ("k_gemm", "k_gemm"),
])
def test_short_kernel_name(raw, short):
    assert bench.short_kernel_name(raw) == short


def _summary(path, kernel, sha, traffic):
    with open(path, "w") as f:
        f.write("# counters\n")
        f.write(f"kernel: {kernel}\ngrid: 0 (one workgroup per tile)\n")
        f.write(f"kernel_sources_sha256: {sha}\ntraffic_bytes_per_launch: {traffic}\n")


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    sha = bench.kernel_sources_sha256()
    _summary(tmp_path / "k_fused_reg_bf16_x_hbm_traffic.txt", "k_fused_reg<13, 4, false, false>",
             sha, 123456)
    assert bench.measured_traffic("k_fused_reg<13,4>") == (123456, "0 (one workgroup per tile)")
    assert bench.measured_traffic("k_fused_reg<13,8>") == (None, "")
    _summary(tmp_path / "k_fused_reg_bf16_x_hbm_traffic.txt", "k_fused_reg<13,4>", "0" * 64, 1)
    assert bench.measured_traffic("k_fused_reg<13,4>") == (None, "")
