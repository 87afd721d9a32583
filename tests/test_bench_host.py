"""Host logic of bench.py: the flop tallies per (sample, bin) pair that the
roofline uses, and the reading of committed counter summaries, which must
give nothing once the kernel sources no longer match the fingerprint the
summary records."""
import os
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(__file__), ".."))
import bench  # noqa: E402


def test_tile_flop_tally():
    # phase 19, phasor 34 (fixed tally), detector 0: 8, each further detector 14
    assert bench.flops_per_pair(3) == 19 + 34 + 8 + 2 * 14 == 89
    assert bench.flops_per_pair(1) == 19 + 34 + 8
    # mixed: the phasor becomes the reduction to a fractional turn (1 add)
    assert bench.flops_per_pair(3, mixed=True) == 19 + 1 + 8 + 2 * 14
    # direct form: 13 per detector plus 6 for each rotated one
    assert bench.flops_per_pair(3, direct=True) == 19 + 34 + 13 + 2 * 19


def test_relbin_flop_tally():
    assert bench.rb_flops_per_pair(3) == 19 + 54 * 3 + 2 * 2 == 185
    assert bench.rb_flops_per_pair(1, mixed=True) == 19 + 21


def _summary(tmp_path, sha):
    text = (f"# test\n\nkernel_source_sha256: {sha}\n\n"
            "traffic_bytes_per_launch_fp64@512x6: 3.25e+07\nexecuted_fp64_flops_per_launch_fp64@512x6: 7.8e+10\n"
            "executed_fp64_flops_per_launch_fp64@256x6: 7.9e+10\n")
    path = tmp_path / "summary.md"
    path.write_text(text)
    return str(path)


def test_profile_values_follow_the_fingerprint(tmp_path):
    # an absolute summary path is read as given, checked against the tile kernel's sources
    tile = bench.PROFILE_SUMMARY
    good = _summary(tmp_path, bench.kernel_fingerprint(tile))
    assert bench.measured_traffic("fp64@512x6", good, tile) == pytest.approx(3.25e7)
    assert bench.measured_executed_flops("fp64@512x6", good, tile) == pytest.approx(7.8e10)
    assert bench.measured_executed_flops("fp64@256x6", good, tile) == pytest.approx(7.9e10)
    assert bench.measured_traffic("fp64@256x6", good, tile) is None
    assert bench.measured_traffic("mixed@512x6", good, tile) is None
    stale = _summary(tmp_path, "0" * 64)
    assert bench.measured_traffic("fp64@512x6", stale, tile) is None
    assert bench.measured_executed_flops("fp64@512x6", stale, tile) is None
    assert bench.measured_traffic("fp64@512x6", str(tmp_path / "missing.md"), tile) is None
    # another kernel's sources give another fingerprint
    assert bench.measured_traffic("fp64@512x6", good, bench.WAVEFORM_PROFILE) is None


def test_figures_are_kept_per_plan(tmp_path):
    tile = bench.PROFILE_SUMMARY
    good = _summary(tmp_path, bench.kernel_fingerprint(tile))
    assert bench.plan_key("fp64", {"tile_bins": 256, "rounds": 6}) == "fp64@256x6"
    assert sorted(bench.profiled_plans("fp64", good, tile)) == ["256x6", "512x6"]
    assert bench.profiled_plans("mixed", good, tile) == []
    assert bench.profiled_plans("fp64", _summary(tmp_path, "0" * 64), tile) == []


def test_executed_flops_per_pair(tmp_path):
    # the mean over the summary's plans, per pair of the profiled batch
    tile = bench.PROFILE_SUMMARY
    good = _summary(tmp_path, bench.kernel_fingerprint(tile))
    assert bench.executed_flops_per_pair("fp64", good, tile) == pytest.approx(7.85e10 / (4096 * 259585))
    assert bench.executed_flops_per_pair("mixed", good, tile) is None
    assert bench.executed_flops_per_pair("fp64", _summary(tmp_path, "0" * 64), tile) is None
    # the committed summary: about 73 FP64 flops per pair on the FP64 path
    committed = bench.executed_flops_per_pair("fp64")
    assert committed is not None and 60 < committed < 89


def test_fingerprints_cover_each_kernels_sources():
    names = {k: [os.path.basename(p) for p in v] for k, v in bench.PROFILE_SOURCES.items()}
    for must in ("gw_kernels.hip", "gw_device_math.h", "gw_plan.h", "gw_phasor_table.h", "build.py"):
        assert must in names[bench.PROFILE_SUMMARY]
    assert "gw_waveform.hip" in names[bench.WAVEFORM_PROFILE]
    assert "gw_relbin.hip" in names[bench.RELBIN_PROFILE]
    prints = {bench.kernel_fingerprint(k) for k in bench.PROFILE_SOURCES}
    assert len(prints) == 3 and all(len(p) == 64 for p in prints)
