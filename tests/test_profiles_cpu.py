"""The committed HBM counters of the headline kernel are self-consistent:
the traffic bench.py reports is the counters' FETCH and WRITE KiB per
dispatch, each scaled by what the same counter read for a plain copy of a
known size, and it lies within a plausible band of the algorithmic bytes."""
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COUNTERS = os.path.join(ROOT, "profiles", "hidft_fused_k4096_b4096_counters.json")


def test_headline_counters_are_consistent():
    with open(COUNTERS) as fh:
        c = json.load(fh)
    assert c["kernel"].startswith("hidft_fused_kernel<12,")
    assert len(c["kernel_source_sha256"]) == 64
    # 4096 signals x 4096 points x (8 B in + 8 B out)
    assert c["algorithmic_bytes_per_launch"] == 4096 * 4096 * 16
    # the copy calibration: a copy of B bytes each way reads B and writes B
    b = c["copy_bytes_each_way"]
    assert abs(c["scale_fetch"] - b / (c["copy_fetch_kib_per_dispatch"] * 1024)) < 1e-9
    assert abs(c["scale_write"] - b / (c["copy_write_kib_per_dispatch"] * 1024)) < 1e-9
    traffic = (c["fetch_kib_per_dispatch"] * c["scale_fetch"]
               + c["write_kib_per_dispatch"] * c["scale_write"]) * 1024
    assert abs(traffic - c["traffic_bytes_per_launch"]) <= 1e-6 * traffic
    ratio = c["traffic_bytes_per_launch"] / c["algorithmic_bytes_per_launch"]
    assert abs(ratio - c["traffic_over_algorithmic"]) < 1e-9
    # every byte is moved at least once, and re-reads stay small
    assert 0.99 <= ratio <= 1.3, ratio
    # one counter per rocprofv3 pass, for the kernel and for the copy
    cmds = c["commands"]
    assert "--pmc FETCH_SIZE" in cmds["fetch"] and "--mode execute" in cmds["fetch"]
    assert "--pmc WRITE_SIZE" in cmds["write"] and "--mode execute" in cmds["write"]
    assert "--pmc FETCH_SIZE" in cmds["copy_fetch"] and "--mode copy" in cmds["copy_fetch"]
    assert "--pmc WRITE_SIZE" in cmds["copy_write"] and "--mode copy" in cmds["copy_write"]
