"""The benchmark's host-side contract (CPU only): it refuses more than one
GPU with a message, and the committed rocprofv3 summaries it reads carry the
fields it reports."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = [("tile_lds_kernel", "haar30"), ("tile_pass_kernel", "qft28"), ("batch_reg_kernel", "batch512")]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("kernel,workload", PROFILES)
def test_profile_summaries_have_what_the_benchmark_reads(kernel, workload):
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")) as fh:
        d = json.load(fh)
    assert len(d["source_hash"]) == 16
    assert d["bytes_per_launch"] > 0 and d["kernel_stats_avg_ms"] > 0
    c = d["counters"]
    for key in ("mfma_busy_frac", "mfma_exec_tflops", "mfma_exec_frac_of_peak", "valu_insts_per_launch",
                "lds_bank_conflict_frac", "valu_fp_insts_per_launch", "valu_fp_busy_frac"):
        assert key in c
    assert 0.0 <= c["mfma_busy_frac"] <= 1.0 and 0.0 <= c["valu_fp_busy_frac"] <= 1.0
    # every command runs committed files only and names its counters
    assert all(cmd.startswith("rocprofv3 ") and " -- python3 bench.py " in cmd for cmd in d["commands"])
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")) as fh:
        md = fh.read()
    assert d["source_hash"] in md
    if "alg_bytes_per_launch" in d:
        assert abs(d["traffic_over_alg"] - 1.0) < 0.01
