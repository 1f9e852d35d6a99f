"""Host-side parts of bench.py: the one-GPU refusal, and the counter lookup that may
only report HBM traffic for the kernel source, sequences per launch and vector size
the counters were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2 and "one GPU" in out.stderr


def test_traffic_lookup_matches_workload():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        t = json.load(f)
    for key, e in t["lanczos_step"].items():
        B = int(key)
        assert e["rhs_block"] == B
        alg = 96.0 * (1 << 24) * B
        assert e["algorithmic_bytes"] == alg
        if e["kernel_source"] == bench.kernel_source_hash():
            assert bench.measured_traffic("lanczos_step", B, alg) == e["fetch_bytes"] + e["write_bytes"]
        # another vector size with the same sequences per launch, or another B, gets nothing
        assert bench.measured_traffic("lanczos_step", B, 96.0 * (1 << 16) * B) is None
        assert bench.measured_traffic("lanczos_step", B + 1, alg) is None
    assert bench.measured_traffic("apply_h", 1, 32.0 * (1 << 8)) is None
