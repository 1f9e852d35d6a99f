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
    """Traffic per unit (a Lanczos sequence-step, an H v launch) from the committed counters:
    scaled by the units of a launch, only for the kernel source, vector size and layouts the
    counters cover."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        t = json.load(f)
    e = t["lanczos_step"]
    per = e["fetch_bytes"] + e["write_bytes"]
    alg = 48.0 * (1 << 24)
    assert e["algorithmic_bytes"] == alg and set(e["layouts"]) == {"single", "stacked"}
    if e["kernel_source"] == bench.kernel_source_hash():
        assert bench.measured_traffic("lanczos_step", "single", 1, alg) == per
        assert bench.measured_traffic("lanczos_step", "stacked", 16, 16 * alg) == 16 * per
    # the block layout, another vector size or a mismatched count get nothing
    assert bench.measured_traffic("lanczos_step", "block", 16, 16 * alg) is None
    assert bench.measured_traffic("lanczos_step", "single", 1, 48.0 * (1 << 16)) is None
    assert bench.measured_traffic("lanczos_step", "stacked", 4, 16 * alg) is None
    assert bench.measured_traffic("apply_h", "single", 1, 32.0 * (1 << 8)) is None
