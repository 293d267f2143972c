"""bench.py's contract where it needs no GPU: more than one GPU is refused with a message, and a committed counter
record is used only while the kernel sources still hash to the value it was taken on (else traffic is null)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_counter_records_are_used_only_on_the_sources_they_were_taken_on():
    sys.path.insert(0, ROOT)
    import bench
    for kind in bench.ROOFLINE_KERNELS:
        h = bench.kernel_source_hash(kind)
        assert len(h) == 16 and h == bench.kernel_source_hash(kind)
    # the engine's record depends on the engine's sources only, the fine-level records on the fine-level ones
    assert bench.kernel_source_hash("engine32") != bench.kernel_source_hash("resid_fine32")
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.startswith("traffic_") and name.endswith(".json"):
            with open(os.path.join(ROOT, "profiles", name)) as f:
                rec = json.load(f)
            assert rec["bytes_per_launch"] > 0 and rec["dispatches"][0] > 0
            want = rec["bytes_per_launch"] if rec["source_hash"] == bench.kernel_source_hash(rec["kernel"]) else None
            assert bench.traffic_from_profiles(rec["kernel"], rec["workload"]) == want, name
