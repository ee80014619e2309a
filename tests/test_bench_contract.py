"""bench.py contract on the CPU: one GPU only, and the committed HBM-traffic summary matches the kernel source."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_recorded_fine_kernel_traffic_is_current():
    """The traffic summary was taken from the current fine-level kernel source, it covers the shape the headline
    run selects (the vector kernel over 3072-nonzero blocks), and every kernel it records is a fine-level launch
    (about 100 MB on the 591,361-DoF workload), not one of the coarse levels that share the kernel."""
    sys.path.insert(0, ROOT)
    import bench
    t = bench.recorded_traffic("k_level_local<float,u8,3072,128,256,vec>")
    assert t is not None, "kernel source changed since the traffic summary was recorded"
    names = [line.split("]", 1)[0][len("traffic["):] for line in open(bench.TRAFFIC_PROFILE).read().splitlines()
             if line.startswith("traffic[")]
    assert names
    for name in names:
        t = bench.recorded_traffic(name)
        assert t is not None and 9.0e7 < t < 1.2e8, (name, t)
