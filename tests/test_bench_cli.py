"""CPU checks of bench.py's command line: more than one GPU is refused with a
message before anything touches a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_measured_traffic_table_names_known_kernels():
    sys.path.insert(0, ROOT)
    import bench
    keys = [k for k in bench.MEASURED_TRAFFIC if k != "sources"]
    assert keys, "no measured traffic"
    for kname, workload in keys:
        assert workload in bench.WORKLOADS
        assert kname.startswith(("k_group<", "k_pool<", "k_binned", "k_persist", "k_plain"))
        assert bench.MEASURED_TRAFFIC[(kname, workload)] > 0
