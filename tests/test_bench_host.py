"""Host-side checks of bench.py's contract (no GPU): the one-GPU guard and the
HBM-traffic records that feed the roofline object."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("record, source", [("SWEEP_RECORD", "k_solve.hip"), ("FINE_RECORD", "k_fine.hip")])
def test_traffic_records_follow_the_kernel_source(tmp_path, record, source):
    import bench
    rec = getattr(bench, record)
    src = os.path.join(ROOT, "paper_1801_08464_amd", "csrc", source)
    # the committed record matches the committed source at the benchmark workload
    traffic, note = bench.measured_traffic(rec, src, 4)
    assert traffic is not None and traffic > 0, note
    # another workload: no traffic
    assert bench.measured_traffic(rec, src, 3)[0] is None
    # a changed kernel source: no traffic
    changed = tmp_path / source
    shutil.copy(src, changed)
    with open(changed, "a") as f:
        f.write("\n// changed\n")
    traffic, note = bench.measured_traffic(rec, str(changed), 4)
    assert traffic is None and "changed" in note
    # no record at all
    assert bench.measured_traffic(str(tmp_path / "none.md"), src, 4)[0] is None
