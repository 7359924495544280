"""CPU checks of bench.py's command-line contract (no GPU needed): it runs
on one GPU only and says so when asked for more; its profiled-build record
names the integrator sources it hashes."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_profiled_record_matches_a_source_hash():
    sys.path.insert(0, ROOT)
    import bench

    h = bench.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    for f in bench.INTEGRATOR_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_1706_07062_amd", "csrc", f))
    assert len(bench.PROFILED["source_hash"]) == 16
    assert bench.PROFILED["traffic_bytes"] > 0 and bench.PROFILED["hw_fp64_flops"] > 0
