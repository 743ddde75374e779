"""bench.py's host-side contract, on the CPU: the one-GPU refusal, the
source hash that ties committed traffic summaries to the kernels they were
taken on, and the lookup of those summaries by kernel instance and R."""
import re
import subprocess
import sys
from pathlib import Path

import bench

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_kernel_source_hash_is_stable():
    h = bench.kernel_source_hash()
    assert re.fullmatch(r"[0-9a-f]{16}", h)
    assert h == bench.kernel_source_hash()


def test_traffic_summaries_are_complete_and_matched_by_kernel_and_R():
    files = sorted((ROOT / "profiles").glob("sweep*_c2_4Mx1M_f32values_f64iter_*traffic.md"))
    assert files
    for p in files:
        text = p.read_text()
        for field in ("kernel_source_hash:", "profiled_kernel:", "profiled_in_flight:", "hbm_bytes_per_launch:",
                      "rocprofv3 --pmc FETCH_SIZE", "rocprofv3 --pmc WRITE_SIZE"):
            assert field in text, (p.name, field)
    # a summary is used only for its own kernel instance and R
    assert bench.traffic_from_profile("sweep_pipe_kernel<F32,F64,4>", 12345) is None
    assert bench.traffic_from_profile("no_such_kernel<F32,F64,4>", 4096) is None
