"""Host-side checks of the benchmark script (no GPU needed): it refuses GPU counts other than
one before any leg runs, and its roofline constants are the chip's published figures."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("extra", [[], ["--only-batched"], ["--only-surrogate"], ["--only-sor"], ["--only-basin2048"],
                                   ["--copy-probe"]])
def test_more_than_one_gpu_is_refused(extra):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", *extra],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_constants():
    sys.path.insert(0, ROOT)
    import bench
    # 8 TB/s of HBM3E; FP32 vector rate without packed two-wide instructions:
    # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
    assert bench.HBM_PEAK_GBS == 8000.0
    assert bench.VALU_PEAK_TFLOPS == pytest.approx(78.6432)
    # eta, u, v, H read and eta, u, v written, 4 bytes each
    assert bench.BYTES_PER_CELL_STEP == 4 * (4 + 3)
    # MI355X's published FP32 vector peak (packed two-wide FMAs counted)
    assert bench.VALU_PEAK_PUBLISHED_TFLOPS == 157.3
    assert bench.REPS >= 5


@pytest.mark.parametrize("m", ["0", "3", "4", "7"])
def test_surrogate_interval_must_divide_the_judge_interval(m):
    """Refused before any GPU work: the rollout needs m to divide the 50-step judge interval."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--surrogate-every", m, "--only-surrogate"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "divisor of the judge interval" in r.stderr
    assert r.stdout == ""
