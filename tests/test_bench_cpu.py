"""The benchmark script's contract on the CPU: it refuses more than one GPU before touching a
device, and the committed counter records its roofline reads match the kernel sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_counter_records_match_the_kernel_sources():
    """The default line's roofline (radius kernel) and the omnibus line's are priced from
    SQ_INSTS_VALU records taken on the current kernel sources, and the traffic record is there."""
    for kern in ("radius", "yz_count", "x_count"):
        assert bench._counter_record("valu_wave_instructions_per_launch", kern) > 0
        assert bench._traffic_record(kern) > 0
    assert bench._counter_record("valu_wave_instructions_per_launch", "window", bench.OMNIBUS_RECORD,
                                 bench.OMNIBUS_SOURCES) > 0


def test_peak_is_the_vector_lane_rate():
    # 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 157.3 TFLOP/s FP32 with an FMA counted twice, / 2
    assert abs(bench.PEAK_VALU - 256 * 4 * 32 * 2.4e9) / bench.PEAK_VALU < 1e-3
