"""bench.py on the host: the multi-GPU refusal and the byte models behind its
roofline figures (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_models_per_node_update():
    sys.path.insert(0, ROOT)
    import bench
    # FP32: 27 deviations read and written (4 B), the (phi, rho) pair and the
    # fraction read (12 B), the (x, V) record written (16 B)
    assert bench.FUSED_BYTES["fp32"] == 27 * 4 * 2 + 12 + 16 == 244
    # density pass: 27 deviations and the source records read, PD and XR written
    assert bench.DENSITY_BYTES["fp32"] == 27 * 4 + 16 + 12 == 136
    # the roofline basis: both colour sets (2 x 27 populations) read once and
    # written once, 4 B each in FP32 and 2 B in 16-bit storage
    assert bench.STEP_BYTES["fp32"] == 2 * 27 * 4 * 2 == 432
    assert bench.STEP_BYTES["bf16"] == 2 * 27 * 2 * 2 == 216
    for st in ("bf16", "fp16"):
        assert bench.FUSED_BYTES[st] == 27 * 2 * 2 + 12 + 16
        assert bench.DENSITY_BYTES[st] == 27 * 2 + 16 + 12
