"""Host-side checks of the benchmark script: one GPU only, and the per-unit
byte figures the roofline divides by."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_streaming_byte_figures():
    """Per point-step: forward reads u, q, c and writes u, q (20 B); the
    recompute and the forward-with-store also write a^n, the adjoint also
    reads it (24 B); a particle-gradient with recompute moves 68 B per
    point-step and shot, with every step stored 48 B."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    B = bench.BYTES_PER_POINT_STEP
    assert B["forward"] == 20 and B["recompute"] == 24 and B["adjoint"] == 24
    assert B["forward_store"] == 24
    assert B["forward"] + B["recompute"] + B["adjoint"] == 68
    assert B["forward_store"] + B["adjoint"] == 48
