"""bench.py's contract on one GPU, and the byte counts its roofline uses
(no device needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_algorithmic_bytes_per_node_stage():
    from paper_2605_16684_amd import perfmodel
    # q, dq read and q_out, dq written (dq not read in 1 of 5 stages), plus
    # the neighbours' face traces: (4 - 1/5) * 40 + 240/Nq B at N = 4
    assert abs(perfmodel.bytes_per_node(4) - 200.0) < 1e-12
    assert abs(perfmodel.bytes_per_node(4, stage=False) - (80.0 + 48.0)) < 1e-12
    # curved meshes add J a^r_d (9 words), 1/J and phi per node
    assert abs(perfmodel.bytes_per_node_curved(4) - 288.0) < 1e-12
