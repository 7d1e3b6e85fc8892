"""Host-side checks of the benchmark script (no GPU): the one-GPU contract and the work models
its JSON line is computed from."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("n,s_w,s_o,mb", [(32, 8, 8, 2.88), (32, 16, 16, 5.77),
                                         (48, 8, 8, 9.73), (48, 16, 16, 19.46)])
def test_pair_solve_model_bytes(n, s_w, s_o, mb):
    # minimum-pass model: the 2 N^3 intermediate written, read and written, read (8 N^3 working
    # elements) and 3 N^3 orbital / potential elements; 32^3 2.88 / 5.77 MB and 48^3
    # 9.73 / 19.46 MB (FP32 / FP64 storage)
    assert abs(bench.pair_solve_model_bytes(n, s_w, s_o) / 1e6 - mb) < 0.01


def test_xy_pass_work_at_48():
    # per transform at N = 48 (P = 96): 2 (N + P) length-P FFTs of 5 P log2 P flops plus the
    # 2 P^2 kernel multiply; N^2 P complex elements read and written
    assert abs(bench.xy_pass_flops(48) / 1e6 - 89.16) < 0.01
    assert bench.xy_pass_bytes(48, 8) == 2 * 48 * 48 * 96 * 8
