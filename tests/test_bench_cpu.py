"""Host-side parts of bench.py: the one-GPU guard and the algorithmic byte
model behind the roofline figures (per-node bytes of the head and of the last
inner stage, as listed for the cuboid and the shell workloads)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_byte_model_cuboid():
    """CRN surrogate (20 ionic variables), s = 1, m = 2: the head reads V and
    z, writes z, S_V and u_1; the last inner stage reads u_1, V and S_V and
    writes V.  FP64: 8 + 2*20*8 + 8 + 8 and 8 + 8 + 8 + 8; mixed: z and S_V
    in float."""
    assert bench.bytes_per_node("head", 20, 8, 2) == 344
    assert bench.bytes_per_node("tail", 20, 8, 2) == 32
    assert bench.bytes_per_node("head", 20, 4, 2) == 180
    assert bench.bytes_per_node("tail", 20, 4, 2) == 28
    # m = 1: the head writes V_{n+1} in place of S_V and u_1
    assert bench.bytes_per_node("head", 20, 8, 1) == 8 + 320 + 8
    # m >= 3: the last stage also reads u_{m-2}
    assert bench.bytes_per_node("tail", 20, 8, 3) == 40


def test_byte_model_shell_rows():
    """TTP surrogate (18 ionic variables) on the tetrahedral shell, m = 1: an
    ELL row of width 14 adds 14 x (4-byte column + 8-byte weight)."""
    row = 14 * (4 + 8)
    assert bench.bytes_per_node("head", 18, 8, 1, row) == 8 + 2 * 18 * 8 + 8 + row == 472
    assert bench.bytes_per_node("inner", 18, 8, 2, row) == 32 + row
    with pytest.raises(ValueError):
        bench.bytes_per_node("nonsense", 18, 8, 1)
