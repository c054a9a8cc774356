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


def test_cpu_sample_of_the_large_slab():
    """The CPU leg times the oracle on whole z-planes of the slab within its
    node bound; smaller workloads run whole."""
    from workloads.configs import get_config
    c5 = get_config("c5_3d_crn_large")
    sub, k = bench.cpu_sample_config(c5)
    assert k == bench.CPU_MAX_NODES // (601 * 601) and sub["n"] == (601, 601, k)
    assert 601 * 601 * k <= bench.CPU_MAX_NODES
    assert sub["stim"] == c5["stim"] and sub["sigma"] == c5["sigma"] and sub["model"] == c5["model"]
    c2 = get_config("c2_3d_crn")
    assert bench.cpu_sample_config(c2) == (c2, None)


def test_planar_reduction_applies_to_face_stimuli_only():
    from workloads.configs import get_config
    red = bench.planar_reduction(get_config("c5_3d_crn_large"))
    assert red["n"] == (601, 2, 2) and red["h"] == (0.1, 0.1, 0.1)
    assert bench.planar_reduction(get_config("c2_3d_crn")) is None
    assert bench.planar_reduction(get_config("c1_2d_hh")) is None


@pytest.mark.slow
def test_planar_reduction_matches_the_full_grid_in_the_oracle():
    """The reduction the bench and the full-size tests rely on: with the
    planar stimulus and a uniform start, the oracle on an n0 x n1 x n2 grid
    gives at every node the value of its run on the n0 x 2 x 2 grid (same
    physics and spacing), through the upstroke."""
    import numpy as np
    from oracle.emrkc import emrkc_run
    from oracle.monodomain import build_grid_problem
    from workloads.configs import get_config
    cfg = get_config("c5_3d_crn_large")
    full = dict(cfg, n=(31, 5, 4))
    red = bench.planar_reduction(full)
    assert red["n"] == (31, 2, 2)
    rho = (50.0, 4.6)
    pf = build_grid_problem(full)
    yf = emrkc_run(pf, pf.uniform_state(), 0.0, cfg["dt"], 60, *rho)
    pr = build_grid_problem(red)
    yr = emrkc_run(pr, pr.uniform_state(), 0.0, cfg["dt"], 60, *rho)
    Vf = yf[:pf.N].reshape(4, 5, 31)
    Vr = yr[:pr.N].reshape(2, 2, 31)[0, 0]
    assert Vr.max() > 0.0                       # the wave has fired
    assert np.abs(Vf - Vr[None, None, :]).max() <= 1e-11 * np.abs(Vr).max()
    # and the bench's error measure is zero on the exact profile
    import torch
    V = torch.from_numpy(np.broadcast_to(Vr, (4, 5, 31)).copy().reshape(-1))
    e2, emax = bench.errors_vs_profile(V, Vr, (31, 5, 4), torch)
    assert e2 == 0.0 and emax == 0.0
    V[7] += 1.0
    e2, emax = bench.errors_vs_profile(V, Vr, (31, 5, 4), torch)
    assert abs(emax - 1.0 / np.abs(Vr).max()) < 1e-15
    assert abs(e2 - 1.0 / (np.linalg.norm(Vr) * np.sqrt(20))) < 1e-15
