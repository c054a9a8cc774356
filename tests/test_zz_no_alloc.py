"""emrkc_step_noalloc, the stepping entry point that allocates nothing,
against emrkc_step through the C ABI.  Both launch the same kernels in the
same order (the no-alloc call with its work buffers in the library's static
scratch array), so their V and z agree bit for bit -- stricter than the
1e-10 FP64 parity bar, which the first call also meets against the oracle.
Consecutive calls share the device's scratch array: the second call of each
pair runs a smaller problem over what the first left there."""
import numpy as np
import pytest

from gpu_util import oracle_run, rel_errors
from workloads.configs import small_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


def run(E, cfg, nsteps, rho, precision="fp64", noalloc=False, flags=0, chunks=None, variants=None):
    import torch
    sim = E.simulation_from_config(cfg, precision=precision, rho=rho, flags=flags)
    if variants is not None:
        E.emrkc_set_variants(sim.ctx, variants)
    E.emrkc_init_state(sim.ctx, sim.state)
    step = E.emrkc_step_noalloc if noalloc else E.emrkc_step
    for n in (chunks or [nsteps]):
        step(sim.ctx, sim.state, cfg["dt"], n)
    torch.cuda.synchronize()
    st = E.emrkc_last_stats(sim.ctx)
    out = (sim.V.cpu().numpy().copy(), sim.z.cpu().numpy().astype(np.float64), st, sim.state.step, sim.state.t)
    sim.close()
    return out


def check_pair(E, cfg, nsteps, rho, **kw):
    print("no-alloc case %s, %d steps, rho %s, %s" % (cfg["name"], nsteps, rho, kw), flush=True)
    Va, za, sa, stepa, ta = run(E, cfg, nsteps, rho, noalloc=True, **kw)
    Vb, zb, sb, stepb, tb = run(E, cfg, nsteps, rho, noalloc=False, **kw)
    assert np.isfinite(Va).all()
    assert np.array_equal(Va, Vb) and np.array_equal(za, zb)
    assert (stepa, ta) == (stepb, tb) == (nsteps, nsteps * cfg["dt"])
    assert (sa.s, sa.m, sa.kernels_per_step) == (sb.s, sb.m, sb.kernels_per_step)
    assert sa.used_graph == 0
    return Va, sa


def test_two_calls_in_a_row_second_smaller_match_emrkc_step(E):
    """A 41x23x13 CRN grid, then a 17x9x5 one, through the no-alloc call;
    each equals emrkc_step's result bit for bit, and the first is within
    1e-10 of the oracle."""
    rho = (51.0, 4.4)
    big = small_config("c2_3d_crn", (41, 23, 13))
    V, st = check_pair(E, big, 40, rho)
    assert (st.s, st.m) == (1, 2)
    _, y = oracle_run(big, 40, rho)
    l2, mx = rel_errors(V, y[:V.size])
    assert l2 < 1e-10 and mx < 1e-10, (l2, mx)
    small = small_config("c2_3d_crn", (17, 9, 5))
    check_pair(E, small, 40, rho)
    # and back up: the larger problem again after the smaller one
    check_pair(E, big, 7, rho)


@pytest.mark.parametrize("case", ["mixed", "fused", "s3", "m1_2d", "splits", "step2d", "split3d"])
def test_other_step_plans_match_emrkc_step(E, case):
    """Mixed precision (float S_V and z_1), the fused chunk (three inner
    buffers, two S_V), s = 3 outer stages (z_1 in the scratch array), the
    one-kernel m = 1 path on a 2-D grid, and call splits."""
    cfg = small_config("c2_3d_crn", (29, 23, 9))
    rho, kw, nsteps = (51.0, 4.4), {}, 35
    if case == "mixed":
        kw = dict(precision="mixed")
    elif case == "fused":
        kw = dict(flags=E.EMRKC_FUSE)
    elif case == "s3":
        rho = (51.0, 200.0)
    elif case == "m1_2d":
        # sigma_l = 0.05: the largest eigenvalue of the operator is
        # 4 sigma_l / (h^2 chi Cm) = 14.3/ms, so rho_F = 16 gives m = 1
        cfg = small_config("c2_3d_crn", (37, 11), sigma=(0.05, 0.019, 0.019))
        cfg["dim"] = 2
        rho = (16.0, 4.4)
    elif case == "splits":
        kw = dict(chunks=[1, 33, 7, 2])
        nsteps = 43
    elif case == "step2d":  # one kernel per step on a 2-D grid (alternating S_V buffers)
        cfg = small_config("c2_3d_crn", (37, 11))
        cfg["dim"] = 2
        rho = (900.0, 4.4)
        kw = dict(variants=(0, 0, 4, 0, 0))
    elif case == "split3d":  # pointwise head and u_1 by the inner kernel
        kw = dict(variants=(8, 0, 1, 4, 0))
    _, st = check_pair(E, cfg, nsteps, rho, **kw)
    if case == "s3":
        assert st.s == 3
    if case == "m1_2d":
        assert (st.s, st.m) == (1, 1)
    if case == "fused":
        assert st.kernels_per_step == st.m - 1


def test_no_device_memory_is_taken(E):
    """With s = 3, emrkc_step allocates the library's z_1 buffer on its first
    call; the no-alloc call takes no device memory (measured after one
    warm-up call, which may still make the runtime load code or grow its
    per-queue scratch)."""
    import torch
    cfg = small_config("c2_3d_crn", (64, 64, 16))
    rho = (51.0, 200.0)
    sim = E.simulation_from_config(cfg, rho=rho)
    E.emrkc_init_state(sim.ctx, sim.state)
    E.emrkc_step_noalloc(sim.ctx, sim.state, cfg["dt"], 1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    E.emrkc_step_noalloc(sim.ctx, sim.state, cfg["dt"], 3)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    E.emrkc_step(sim.ctx, sim.state, cfg["dt"], 3)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    sim.close()
    z1_bytes = 20 * 64 * 64 * 16 * 8
    assert free1 == free0, (free0, free1)
    assert free0 - free2 >= z1_bytes, (free0, free2, z1_bytes)


def test_refusals(E):
    """Beyond the scratch array's 64 MiB: EINVAL with the reason; mRKC and
    EMRKC_CHECK_FINITE contexts: EUNSUPPORTED."""
    cfg = small_config("c1_2d_hh", (1500, 1500))  # 2.25M nodes: 4 x 8 B x N > 64 MiB
    sim = E.simulation_from_config(cfg, rho=(100.0, 4.0))
    E.emrkc_init_state(sim.ctx, sim.state)
    with pytest.raises(E.EmrkcError) as err:
        E.emrkc_step_noalloc(sim.ctx, sim.state, cfg["dt"], 1)
    assert err.value.code == E.EMRKC_EINVAL and "scratch" in str(err.value)
    assert sim.state.step == 0
    sim.close()
    small = small_config("c2_3d_crn", (9, 7, 5))
    for kw in [dict(method="mrkc"), dict(flags=E.EMRKC_CHECK_FINITE)]:
        sim = E.simulation_from_config(small, rho=(51.0, 4.4), **kw)
        E.emrkc_init_state(sim.ctx, sim.state)
        with pytest.raises(E.EmrkcError) as err:
            E.emrkc_step_noalloc(sim.ctx, sim.state, small["dt"], 1)
        assert err.value.code == E.EMRKC_EUNSUPPORTED
        sim.close()
