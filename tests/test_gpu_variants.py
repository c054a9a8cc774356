"""GPU parity of the stepping variants: stability condition A, the
progressive splitting, and the periodic warm-started re-estimation of the
radii, each against the oracle's variant on the same inputs (FP64, 1e-10
relative in V)."""
import numpy as np
import pytest

from gpu_util import gpu_run, oracle_rho, rel_errors
from oracle.emrkc import emrkc_run, stage_counts
from oracle.monodomain import build_grid_problem
from oracle.powiter import compute_rho, random_unit_interval
from workloads.configs import small_config

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


def _check(prob, y, V, z):
    Y = y.reshape(prob.nv, prob.N)
    l2, mx = rel_errors(V, Y[0])
    assert l2 <= TOL and mx <= TOL, (l2, mx)
    for c in range(1, prob.nv):
        zl2, zmx = rel_errors(z[c - 1], Y[c])
        assert zl2 <= TOL and zmx <= TOL, (c, zl2, zmx)


@pytest.mark.parametrize("rho", [(51.0, 4.4), (700.0, 30.0)])
def test_condition_a(E, rho):
    """Condition-A stage counts (m >= 2, the larger eta) on a propagating
    CRN_SURR wave, against the oracle's condition-A run."""
    cfg = small_config("c2_3d_crn", (37, 29, 11))
    prob = build_grid_problem(cfg)
    y = emrkc_run(prob, prob.uniform_state(), 0.0, cfg["dt"], 80, *rho, cond="A")
    V, z, st = gpu_run(cfg, 80, rho, flags=E.EMRKC_COND_A)
    s, m, eta = stage_counts(cfg["dt"], *rho, cond="A")
    assert (st.s, st.m) == (s, m) and st.eta == pytest.approx(eta, rel=1e-15)
    assert (s, m) != stage_counts(cfg["dt"], *rho)[:2]
    _check(prob, y, V, z)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_progressive_splitting(E, precision):
    """Progressive splitting against the oracle's literal progressive inner
    problem (FP64), and against the standard splitting on the GPU: on the
    monodomain split both agree up to the rounding of c'_m."""
    cfg = small_config("c2_3d_crn", (41, 19, 9), model="TTP_SURR")
    rho = (51.0, 9.0)
    Vp, zp, _ = gpu_run(cfg, 100, rho, precision=precision, flags=E.EMRKC_PROGRESSIVE)
    Vs, zs, _ = gpu_run(cfg, 100, rho, precision=precision)
    l2, mx = rel_errors(Vp, Vs)
    assert mx <= (1e-12 if precision == "fp64" else 1e-5), (l2, mx)
    if precision == "fp64":
        prob = build_grid_problem(cfg)
        y = emrkc_run(prob, prob.uniform_state(), 0.0, cfg["dt"], 100, *rho, progressive=True)
        _check(prob, y, Vp, zp)


def test_periodic_reestimation(E):
    """rho_every = 20 on a firing TTP_SURR slab: the library re-estimates
    both radii before steps 20, 40, ... (warm started), as the oracle does
    with its own Compute_Rho; the radii agree to the power iteration's
    rounding noise, so the stage counts and the trajectory agree to 1e-10."""
    import torch
    cfg = small_config("c2_3d_crn", (41, 19, 9), model="TTP_SURR")
    prob = build_grid_problem(cfg)
    dt, nsteps, K = cfg["dt"], 120, 20
    y0 = prob.uniform_state()
    v0 = random_unit_interval(y0.size, 0)
    vF, rF, _, _ = compute_rho(0.0, y0, prob.f_F, v0.copy())
    vS, rS, _, _ = compute_rho(0.0, y0, prob.f_S, v0.copy())
    seen, track = [], []
    y = emrkc_run(prob, y0, 0.0, dt, nsteps, 1.05 * rF, 1.05 * rS, rho_every=K,
                  rho_state=dict(vF=vF, vS=vS, rF=rF, rS=rS),
                  on_estimate=lambda n, a, b, i, j: seen.append((n, a, b)),
                  callback=lambda n, yy: track.append(float(yy[:prob.N].max())))
    assert max(track) > 0.0  # the slab fired
    sim = E.simulation_from_config(cfg, rho_every=K)
    E.emrkc_init_state(sim.ctx, sim.state)
    gF, gS, _, _, _ = E.emrkc_estimate_rho(sim.ctx, sim.state)
    assert gF == pytest.approx(1.05 * rF, rel=1e-6) and gS == pytest.approx(1.05 * rS, rel=1e-6)
    got = []
    for a in range(0, nsteps, 30):  # calls that straddle the re-estimation points
        E.emrkc_step(sim.ctx, sim.state, dt, 30)
        got.append(E.emrkc_get_rho(sim.ctx))
    torch.cuda.synchronize()
    # the radii in force after step 120 are the ones estimated before step 100
    n, a, b = seen[-1]
    assert n == 100
    assert got[-1][0] == pytest.approx(a, rel=1e-6) and got[-1][1] == pytest.approx(b, rel=1e-6)
    assert [e[0] for e in seen] == [20, 40, 60, 80, 100]
    _check(prob, y, sim.V.cpu().numpy(), sim.z.cpu().numpy().astype(np.float64))
    sim.close()
