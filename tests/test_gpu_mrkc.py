"""GPU parity of the mRKC method (EMRKC_METHOD_MRKC) against the oracle's
mRKC: the split terms, the power iteration on them, full runs for several
stage plans, and the stage counts next to emRKC's on the same workload."""
import numpy as np
import pytest

from gpu_util import rel_errors
from oracle.monodomain import build_grid_problem, build_tet_problem
from oracle.mrkc import MrkcSplit, mrkc_run
from oracle.powiter import compute_rho, random_unit_interval
from workloads.configs import small_config
from workloads.tetmesh import build_shell, small_shell_config

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


def _radii(sp, y):
    v0 = random_unit_interval(y.size, 0)
    _, rF, itF, _ = compute_rho(0.0, y, sp.f_F, v0.copy())
    _, rS, itS, _ = compute_rho(0.0, y, sp.f_S, v0.copy())
    return 1.05 * rF, 1.05 * rS, itF, itS


def _run_gpu(E, sim, dt, nsteps):
    import torch
    E.emrkc_init_state(sim.ctx, sim.state)
    E.emrkc_step(sim.ctx, sim.state, dt, nsteps)
    torch.cuda.synchronize()
    out = sim.V.cpu().numpy().copy(), sim.z.cpu().numpy().astype(np.float64), E.emrkc_last_stats(sim.ctx)
    return out


def _check(prob, y, V, z):
    Y = y.reshape(prob.nv, prob.N)
    l2, mx = rel_errors(V, Y[0])
    assert l2 <= TOL and mx <= TOL, (l2, mx)
    for c in range(1, prob.nv):
        zl2, zmx = rel_errors(z[c - 1], Y[c])
        assert zl2 <= TOL and zmx <= TOL, (c, zl2, zmx)


@pytest.mark.parametrize("model", ["HH", "CRN_SURR", "TTP_SURR"])
def test_split_terms(E, model):
    import torch
    cfg = small_config("c2_3d_crn", (9, 7, 5), model=model)
    prob = build_grid_problem(cfg)
    sp = MrkcSplit(prob, 0)
    rng = np.random.default_rng(3)
    y = prob.uniform_state() * (1 + 1e-2 * rng.standard_normal(prob.nv * prob.N))
    sim = E.simulation_from_config(cfg, rho=(1.0, 1.0), method="mrkc")
    Y = y.reshape(prob.nv, prob.N)
    sim.V.copy_(torch.from_numpy(Y[0].copy()))
    sim.z.copy_(torch.from_numpy(Y[1:].copy()))
    out = torch.empty(prob.nv * prob.N, dtype=torch.float64, device="cuda")
    for which, f in [(0, sp.f_F), (1, sp.f_S)]:
        E.emrkc_eval_mrkc_terms(sim.ctx, sim.state, 0.5, which, out)
        ref = f(0.5, y)
        scale = np.abs(ref.reshape(prob.nv, prob.N)).max(axis=1)
        err = np.abs(out.cpu().numpy() - ref).reshape(prob.nv, prob.N).max(axis=1)
        assert np.all(err <= 1e-12 * np.maximum(scale, 1e-300) + 1e-300), (which, err / scale)
    sim.close()


@pytest.mark.parametrize("model,n", [("CRN_SURR", (37, 29, 11)), ("TTP_SURR", (21, 17, 9))])
def test_estimate_rho(E, model, n):
    cfg = small_config("c2_3d_crn", n, model=model)
    prob = build_grid_problem(cfg)
    sp = MrkcSplit(prob, 0)
    rF, rS, itF, itS = _radii(sp, prob.uniform_state())
    sim = E.simulation_from_config(cfg, method="mrkc")
    E.emrkc_init_state(sim.ctx, sim.state)
    gF, gS, gitF, gitS, _ = E.emrkc_estimate_rho(sim.ctx, sim.state)
    assert (gitF, gitS) == (itF, itS)
    assert gF == pytest.approx(rF, rel=1e-6) and gS == pytest.approx(rS, rel=1e-6)
    sim.close()


@pytest.mark.parametrize("model,n,nsteps,rho", [("CRN_SURR", (37, 29, 11), 120, None),
                                                ("TTP_SURR", (41, 19, 9), 120, (3000.0, 20.0)),
                                                ("HH", (33, 33), 60, (1610.0, 0.86))])
def test_full_run(E, model, n, nsteps, rho):
    """mRKC on a firing slab, with the oracle's radii of f~_F and f~_S at
    rest (CRN_SURR) or given ones: the TTP_SURR m gate is so much stiffer
    during the upstroke than at rest that mRKC with radii estimated once at
    rest diverges (emRKC's exponential stage is what removes that
    stiffness); the HH f~_S power iteration does not converge in 100
    iterations at rest."""
    base = "c1_2d_hh" if len(n) == 2 else "c2_3d_crn"
    cfg = small_config(base, n, model=model)
    prob = build_grid_problem(cfg)
    sp = MrkcSplit(prob, 0)
    y0 = prob.uniform_state()
    rF, rS = rho if rho is not None else _radii(sp, y0)[:2]
    y = mrkc_run(sp, y0, 0.0, cfg["dt"], nsteps, rF, rS)
    assert np.all(np.isfinite(y))
    sim = E.simulation_from_config(cfg, rho=(rF, rS), method="mrkc")
    V, z, st = _run_gpu(E, sim, cfg["dt"], nsteps)
    sim.close()
    _check(prob, y, V, z)


@pytest.mark.parametrize("rho,sm", [((2000.0, 300.0), (3, 3)), ((51.0, 700.0), (5, 1)), ((5000.0, 100.0), (2, 6))])
def test_stage_plans(E, rho, sm):
    """Outer stages s >= 2 and m = 1 on the mRKC path (buffer rotation of
    gate 0 through the inner stages and across outer stages)."""
    cfg = small_config("c2_3d_crn", (23, 17, 7))
    prob = build_grid_problem(cfg)
    sp = MrkcSplit(prob, 0)
    y = mrkc_run(sp, prob.uniform_state(), 0.0, cfg["dt"], 40, *rho)
    sim = E.simulation_from_config(cfg, rho=rho, method="mrkc")
    V, z, st = _run_gpu(E, sim, cfg["dt"], 40)
    sim.close()
    assert (st.s, st.m) == sm
    _check(prob, y, V, z)


def test_shell(E):
    """The TTP_SURR shell (ELL operator) with radii that cover the upstroke
    (rest radii diverge, as on the slab)."""
    cfg = small_shell_config()
    mesh, mask = build_shell(cfg)
    prob = build_tet_problem(cfg, mesh, mask)
    sp = MrkcSplit(prob, 0)
    y0 = prob.uniform_state()
    rF, rS = 3000.0, 20.0
    y = mrkc_run(sp, y0, 0.0, cfg["dt"], 60, rF, rS)
    assert np.all(np.isfinite(y))
    sim = E.simulation_from_tet_config(cfg, mesh, mask, rho=(rF, rS), method="mrkc")
    V, z, _ = _run_gpu(E, sim, cfg["dt"], 60)
    sim.close()
    _check(prob, y, V, z)


def test_stage_counts_next_to_emrkc(E):
    """TTP_SURR slab at rest: the m gate's rate (110 times the classical
    one) makes f~_F several times stiffer than f_F, so mRKC takes more
    inner stages per step than emRKC; the other gates are slow at rest, so
    f~_S has the radius of f_S to the power iteration's tolerance."""
    cfg = small_config("c2_3d_crn", (41, 19, 9), model="TTP_SURR")
    counts = {}
    for method in ("emrkc", "mrkc"):
        sim = E.simulation_from_config(cfg, method=method)
        E.emrkc_init_state(sim.ctx, sim.state)
        E.emrkc_estimate_rho(sim.ctx, sim.state)
        counts[method] = E.emrkc_stages(sim.ctx, cfg["dt"])[:2] + E.emrkc_get_rho(sim.ctx)
        sim.close()
    (se, me, rFe, rSe), (sm, mm, rFm, rSm) = counts["emrkc"], counts["mrkc"]
    assert rFm > 5 * rFe
    assert rSm == pytest.approx(rSe, rel=3e-2)
    assert sm == se and mm > me


@pytest.mark.parametrize("name,model", [("c1_2d_hh", None), ("c2_3d_crn", None), ("c2_3d_crn", "TTP_SURR"),
                                        ("c5_3d_crn_large", None)])
def test_stage_counts_table(E, name, model):
    """emRKC against mRKC at full size: the radii each method estimates at
    rest (f_F and f_S, and f~_F and f~_S) and the stage counts they give at
    the workload's dt (run with -s for the table).  Moving the stiffest
    gate into the fast term can only add to its radius."""
    from workloads.configs import get_config
    cfg = get_config(name) if model is None else get_config(name, model=model)
    row = {}
    for method in ("emrkc", "mrkc"):
        sim = E.simulation_from_config(cfg, method=method)
        E.emrkc_init_state(sim.ctx, sim.state)
        rF, rS, itF, itS, _ = E.emrkc_estimate_rho(sim.ctx, sim.state, allow_noconv=True)
        s, m = E.emrkc_stages(sim.ctx, cfg["dt"])[:2]
        row[method] = (rF, rS, s, m, itF, itS)
        sim.close()
    print("\n  %s %s dt=%g: emRKC rho_F %.4g rho_S %.4g (s, m) = (%d, %d) its (%d, %d); "
          "mRKC rho_F %.4g rho_S %.4g (s, m) = (%d, %d) its (%d, %d)"
          % ((name, cfg["model"], cfg["dt"]) + row["emrkc"][:2] + row["emrkc"][2:4] + row["emrkc"][4:] + row["mrkc"][:2]
             + row["mrkc"][2:4] + row["mrkc"][4:]))
    assert row["mrkc"][0] >= 0.99 * row["emrkc"][0]
    assert row["mrkc"][3] >= row["emrkc"][3]


@pytest.mark.parametrize("model", ["CRN_SURR", "TTP_SURR", "HH"])
def test_gate_terms_over_the_voltage_range(E, model):
    """Every gate's Lambda (z - z_inf), node by node, over V from -120 to 80
    mV (both removable singularities of x/(e^x - 1) included, and points
    within 1e-9 mV of them) with gates drawn on [0, 1]: the split's fast
    term holds the stiff gate, its slow term the others.  Bound per node:
    1e-13 of |Lambda| (|z| + |z_inf|), a few hundred ulp, against O(1) for a
    wrong rate constant, sign or slope."""
    import torch
    cfg = small_config("c2_3d_crn", (41, 25, 5), model=model)
    prob = build_grid_problem(cfg)
    N, nE = prob.N, prob.nE
    rng = np.random.default_rng(11)
    V = np.linspace(-120.0, 80.0, N)
    special = np.array([-40.0, -55.0, -40.0 + 1e-9, -40.0 - 1e-9, -55.0 + 1e-9, -55.0 - 1e-9, -35.0, -65.0])
    V[rng.choice(N, special.size, replace=False)] = special
    Y = prob.uniform_state().reshape(prob.nv, N).copy()
    Y[0] = V
    Y[1:1 + nE] = rng.uniform(0.0, 1.0, (nE, N))
    y = Y.reshape(-1)
    lam, zinf = prob.model.gates(V)
    sp = MrkcSplit(prob, 0)
    sim = E.simulation_from_config(cfg, rho=(1.0, 1.0), method="mrkc")
    sim.V.copy_(torch.from_numpy(Y[0].copy()))
    sim.z.copy_(torch.from_numpy(Y[1:].copy()))
    out = torch.empty(prob.nv * N, dtype=torch.float64, device="cuda")
    for which, f, gates in [(0, sp.f_F, [0]), (1, sp.f_S, range(1, nE))]:
        E.emrkc_eval_mrkc_terms(sim.ctx, sim.state, 0.5, which, out)
        got = out.cpu().numpy().reshape(prob.nv, N)
        ref = f(0.5, y).reshape(prob.nv, N)
        for g in gates:
            bound = 1e-13 * np.abs(lam[g]) * (np.abs(Y[1 + g]) + np.abs(zinf[g]))
            err = np.abs(got[1 + g] - ref[1 + g])
            assert np.all(err <= bound), (which, g, (err / bound).max(), V[np.argmax(err / bound)])
    sim.close()
