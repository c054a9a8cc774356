"""Pins for the oracle's IMEX-RL step (algorithm "One step of the IMEX-RL
method"): closed form on cosine modes with the linear test model, bounded
diffusion at any step, first-order convergence to the EXEX-RL reference."""
import numpy as np
import pytest

from oracle import fem
from oracle.exexrl import exexrl_run, imexrl_cg_solver, imexrl_run, imexrl_step
from oracle.monodomain import build_grid_problem
from workloads.configs import small_config


def _cosine_mode(n, k):
    x = [np.cos(np.pi * kk * np.arange(nn) / (nn - 1)) for nn, kk in zip(n, k)]
    out = x[0]
    for a in x[1:]:
        out = np.multiply.outer(a, out)
    return out.reshape(-1)


@pytest.mark.parametrize("dt", [0.01, 0.5, 5.0])
def test_linear_model_cosine_mode_closed_form(dt):
    """LINEAR model (i_ion = a V, gate rate lam_E): a cosine mode of the
    lumped Q1 operator with eigenvalue lam (its closed form on a uniform
    grid) gives V^{n+1} = (1 - dt a)/(1 - dt lam) V^n and the gate
    e^{dt lam_E} z^n, at any dt."""
    n, k = (17, 9), (3, 2)
    cfg = small_config("c1_2d_hh", n, model="LINEAR")
    cfg["stim"]["amp"] = 0.0
    h = cfg["h"]
    a, lamE = 0.3, -5.0
    prob = build_grid_problem(cfg, model_kw=dict(a=a, lam_E=lamE))
    V0 = _cosine_mode(n, k)
    # 1-D lumped Q1: L = [-1, 2, -1]/h^2, Mhat = [1/6, 2/3, 1/6], lumped to 1:
    # mode cos(pi k x/(n-1)) has eigenvalue (2 - 2c)/h^2 and mass (4 + 2c)/6
    c = [np.cos(np.pi * kk / (nn - 1)) for nn, kk in zip(n, k)]
    Lx, Ly = [(2 - 2 * cc) / hh ** 2 for cc, hh in zip(c, h)]
    Mx, My = [(4 + 2 * cc) / 6 for cc in c]
    lam = -cfg["sigma"][0] * (Lx * My + Mx * Ly) / (cfg["chi"] * cfg["Cm"])
    y0 = np.concatenate([V0, 0.5 * np.ones(prob.N)])
    y1 = imexrl_step(0.0, y0, dt, prob)
    assert np.abs(y1[:prob.N] - (1 - dt * a) / (1 - dt * lam) * V0).max() <= 1e-12
    assert np.abs(y1[prob.N:] - 0.5 * np.exp(dt * lamE)).max() <= 1e-14


def test_implicit_diffusion_is_bounded_at_large_steps():
    """dt rho_F = 100 and no ionic current: every step contracts V."""
    cfg = small_config("c2_3d_crn", (9, 7, 5), model="LINEAR")
    cfg["stim"]["amp"] = 0.0
    prob = build_grid_problem(cfg, model_kw=dict(a=0.0, lam_E=-1.0))
    rng = np.random.default_rng(2)
    y = np.concatenate([rng.standard_normal(prob.N), np.zeros(prob.N)])
    dt = 100.0 / 50.0
    for _ in range(20):
        y1 = imexrl_step(0.0, y, dt, prob)
        assert np.linalg.norm(y1[:prob.N]) <= np.linalg.norm(y[:prob.N]) * (1 + 1e-12)
        y = y1


def test_first_order_convergence_against_exexrl():
    cfg = small_config("c1_2d_hh", (17, 17))
    cfg["h"] = (1 / 16, 1 / 16)
    cfg["stim"]["amp"] = 40.0
    prob = build_grid_problem(cfg)
    y0 = prob.uniform_state()
    T = 2.0
    ref = exexrl_run(prob, y0, 0.0, 1e-4, int(round(T / 1e-4)))
    dts = [0.05, 0.025, 0.0125, 0.00625]
    errs = []
    for dt in dts:
        y = imexrl_run(prob, y0, 0.0, dt, int(round(T / dt)))
        errs.append(np.linalg.norm(y[:prob.N] - ref[:prob.N]) / np.linalg.norm(ref[:prob.N]))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(dts))
    assert np.all((slopes > 0.8) & (slopes < 1.2)), (errs, slopes)


@pytest.mark.parametrize("dt", [0.05, 1.0])
def test_cg_solve_matches_direct_solve(dt):
    """The symmetric CG form of the implicit line gives the LU solution."""
    cfg = small_config("c2_3d_crn", (11, 9, 5))
    prob = build_grid_problem(cfg)
    rng = np.random.default_rng(5)
    y = prob.uniform_state() * (1 + 1e-2 * rng.standard_normal(prob.nv * prob.N))
    a = imexrl_step(0.3, y, dt, prob)
    b = imexrl_step(0.3, y, dt, prob, imexrl_cg_solver(dt, prob))
    assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()
