"""Pins for the oracle's mRKC step (mRKC algorithm; the mRKC method for the
monodomain model; stability analysis of the mRKC method)."""
import numpy as np
import pytest
import scipy.linalg as la

from oracle.emrkc import emrkc_step, stage_counts
from oracle.exexrl import exexrl_run
from oracle.monodomain import build_grid_problem
from oracle.mrkc import MrkcSplit, mrkc_run, mrkc_step
from workloads.configs import small_config

from test_oracle_emrkc import P_cheb, Phi, ScalarTest


def test_split_sums_to_the_full_right_hand_side():
    """f~_F + f~_S = f_F + f_S + f_E, the stiffest gate's component in f~_F
    only, the other gates' in f~_S only (eq. mRCK_fFfS_monodomain)."""
    cfg = small_config("c2_3d_crn", (7, 5, 4))
    prob = build_grid_problem(cfg)
    rng = np.random.default_rng(2)
    y = prob.uniform_state() * (1 + 1e-2 * rng.standard_normal(prob.nv * prob.N))
    sp = MrkcSplit(prob, 0)
    full = prob.f_F(0.3, y) + prob.f_S(0.3, y) + prob.f_E(0.3, y)
    assert np.allclose(sp.f_F(0.3, y) + sp.f_S(0.3, y), full, rtol=1e-14, atol=1e-14 * np.abs(full).max())
    N = prob.N
    fE = prob.f_E(0.3, y)
    assert np.array_equal(sp.f_F(0.3, y)[N:2 * N], fE[N:2 * N])
    assert np.all(sp.f_F(0.3, y)[2 * N:] == 0)
    assert np.all(sp.f_S(0.3, y)[N:2 * N] == 0)


def test_scalar_test_equation_closed_form():
    """mRKC on y' = lam_F y + lam_S y: the averaged force is
    Phi_m(eta lam_F)(lam_F + lam_S) y (stability analysis), so
    y_{n+1} = P_s(dt Phi_m(eta lam_F)(lam_F + lam_S)) y_n; with f_E = 0 the
    emRKC step is the same step."""
    rng = np.random.default_rng(13)
    for _ in range(30):
        dt = 10 ** rng.uniform(-2, 0.5)
        rF = 10 ** rng.uniform(0, 4)
        rS = 10 ** rng.uniform(-1, 2)
        s, m, eta = stage_counts(dt, rF, rS)
        k = 64
        lF, lS = -rng.uniform(0, rF, k), -rng.uniform(0, rS, k)
        y0 = rng.uniform(0.5, 1.5, k)
        y1 = mrkc_step(0.0, y0, dt, lambda t, y: lF * y, lambda t, y: lS * y, rF, rS)
        ref = P_cheb(s, dt * Phi(m, eta * lF) * (lF + lS)) * y0
        assert np.abs(y1 - ref).max() <= 1e-11 * np.abs(ref).max() + 1e-14
        ye = emrkc_step(0.0, y0, dt, ScalarTest(lF, lS, np.zeros(k)), rF, rS)
        assert np.abs(ye - y1).max() <= 1e-13 * np.abs(y1).max()


@pytest.mark.parametrize("shape", [(3, 3), (4, 3, 2)])
def test_linear_model_matrix_function(shape):
    """LINEAR model (i_ion = a V, one gate with constant rate lam_E moved into
    f~_F): one mRKC step equals P_s(dt Phi_m(eta A_F)(A_F + A_S)) y0 with the
    matrices of f~_F and f~_S, evaluated by eigendecomposition."""
    base = "c2_3d_crn" if len(shape) == 3 else "c1_2d_hh"
    cfg = small_config(base, shape, model="LINEAR")
    if len(shape) == 2:
        cfg["h"] = (0.25, 0.25)
    cfg["stim"]["amp"] = 0.0  # linear (not affine) right-hand sides
    a, lamE = 0.7, -40.0
    prob = build_grid_problem(cfg, model_kw=dict(a=a, lam_E=lamE))
    sp = MrkcSplit(prob, 0)
    n = prob.nv * prob.N
    I = np.eye(n)
    AF = np.stack([sp.f_F(0.0, I[:, k]) for k in range(n)], axis=1)
    AS = np.stack([sp.f_S(0.0, I[:, k]) for k in range(n)], axis=1)
    rF = 1.05 * np.abs(np.linalg.eigvals(AF)).max()
    rS = 1.05 * np.abs(np.linalg.eigvals(AS)).max()
    dt = 0.05
    s, m, eta = stage_counts(dt, rF, rS)
    rng = np.random.default_rng(4)
    y0 = rng.uniform(-1, 1, n)
    y1 = mrkc_step(0.0, y0, dt, sp.f_F, sp.f_S, rF, rS)

    def matfun(A, f):
        w, Vr = la.eig(A)
        return (Vr @ np.diag(f(w)) @ la.inv(Vr)).real

    # Phi_m(0) = P_m'(0) = 1; the constant mode's eigenvalue comes out as
    # ~1e-16, where (P_m(z) - 1)/z cancels completely
    PhiF = matfun(eta * AF, lambda z: np.where(np.abs(z.real) < 1e-8, 1.0, Phi(m, z.real)))
    Mbar = PhiF @ (AF + AS)
    ref = matfun(dt * Mbar, lambda z: P_cheb(s, z.real)) @ y0
    assert np.abs(y1 - ref).max() <= 1e-10 * np.abs(ref).max()


def test_first_order_convergence_against_exexrl():
    """Error at T against EXEX-RL with dt = 1e-4 ms decays with slope ~1."""
    cfg = small_config("c1_2d_hh", (17, 17))
    cfg["h"] = (1 / 16, 1 / 16)
    cfg["stim"]["amp"] = 40.0
    prob = build_grid_problem(cfg)
    sp = MrkcSplit(prob, 0)
    y0 = prob.uniform_state()
    T = 2.0
    ref = exexrl_run(prob, y0, 0.0, 1e-4, int(round(T / 1e-4)))
    from oracle.powiter import compute_rho, random_unit_interval
    v0 = random_unit_interval(y0.size, 0)
    _, rF, _, _ = compute_rho(0.0, y0, sp.f_F, v0.copy())
    _, rS, _, _ = compute_rho(0.0, y0, sp.f_S, v0.copy())
    dts = [0.05, 0.025, 0.0125, 0.00625]
    errs = []
    for dt in dts:
        y = mrkc_run(sp, y0, 0.0, dt, int(round(T / dt)), 1.05 * rF, 1.05 * rS)
        errs.append(np.linalg.norm(y[:prob.N] - ref[:prob.N]) / np.linalg.norm(ref[:prob.N]))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(dts))
    assert np.all((slopes > 0.8) & (slopes < 1.2)), (errs, slopes)
