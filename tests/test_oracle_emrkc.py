"""Pins for the oracle's emRKC step (emRKC algorithm; stability analysis of
the emRKC method; accuracy analysis), against closed forms, a matrix-function
brute force on tiny meshes, uniform-state reduction to the ionic ODE and the
first-order convergence against the fine EXEX-RL reference."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem
from oracle.emrkc import emrkc_run, emrkc_step, exponential_euler, stage_counts
from oracle.exexrl import exexrl_run
from oracle.ionic import HH, LinearTest, make_model
from oracle.monodomain import Monodomain, build_grid_problem
from oracle.rkc import beta_of
from workloads.configs import get_config, small_config


def P_cheb(s, z, eps=0.05):
    """Shifted Chebyshev stability polynomial T_s(w0 + w1 z)/T_s(w0) from
    the closed forms of T_s and T_s'."""
    w0 = 1.0 + eps / s ** 2
    th = math.acosh(w0)
    Ts = math.cosh(s * th)
    dTs = s * math.sinh(s * th) / math.sinh(th)
    w1 = Ts / dTs
    x = w0 + w1 * np.asarray(z, dtype=np.float64)
    xc = np.clip(x, -1, 1)
    inside = np.cos(s * np.arccos(xc))
    big = np.cosh(s * np.arccosh(np.maximum(np.abs(x), 1.0))) * np.where(x < 0, (-1.0) ** s, 1.0)
    return np.where(np.abs(x) <= 1, inside, big) / Ts


def Phi(m, z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z == 0, 1.0, (P_cheb(m, z) - 1.0) / np.where(z == 0, 1.0, z))


def phi(z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z == 0, 1.0, np.expm1(z) / np.where(z == 0, 1.0, z))


class ScalarTest:
    """y' = lam_F y + lam_S y + lam_E y on independent scalar components."""

    def __init__(self, lF, lS, lE):
        self.lF, self.lS, self.lE = map(np.asarray, (lF, lS, lE))

    def f_F(self, t, y):
        return self.lF * y

    def f_S(self, t, y):
        return self.lS * y

    def lambda_yinf(self, y):
        return self.lE * np.ones_like(y), np.zeros_like(y)


def test_scalar_test_equation_closed_form():
    """y_{n+1} = P_s(dt lam_bar) y_n with
    lam_bar = Phi_m(eta lam_F)(lam_F + lam_S) e^{eta lam_E} + phi(eta lam_E) lam_E."""
    rng = np.random.default_rng(11)
    for _ in range(40):
        dt = 10 ** rng.uniform(-2, 0.5)
        rho_F = 10 ** rng.uniform(0, 4)
        rho_S = 10 ** rng.uniform(-1, 2)
        s, m, eta = stage_counts(dt, rho_F, rho_S)
        k = 64
        lF = -rng.uniform(0, rho_F, k)
        lS = -rng.uniform(0, rho_S, k)
        lE = -10 ** rng.uniform(-2, 3, k)
        prob = ScalarTest(lF, lS, lE)
        y0 = rng.uniform(0.5, 1.5, k)
        y1 = emrkc_step(0.0, y0, dt, prob, rho_F, rho_S)
        lbar = Phi(m, eta * lF) * (lF + lS) * np.exp(eta * lE) + phi(eta * lE) * lE
        ref = P_cheb(s, dt * lbar) * y0
        assert np.abs(y1 - ref).max() <= 1e-12 * np.abs(ref).max() + 1e-14
        # stability theorem of the emRKC method: wherever the mRKC condition
        # -l_s <= dt Phi_m(eta lam_F)(lam_F + lam_S) <= 0 holds, any
        # lam_E <= 0 keeps the amplification factor within [-1, 1]
        ls = beta_of(0.05) * s * s
        x = dt * Phi(m, eta * lF) * (lF + lS)
        hyp = (x >= -ls) & (x <= 0)
        assert hyp.sum() > 0
        assert np.all(np.abs(ref / y0)[hyp] <= 1.0 + 1e-12)


def test_exponential_euler_exact_for_frozen_rates():
    """With Lambda and y_inf constant the exponential Euler step is the exact
    flow y_inf + e^{eta Lambda}(y - y_inf)."""
    rng = np.random.default_rng(2)
    y = rng.uniform(0, 1, 100)
    lam = -10 ** rng.uniform(-6, 4, 100)
    yinf = rng.uniform(0, 1, 100)
    for eta in [1e-6, 0.05, 3.0]:
        got = exponential_euler(y, eta, lam, yinf)
        ref = yinf + np.exp(eta * lam) * (y - yinf)
        assert np.abs(got - ref).max() < 1e-15
        assert np.all((got >= 0) & (got <= 1))


def cosine_mode(n, ks):
    vecs = [np.cos(np.pi * k * np.arange(nn) / (nn - 1)) for nn, k in zip(n, ks)]
    v = vecs[0]
    for w in vecs[1:]:
        v = np.multiply.outer(w, v)
    return v.reshape(-1)


@pytest.mark.parametrize("s_target", [1, 3])
def test_linear_model_on_cosine_mode(s_target):
    """LINEAR model, V0 a cosine mode (eigenvector of M_L^{-1}K with known
    eigenvalue), decoupled gate with constant lam_E: the step is exactly
    V1 = P_s(dt Phi_m(eta lam_F)(lam_F + lam_S)) V0 and
    z1 = P_s(dt phi(eta lam_E) lam_E) z0."""
    n, h, sig = (9, 7), (0.125, 0.125), (0.1, 0.04)
    chi, Cm, a, lamE = 1.3, 0.7, 2.0, -40.0
    K, ML, _ = fem.assemble_q1_grid(list(n), list(h), list(sig))
    prob = Monodomain(K, ML, chi, Cm, LinearTest(a=a, lam_E=lamE))
    ks = (3, 2)
    th = [np.pi * k / (nn - 1) for k, nn in zip(ks, n)]
    lam_d = [(2 - 2 * np.cos(t)) / hh ** 2 for t, hh in zip(th, h)]
    mu_d = [(2 + np.cos(t)) / 3 for t in th]
    eig = sig[0] * lam_d[0] * mu_d[1] + sig[1] * lam_d[1] * mu_d[0]
    lF = -eig / (chi * Cm)
    lS = -a
    V0 = cosine_mode(n, ks)
    N = V0.size
    z0 = np.linspace(0.2, 0.9, N)
    y0 = np.concatenate([V0, z0])
    rho_F = 4 * max(sig) / 0.125 ** 2 / (chi * Cm) * 1.05
    dt = 0.08 if s_target == 1 else 4.0
    rho_S = a * 1.05
    s, m, eta = stage_counts(dt, rho_F, rho_S)
    assert s == s_target
    y1 = emrkc_step(0.0, y0, dt, prob, rho_F, rho_S)
    ampV = P_cheb(s, dt * Phi(m, eta * lF) * (lF + lS))
    ampZ = P_cheb(s, dt * phi(eta * lamE) * lamE)
    assert np.abs(y1[:N] - ampV * V0).max() < 1e-13
    assert np.abs(y1[N:] - ampZ * z0).max() < 1e-13


@pytest.mark.parametrize("shape", [(3, 3), (4, 3), (3, 2, 2)])
def test_linear_model_matrix_function_brute_force(shape):
    """Tiny meshes, arbitrary V0: the emRKC step for the LINEAR model is the
    matrix polynomial P_s(dt Phi_m(eta F)(F + lam_S I)) V0 with
    F = -(chi Cm M_L)^{-1}K, evaluated through the eigendecomposition of the
    symmetrised operator."""
    d = len(shape)
    h = [0.3, 0.25, 0.2][:d]
    sig = [0.2, 0.05, 0.1][:d]
    chi, Cm, a = 1.0, 1.0, 0.5
    K, ML, _ = fem.assemble_q1_grid(list(shape), h, sig)
    prob = Monodomain(K, ML, chi, Cm, LinearTest(a=a, lam_E=-3.0))
    N = ML.size
    rng = np.random.default_rng(5)
    V0 = rng.normal(size=N)
    y0 = np.concatenate([V0, rng.uniform(size=N)])
    Ms = 1.0 / np.sqrt(ML)
    S = (K.toarray() * Ms).T * Ms / (chi * Cm)
    w, Q = np.linalg.eigh(S)           # F = -M^{-1/2} S M^{1/2}
    w[np.abs(w) < 1e-12 * w.max()] = 0.0   # the constant mode (K.1 = 0)
    lF = -w
    rho_F = w.max() * 1.05
    for dt, rho_S in [(0.05, 0.6), (1.5, 0.6), (0.4, 30.0)]:
        s, m, eta = stage_counts(dt, rho_F, rho_S)
        amp = P_cheb(s, dt * Phi(m, eta * lF) * (lF - a))
        x = Q.T @ (V0 / Ms)
        ref = Ms * (Q @ (amp * x))
        y1 = emrkc_step(0.0, y0, dt, prob, rho_F, rho_S)
        assert np.abs(y1[:N] - ref).max() < 1e-12 * np.abs(V0).max()


def test_uniform_state_reduces_to_ionic_ode():
    """K.1 = 0: a spatially uniform state with a uniform stimulus stays
    uniform and equals the same step on a single node (no diffusion)."""
    cfg = small_config("c2_3d_crn", (6, 5, 4))
    prob = build_grid_problem(cfg, stim_mask=np.ones(6 * 5 * 4, np.uint8))
    one = Monodomain(sp.csr_matrix((1, 1)), np.ones(1), cfg["chi"], cfg["Cm"],
                     make_model("CRN_SURR"), np.ones(1, np.uint8), cfg["stim"]["amp"],
                     cfg["stim"]["t_on"], cfg["stim"]["t_off"])
    y = prob.uniform_state()
    y1 = one.uniform_state()
    rho_F, rho_S = 51.0, 30.0    # s = 1, m = 2 at dt = 0.05
    yn = emrkc_run(prob, y, 0.0, 0.05, 60, rho_F, rho_S)
    y1n = emrkc_run(one, y1, 0.0, 0.05, 60, rho_F, rho_S)
    Y = yn.reshape(prob.nv, prob.N)
    assert np.abs(Y - Y[:, :1]).max() <= 1e-12 * np.abs(Y).max()
    assert np.abs(Y[:, 0] - y1n).max() <= 1e-12 * np.abs(y1n).max()
    assert abs(Y[0, 0] - y1[0]) > 10.0    # the uniform stimulus excited the cell


@pytest.mark.slow
def test_first_order_convergence_against_exexrl():
    """Error at T against EXEX-RL with dt = 1e-4 ms decays with slope ~1 in dt
    (first-order theorem of the accuracy analysis)."""
    cfg = small_config("c1_2d_hh", (17, 17))
    cfg["h"] = (1 / 16, 1 / 16)
    cfg["stim"]["amp"] = 40.0
    prob = build_grid_problem(cfg)
    y0 = prob.uniform_state()
    T = 2.0
    ref = exexrl_run(prob, y0, 0.0, 1e-4, int(round(T / 1e-4)))
    rho_F = 4 * 0.1 * 16 ** 2 * 1.05
    rho_S = 0.75
    dts = [0.05, 0.025, 0.0125, 0.00625]
    errs = []
    for dt in dts:
        y = emrkc_run(prob, y0, 0.0, dt, int(round(T / dt)), rho_F, rho_S)
        errs.append(np.linalg.norm(y[:prob.N] - ref[:prob.N]) / np.linalg.norm(ref[:prob.N]))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(dts))
    assert np.all((slopes > 0.8) & (slopes < 1.2)), (errs, slopes)


def test_stage_counts_c1():
    """C1 (unit square, h = 1/64, sigma = 0.1, chi = Cm = 1): the closed-form
    rho_F = 4 sigma/h^2 with the safety factor gives s = 1, m = 7."""
    rho_F = 4 * 0.1 * 64 ** 2 * 1.05
    s, m, eta = stage_counts(0.05, rho_F, 0.71)
    assert (s, m) == (1, 7)
    assert eta == pytest.approx(2 * 0.05 / beta_of(0.05))
