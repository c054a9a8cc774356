"""Pins for the RKC building blocks of the oracle (RKC algorithm, section
"Explicit stabilized methods"; identities of the accuracy analysis)."""
import json
import math
import os

import numpy as np
import pytest

from oracle.rkc import beta_of, get_coeffs, get_stages, rkc_iteration

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def closed_T(s, x):
    return math.cosh(s * math.acosh(x))


def closed_dT(s, x):
    th = math.acosh(x)
    return s * math.sinh(s * th) / math.sinh(th)


def closed_U(k, x):
    th = math.acosh(x)
    return math.sinh((k + 1) * th) / math.sinh(th)


def test_beta_matches_paper_formula():
    eps = GOLDEN["rkc_damping_eps"]["value"]
    assert beta_of(eps) == pytest.approx(2.0 - 4.0 * 0.05 / 3.0, rel=0, abs=0)
    assert beta_of(eps) == pytest.approx(1.9333333333333333, abs=1e-15)


@pytest.mark.parametrize("s", [1, 2, 3, 5, 8, 17, 50, 137, 500])
def test_coeffs_against_closed_form_chebyshev(s):
    """mu, nu, kappa from cosh/sinh closed forms of T_j and T_s'."""
    eps = 0.05
    cf = get_coeffs(s, eps)
    w0 = 1.0 + eps / s ** 2
    assert cf["w0"] == w0
    w1 = closed_T(s, w0) / closed_dT(s, w0)
    assert cf["w1"] == pytest.approx(w1, rel=1e-13)
    b = [1.0 / closed_T(j, w0) for j in range(s + 1)]
    assert cf["mu"][1] == pytest.approx(w1 / w0, rel=1e-13)
    for j in range(2, s + 1):
        assert cf["mu"][j] == pytest.approx(2 * w1 * b[j] / b[j - 1], rel=1e-12)
        assert cf["nu"][j] == pytest.approx(2 * w0 * b[j] / b[j - 1], rel=1e-12)
        assert cf["kappa"][j] == pytest.approx(-b[j] / b[j - 2], rel=1e-12)


@pytest.mark.parametrize("s", list(range(2, 40)) + [100, 250, 500])
def test_nu_plus_kappa_is_one(s):
    """nu_j + kappa_j = 1 (used in the accuracy analysis to pass to d_j)."""
    cf = get_coeffs(s)
    for j in range(2, s + 1):
        assert cf["nu"][j] + cf["kappa"][j] == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("s", list(range(1, 60)) + [100, 200, 300, 400, 500])
def test_c_s_is_one(s):
    """c_s = 1: the last stage sits at t + dt (first-order consistency)."""
    assert get_coeffs(s)["c"][s] == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 7, 12, 33, 100])
def test_accuracy_identity_sum_bs_over_bj_U_mu(s):
    """sum_j (b_s/b_j) U_{s-j}(w0) mu_j = 1 (accuracy analysis), with U from
    its closed form."""
    cf = get_coeffs(s)
    w0 = cf["w0"]
    b = cf["b"]
    tot = sum(b[s] / b[j] * closed_U(s - j, w0) * cf["mu"][j] for j in range(1, s + 1))
    assert tot == pytest.approx(1.0, abs=1e-12)


def P_closed(s, z, eps=0.05):
    w0 = 1.0 + eps / s ** 2
    w1 = closed_T(s, w0) / closed_dT(s, w0)
    x = w0 + w1 * z
    if abs(x) <= 1.0:
        Tx = math.cos(s * math.acos(x))
    elif x > 1:
        Tx = math.cosh(s * math.acosh(x))
    else:
        Tx = (-1) ** s * math.cosh(s * math.acosh(-x))
    return Tx / closed_T(s, w0)


@pytest.mark.parametrize("s", [1, 2, 3, 6, 10, 25])
def test_rkc_iteration_linear_is_chebyshev_polynomial(s):
    """RKC on y' = lambda y gives P_s(dt lambda) y0 with the shifted Chebyshev
    stability polynomial T_s(w0 + w1 z)/T_s(w0)."""
    beta = beta_of(0.05)
    lam = -np.linspace(0.0, beta * s * s, 41)
    dt = 1.0
    y = rkc_iteration(0.0, np.ones_like(lam), dt, lambda t, y: lam * y, s)
    ref = np.array([P_closed(s, dt * l) for l in lam])
    assert np.max(np.abs(y - ref)) < 1e-12


@pytest.mark.parametrize("s", [1, 2, 3, 5, 10, 40, 100, 500])
def test_damping_bound_on_stability_interval(s):
    """|P_s(z)| <= 1/T_s(w0) < 1 on [-beta s^2, -delta] (damping), evaluated on
    a dense grid; also checks beta s^2 does not exceed the exact stability
    length (1 + w0)/w1."""
    eps = 0.05
    w0 = 1.0 + eps / s ** 2
    w1 = closed_T(s, w0) / closed_dT(s, w0)
    assert beta_of(eps) * s * s <= (1.0 + w0) / w1 + 1e-12
    delta = (w0 - 1.0) / w1          # where w0 + w1 z = 1
    zs = -np.linspace(delta, beta_of(eps) * s * s, 2001)
    bound = 1.0 / closed_T(s, w0)
    vals = np.array([abs(P_closed(s, z)) for z in zs])
    assert np.all(vals <= bound + 1e-12)
    assert bound < 1.0


def test_rkc_constant_forcing_reaches_t_plus_dt():
    """With f constant, g_j = y0 + c_j dt f, so the result is y0 + c_s dt f."""
    for s in [1, 2, 5, 9]:
        y = rkc_iteration(0.0, np.array([2.0]), 0.3, lambda t, y: np.array([1.5]), s)
        assert y[0] == pytest.approx(2.0 + 0.3 * 1.5, abs=1e-13)


def test_rkc_stage_times():
    """f(t) = t integrates to dt^2/2 at first order: stage times c_j dt are
    passed to f (exact for s=1: t0*dt)."""
    seen = []

    def f(t, y):
        seen.append(t)
        return np.zeros(1)

    rkc_iteration(1.0, np.zeros(1), 0.5, f, 4)
    cf = get_coeffs(4)
    assert seen[0] == 1.0
    for j in range(2, 5):
        assert seen[j - 1] == 1.0 + cf["c"][j - 1] * 0.5


@pytest.mark.parametrize("k", [1, 2, 3, 7, 20, 100])
def test_get_stages_bracket(k):
    beta = beta_of(0.05)
    s, ls = get_stages(1.0, beta * k * k * (1 - 1e-9))
    assert s == k and ls == pytest.approx(beta * k * k)
    s, _ = get_stages(1.0, beta * k * k * (1 + 1e-9))
    assert s == k + 1


def test_get_stages_random_bracket():
    rng = np.random.default_rng(7)
    beta = beta_of(0.05)
    for _ in range(1000):
        dt = 10 ** rng.uniform(-3, 0)
        rho = 10 ** rng.uniform(-2, 5)
        s, _ = get_stages(dt, rho)
        assert s >= 1
        assert dt * rho <= beta * s * s * (1 + 1e-14)
        if s > 1:
            assert beta * (s - 1) ** 2 < dt * rho


def test_get_stages_zero_rho_is_one_stage():
    assert get_stages(0.1, 0.0)[0] == 1
