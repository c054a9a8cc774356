"""Runge-Kutta-Chebyshev building blocks (first-order RKC with damping).

Follows the RKC algorithm of the section "Explicit stabilized methods":
``get_stages``, ``get_coeffs`` and ``RKC_Iteration``.  FP64 numpy.
Test infrastructure only.
"""
import math

import numpy as np


def beta_of(eps):
    """Stability-interval constant beta = 2 - 4*eps/3 (RKC algorithm, get_stages)."""
    return 2.0 - 4.0 * eps / 3.0


def get_stages(dt, rho, eps=0.05):
    """Number of stages s and stability length l_s = beta*s^2.

    s = ceil(sqrt(dt*rho/beta)), clamped to at least 1 (with rho -> 0 the
    formula would give s = 0, which is not a method).
    """
    beta = beta_of(eps)
    s = max(1, int(math.ceil(math.sqrt(dt * rho / beta))))
    return s, beta * s * s


def chebyshev_T(s, x):
    """T_0(x) .. T_s(x) by the three-term recurrence T_j = 2x T_{j-1} - T_{j-2}."""
    T = np.empty(s + 1)
    T[0] = 1.0
    if s >= 1:
        T[1] = x
    for j in range(2, s + 1):
        T[j] = 2.0 * x * T[j - 1] - T[j - 2]
    return T


def chebyshev_dT(s, x):
    """T_0'(x) .. T_s'(x) by differentiating the recurrence:
    T_j' = 2 T_{j-1} + 2x T_{j-1}' - T_{j-2}'."""
    T = chebyshev_T(s, x)
    dT = np.empty(s + 1)
    dT[0] = 0.0
    if s >= 1:
        dT[1] = 1.0
    for j in range(2, s + 1):
        dT[j] = 2.0 * T[j - 1] + 2.0 * x * dT[j - 1] - dT[j - 2]
    return dT


def get_coeffs(s, eps=0.05):
    """RKC coefficients mu_j, nu_j, kappa_j (j = 1..s) and c_j (j = 0..s).

    omega0 = 1 + eps/s^2, omega1 = T_s(omega0)/T_s'(omega0), b_j = 1/T_j(omega0),
    mu_1 = omega1/omega0, c_1 = mu_1 and for j >= 2
    mu_j = 2 omega1 b_j/b_{j-1}, nu_j = 2 omega0 b_j/b_{j-1},
    kappa_j = -b_j/b_{j-2}, c_j = nu_j c_{j-1} + kappa_j c_{j-2} + mu_j.
    Arrays are indexed by j; unused entries (nu_1, kappa_1, index 0) are 0.
    """
    w0 = 1.0 + eps / (s * s)
    T = chebyshev_T(s, w0)
    dT = chebyshev_dT(s, w0)
    w1 = T[s] / dT[s]
    b = 1.0 / T
    mu = np.zeros(s + 1)
    nu = np.zeros(s + 1)
    kappa = np.zeros(s + 1)
    c = np.zeros(s + 1)
    mu[1] = w1 / w0
    c[1] = mu[1]
    for j in range(2, s + 1):
        mu[j] = 2.0 * w1 * b[j] / b[j - 1]
        nu[j] = 2.0 * w0 * b[j] / b[j - 1]
        kappa[j] = -b[j] / b[j - 2]
        c[j] = nu[j] * c[j - 1] + kappa[j] * c[j - 2] + mu[j]
    return dict(mu=mu, nu=nu, kappa=kappa, c=c, w0=w0, w1=w1, b=b)


def rkc_iteration(t, y, dt, f, s, eps=0.05):
    """RKC_Iteration: g_0 = y, g_1 = g_0 + mu_1 dt f(t, g_0),
    g_j = nu_j g_{j-1} + kappa_j g_{j-2} + mu_j dt f(t + c_{j-1} dt, g_{j-1})."""
    cf = get_coeffs(s, eps)
    mu, nu, kappa, c = cf["mu"], cf["nu"], cf["kappa"], cf["c"]
    g_prev2 = y
    g_prev = y + mu[1] * dt * f(t, y)
    for j in range(2, s + 1):
        g = nu[j] * g_prev + kappa[j] * g_prev2 + mu[j] * dt * f(t + c[j - 1] * dt, g_prev)
        g_prev2, g_prev = g_prev, g
    return g_prev
