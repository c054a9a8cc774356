"""The emRKC step, written out from the emRKC algorithm (section "Pseudo-code
for the exponential multirate explicit stabilized method") on the full state
vector y = (V, z_E, z_S).  FP64 numpy.  Test infrastructure only.

Readings taken where the paper leaves a choice (each one listed in the design
notes of the repository):
  * the inner RKC iteration runs on the full state vector, literally;
  * the averaged force is evaluated at t_j = t_n + c_{j-1} dt with
    t_n = t0 + n*dt computed by multiplication, and f_S is frozen at that time
    for the whole inner iteration;
  * e^{eta*Lambda} - 1 is evaluated with expm1 (the identity the emRKC
    algorithm uses to avoid round-off for small eta*Lambda).
"""
import numpy as np

from .rkc import get_stages, rkc_iteration


def exponential_euler(y, eta, lam, yinf):
    """Exponential Euler step y + (e^{eta Lambda} - I)(y - y_inf) for diagonal
    Lambda (given as a vector), eq. exp_E with the identity of the emRKC
    algorithm."""
    return y + np.expm1(eta * lam) * (y - yinf)


def stage_counts(dt, rho_F, rho_S, eps=0.05):
    """(s, m, eta): s from rho_S and dt, eta = 2 dt / l_s, m from rho_F and eta
    (emRKC_Step; stability condition B of the stability lemma)."""
    s, ls = get_stages(dt, rho_S, eps)
    eta = 2.0 * dt / ls
    m, _ = get_stages(eta, rho_F, eps)
    return s, m, eta


def averaged_force(t, y, eta, prob, m, eps=0.05):
    """Averaged_Force of the emRKC algorithm: exponential Euler on the gates,
    then m inner RKC stages of u' = f_F(u) + f_S(t, y_E) from u(0) = y_E,
    returning (u_eta - y)/eta."""
    lam, yinf = prob.lambda_yinf(y)
    yE = exponential_euler(y, eta, lam, yinf)
    fS_frozen = prob.f_S(t, yE)

    def f_u(r, u):
        return prob.f_F(r, u) + fS_frozen

    u_eta = rkc_iteration(t, yE, eta, f_u, m, eps)
    return (u_eta - y) / eta


def emrkc_step(tn, yn, dt, prob, rho_F, rho_S, eps=0.05):
    """emRKC_Step: outer s-stage RKC iteration on the averaged force."""
    s, m, eta = stage_counts(dt, rho_F, rho_S, eps)

    def fbar(t, y):
        return averaged_force(t, y, eta, prob, m, eps)

    return rkc_iteration(tn, yn, dt, fbar, s, eps)


def emrkc_run(prob, y0, t0, dt, nsteps, rho_F, rho_S, eps=0.05, callback=None):
    """nsteps emRKC steps from (t0, y0); t_n = t0 + n*dt."""
    y = np.array(y0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        tn = t0 + n * dt
        y = emrkc_step(tn, y, dt, prob, rho_F, rho_S, eps)
        if callback is not None:
            callback(n + 1, y)
    return y
