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

Stepping variants (the rows after the plain method):
  * stability condition A of the stability lemma for (s, m, eta) instead of
    condition B (``cond="A"``);
  * the progressive splitting of the auxiliary problem of the remark after
    eq. auxp_exp (``progressive=True``);
  * re-estimation of the radii every K steps, warm started from the previous
    estimate as the appendix suggests (``emrkc_run(..., rho_every=K)``).
"""
import numpy as np

from .rkc import get_stages, rkc_iteration


def exponential_euler(y, eta, lam, yinf):
    """Exponential Euler step y + (e^{eta Lambda} - I)(y - y_inf) for diagonal
    Lambda (given as a vector), eq. exp_E with the identity of the emRKC
    algorithm."""
    return y + np.expm1(eta * lam) * (y - yinf)


def stage_counts(dt, rho_F, rho_S, eps=0.05, cond="B"):
    """(s, m, eta): s from rho_S and dt (dt rho_S <= l_s), then
      condition B (emRKC_Step): eta = 2 dt / l_s and m from rho_F and eta;
      condition A: eta = (6 dt / l_s) m^2 / (m^2 - 1) with the smallest
        m >= 2 such that eta rho_F <= l_m = beta m^2 (eta depends on m, so
        m is searched upwards; eta decreases and l_m grows with m).
    l_s = beta s^2, l_m = beta m^2 (stability lemma)."""
    s, ls = get_stages(dt, rho_S, eps)
    if cond == "B":
        eta = 2.0 * dt / ls
        m, _ = get_stages(eta, rho_F, eps)
        return s, m, eta
    if cond != "A":
        raise ValueError(cond)
    beta = 2.0 - 4.0 * eps / 3.0
    m = 2
    while True:
        eta = (6.0 * dt / ls) * (m * m / (m * m - 1.0))
        if eta * rho_F <= beta * m * m:
            return s, m, eta
        m += 1


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


def averaged_force_progressive(t, y, eta, prob, m, eps=0.05):
    """The progressive splitting of the remark after eq. auxp_exp: y_E as
    before, but the inner problem starts from u(0) = y and carries the
    exponential increment as a constant forcing,
      u' = f_F(u) + f_S(t, y_E) + phi(eta Lambda(y)) f_E(y),
    where phi(eta Lambda) f_E(y) = (y_E - y)/eta."""
    lam, yinf = prob.lambda_yinf(y)
    yE = exponential_euler(y, eta, lam, yinf)
    forcing = prob.f_S(t, yE) + (yE - y) / eta

    def f_u(r, u):
        return prob.f_F(r, u) + forcing

    u_eta = rkc_iteration(t, y, eta, f_u, m, eps)
    return (u_eta - y) / eta


def emrkc_step(tn, yn, dt, prob, rho_F, rho_S, eps=0.05, cond="B", progressive=False):
    """emRKC_Step: outer s-stage RKC iteration on the averaged force."""
    s, m, eta = stage_counts(dt, rho_F, rho_S, eps, cond)
    af = averaged_force_progressive if progressive else averaged_force

    def fbar(t, y):
        return af(t, y, eta, prob, m, eps)

    return rkc_iteration(tn, yn, dt, fbar, s, eps)


def emrkc_run(prob, y0, t0, dt, nsteps, rho_F, rho_S, eps=0.05, callback=None, cond="B",
              progressive=False, rho_every=0, rho_state=None, safety=1.05, on_estimate=None):
    """nsteps emRKC steps from (t0, y0); t_n = t0 + n*dt.

    rho_every = K > 0: before every step n that is a positive multiple of K
    the radii are estimated again with Compute_Rho on (t_n, y_n), warm
    started from rho_state = {"vF", "vS", "rF", "rS"} (the raw estimates and
    eigenvector guesses of the previous call, updated in place), and
    multiplied by `safety`.  on_estimate(n, rho_F, rho_S, itF, itS) is called
    after each estimate."""
    from .powiter import compute_rho
    y = np.array(y0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        tn = t0 + n * dt
        if rho_every > 0 and n > 0 and n % rho_every == 0:
            vF, rF, itF, _ = compute_rho(tn, y, prob.f_F, rho_state["vF"], rho_state["rF"])
            vS, rS, itS, _ = compute_rho(tn, y, prob.f_S, rho_state["vS"], rho_state["rS"])
            rho_state.update(vF=vF, vS=vS, rF=rF, rS=rS)
            rho_F, rho_S = safety * rF, safety * rS
            if on_estimate is not None:
                on_estimate(n, rho_F, rho_S, itF, itS)
        y = emrkc_step(tn, y, dt, prob, rho_F, rho_S, eps, cond, progressive)
        if callback is not None:
            callback(n + 1, y)
    return y
