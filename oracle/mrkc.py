"""The mRKC step for the monodomain model, written out from the mRKC algorithm
(section "Multirate explicit stabilized method algorithm") and the way the
paper applies it to the monodomain model (section "The mRKC method for the
monodomain model", eq. mono_in_FS and eq. mRCK_fFfS_monodomain).  FP64
numpy.  Test infrastructure only.

The ionic term f_E is split into f_E^1, the component of the stiffest gate,
which joins the diffusion in the fast term, and f_E^2, the other gates,
which join the slow term:
    f~_F = f_F + f_E^1,   f~_S = f_S + f_E^2.
The mRKC step is then the multirate RKC step of f~_F + f~_S: an outer
s-stage RKC iteration on the averaged force, whose inner m-stage RKC
iteration integrates u' = f~_F(u) + f~_S(t, y) from u(0) = y over [0, eta]
(no exponential stage).  Stage counts follow the same get_stages rules on
the radii of f~_F and f~_S.
"""
import numpy as np

from .emrkc import stage_counts
from .rkc import rkc_iteration


class MrkcSplit:
    """f~_F and f~_S of a Monodomain problem, with the gate `stiff_gate`
    (index among the gates) moved into the fast term."""

    def __init__(self, prob, stiff_gate=0):
        self.prob = prob
        N = prob.N
        self.gate = slice(N * (1 + stiff_gate), N * (2 + stiff_gate))

    def f_F(self, t, y):
        out = self.prob.f_F(t, y)
        out[self.gate] += self.prob.f_E(t, y)[self.gate]
        return out

    def f_S(self, t, y):
        fE = self.prob.f_E(t, y)
        fE[self.gate] = 0.0
        return self.prob.f_S(t, y) + fE


def averaged_force(t, y, eta, f_F, f_S, m, eps=0.05):
    """Averaged_Force of the mRKC algorithm: m inner RKC stages of
    u' = f_F(u) + f_S(t, y) (f_S frozen at the outer stage) from u(0) = y;
    returns (u_eta - y)/eta."""
    fS_frozen = f_S(t, y)

    def f_u(r, u):
        return f_F(r, u) + fS_frozen

    u_eta = rkc_iteration(t, y, eta, f_u, m, eps)
    return (u_eta - y) / eta


def mrkc_step(tn, yn, dt, f_F, f_S, rho_F, rho_S, eps=0.05, cond="B"):
    """mRKC_Step: s, eta, m from the radii, then the outer RKC iteration on
    the averaged force."""
    s, m, eta = stage_counts(dt, rho_F, rho_S, eps, cond)

    def fbar(t, y):
        return averaged_force(t, y, eta, f_F, f_S, m, eps)

    return rkc_iteration(tn, yn, dt, fbar, s, eps)


def mrkc_run(split, y0, t0, dt, nsteps, rho_F, rho_S, eps=0.05, callback=None):
    """nsteps mRKC steps of a MrkcSplit from (t0, y0); t_n = t0 + n*dt."""
    y = np.array(y0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        y = mrkc_step(t0 + n * dt, y, dt, split.f_F, split.f_S, rho_F, rho_S, eps)
        if callback is not None:
            callback(n + 1, y)
    return y
