"""Pins of the oracle's nonlinear trajectories that do not come from the
oracle itself.

On a single cell (no diffusion, section "The monodomain model" without the
divergence term) the monodomain model is the cell ODE system:
  dV/dt = I_stim/Cm - i_ion(V, z),  dz_E/dt = Lambda_E(V) (z_E - z_inf(V))
(the gate equation in exponential form) and dz_S/dt = g_S(V, z).  scipy's
Radau integrator (implicit, order 5, tight tolerances) solves it here from
the model's rates and currents; the oracle's emRKC run on the same cell must
converge to that solution at first order (the first-order theorem of the
accuracy analysis).  This checks the whole nonlinear step (exponential
Euler, averaged force, RKC stages, stimulus window) against an independent
integrator, on the classical Hodgkin-Huxley model and both surrogates.

The HH constants are pinned by the classical model's resting potential:
with the leak reversal at -54.387 mV the membrane rests at -65 mV."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

from oracle.emrkc import emrkc_run
from oracle.ionic import make_model
from oracle.monodomain import Monodomain


def cell_ode(model, Cm, amp, t_on, t_off):
    nE = model.n_gates

    def f(t, y):
        V = y[0:1]
        zE = y[1:1 + nE].reshape(nE, 1)
        zS = y[1 + nE:].reshape(-1, 1)
        lam, zinf = model.gates(V)
        Is = amp if t_on <= t <= t_off else 0.0
        dV = Is / Cm - model.i_ion(V, zE, zS)
        dzE = lam[:, 0] * (zE[:, 0] - zinf[:, 0])
        dzS = model.g_S(V, zE, zS).reshape(-1)
        return np.concatenate([dV, dzE, dzS])

    return f


# (model, Cm, stimulus amplitude, stimulus end, T, rho_S): a 1 ms (HH) or
# 2 ms (surrogates, tissue units of the cuboid workload) stimulus that fires
# an action potential, followed to T = 5 ms through the repolarisation
CASES = [("HH", 1.0, 20.0, 1.0, 5.0, 140.0),
         ("CRN_SURR", 0.01, 50.0 / 140.0, 2.0, 5.0, 40.0),
         ("TTP_SURR", 0.01, 50.0 / 140.0, 2.0, 5.0, 40.0)]


@pytest.mark.slow
@pytest.mark.parametrize("name,Cm,amp,t_off,T,rho_S", CASES)
def test_single_cell_converges_to_radau_solution(name, Cm, amp, t_off, T, rho_S):
    model = make_model(name)
    cell = Monodomain(sp.csr_matrix((1, 1)), np.ones(1), 140.0, Cm, model, np.ones(1, np.uint8), amp, 0.0, t_off)
    y0 = cell.uniform_state()
    f = cell_ode(model, Cm, amp, 0.0, t_off)
    # the stimulus switches off at t_off: integrate the two smooth pieces
    a = solve_ivp(f, (0.0, t_off), y0, method="Radau", rtol=1e-11, atol=1e-12)
    b = solve_ivp(f, (t_off, T), a.y[:, -1], method="Radau", rtol=1e-11, atol=1e-12)
    assert a.success and b.success
    ref = b.y[:, -1]
    assert max(a.y[0].max(), b.y[0].max()) > 20.0     # an action potential fired
    dts = [0.01, 0.005, 0.0025]
    errs = []
    for dt in dts:
        y = emrkc_run(cell, y0, 0.0, dt, int(round(T / dt)), 1.0, rho_S)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[-1] < 5e-4, errs
    # first order: halving dt takes off close to half of the error
    ratios = [errs[k] / errs[k + 1] for k in range(len(dts) - 1)]
    assert ratios[-1] > 1.6 and all(r > 1.3 for r in ratios), (errs, ratios)


def test_hh_rests_at_minus_65_mV():
    model = make_model("HH")

    def current_at_steady_gates(V):
        v = np.array([V])
        _, zinf = model.gates(v)
        return float(model.i_ion(v, zinf, np.zeros((0, 1)))[0])

    V_rest = brentq(current_at_steady_gates, -80.0, -55.0, xtol=1e-12)
    assert abs(V_rest - (-65.0)) < 0.05, V_rest
    assert np.allclose(model.rest()[0], -65.0)
