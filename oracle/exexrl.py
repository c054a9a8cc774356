"""EXEX-RL: the IMEX Rush-Larsen step of the section "Numerical experiments"
with its implicit diffusion solve replaced by an explicit update (the fine
reference method of the error measurements).  FP64 numpy.
Test infrastructure only.

  z_E^{n+1} = z_E + (e^{dt Lambda_E(V_n)} - 1)(z_E - z_inf(V_n))
  z_S^{n+1} = z_S + dt g_S(V_n, z_E^{n+1}, z_S^n)
  V^{n+1}   = V_n + dt [ (chi Cm M_L)^{-1} A V_n
                          + Cm^{-1}(I_stim(t_n) - I_ion(V_n, z_E^{n+1}, z_S^{n+1})) ]
"""
import numpy as np


def exexrl_step(tn, y, dt, prob):
    V, zE, zS = prob.split(y)
    LE, zinf = prob.model.gates(V)
    zE1 = zE + np.expm1(dt * LE) * (zE - zinf)
    zS1 = zS + dt * prob.model.g_S(V, zE1, zS) if prob.nS else zS
    diff = (prob.A @ V) / (prob.chi * prob.Cm * prob.ML)
    I_ion = prob.Cm * prob.model.i_ion(V, zE1, zS1)
    V1 = V + dt * (diff + (prob.I_stim(tn) - I_ion) / prob.Cm)
    return np.concatenate([V1, zE1.reshape(-1), np.asarray(zS1).reshape(-1)])


def exexrl_run(prob, y0, t0, dt, nsteps):
    y = np.array(y0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        y = exexrl_step(t0 + n * dt, y, dt, prob)
    return y
