"""The semi-discrete monodomain system in F/S/E form (eq. sd_sys and
eq. mono_in_FSE), on the full state y = (V, z_E, z_S) stored as one flat
vector [V (N), gate_0 (N), ..., gate_{nE-1} (N), slow_0 (N), ...].
FP64 numpy/scipy.  Test infrastructure only.

  f_F(t, y) = ((chi Cm M_L)^{-1} A V, 0, 0)            with A = -K
  f_S(t, y) = (Cm^{-1}(I_stim(t) - I_ion), 0, g_S)      with I_ion = Cm i_ion
  f_E(t, y) = Lambda(y)(y - y_inf(y))                   gates only

I_stim(t) = amp * mask on the closed window t_on <= t <= t_off (nodal values,
ionic current interpolation).
"""
import numpy as np

from . import fem
from .ionic import make_model


class Monodomain:
    def __init__(self, K, ML, chi, Cm, model, stim_mask=None, stim_amp=0.0,
                 t_on=0.0, t_off=-1.0):
        self.A = (-K).tocsr()
        self.ML = np.asarray(ML, dtype=np.float64)
        self.N = self.ML.size
        self.chi = float(chi)
        self.Cm = float(Cm)
        self.model = model
        self.nE = model.n_gates
        self.nS = model.n_slow
        self.nv = 1 + self.nE + self.nS
        mask = np.zeros(self.N) if stim_mask is None else np.asarray(stim_mask, dtype=np.float64)
        self.stim_vec = float(stim_amp) * mask
        self.t_on = float(t_on)
        self.t_off = float(t_off)

    # -- state layout helpers -------------------------------------------------
    def split(self, y):
        N, nE = self.N, self.nE
        V = y[:N]
        zE = y[N:N * (1 + nE)].reshape(nE, N)
        zS = y[N * (1 + nE):].reshape(self.nS, N)
        return V, zE, zS

    def uniform_state(self):
        r = self.model.rest()
        return np.repeat(r, self.N)

    def I_stim(self, t):
        if self.t_on <= t <= self.t_off:
            return self.stim_vec
        return np.zeros(self.N)

    # -- the three right-hand sides --------------------------------------------
    def f_F(self, t, y):
        out = np.zeros_like(y)
        V = y[:self.N]
        out[:self.N] = (self.A @ V) / (self.chi * self.Cm * self.ML)
        return out

    def f_S(self, t, y):
        V, zE, zS = self.split(y)
        out = np.zeros_like(y)
        I_ion = self.Cm * self.model.i_ion(V, zE, zS)
        out[:self.N] = (self.I_stim(t) - I_ion) / self.Cm
        if self.nS:
            out[self.N * (1 + self.nE):] = self.model.g_S(V, zE, zS).reshape(-1)
        return out

    def lambda_yinf(self, y):
        V = y[:self.N]
        lam = np.zeros_like(y)
        yinf = np.zeros_like(y)
        LE, zinf = self.model.gates(V)
        sl = slice(self.N, self.N * (1 + self.nE))
        lam[sl] = LE.reshape(-1)
        yinf[sl] = zinf.reshape(-1)
        return lam, yinf

    def f_E(self, t, y):
        lam, yinf = self.lambda_yinf(y)
        return lam * (y - yinf)


def build_grid_problem(cfg, model_kw=None, stim_mask=None):
    """Monodomain problem on a structured Q1 grid described by a workload
    dictionary (see the workloads package)."""
    from workloads.configs import stim_mask as make_mask
    d = cfg["dim"]
    K, ML, _ = fem.assemble_q1_grid(list(cfg["n"]), list(cfg["h"][:d]), list(cfg["sigma"][:d]))
    model = make_model(cfg["model"], **(model_kw or {}))
    st = cfg["stim"]
    mask = make_mask(cfg) if stim_mask is None else stim_mask
    return Monodomain(K, ML, cfg["chi"], cfg["Cm"], model, mask, st["amp"], st["t_on"], st["t_off"])


def build_tet_problem(cfg, mesh, mask, model_kw=None):
    """Monodomain problem on a P1 tetrahedral mesh (unstructured workload)."""
    K, ML, _ = fem.assemble_p1_tets(mesh["coords"], mesh["tets"], mesh["fibres"], cfg["sigma"][0], cfg["sigma"][1])
    model = make_model(cfg["model"], **(model_kw or {}))
    st = cfg["stim"]
    return Monodomain(K, ML, cfg["chi"], cfg["Cm"], model, mask, st["amp"], st["t_on"], st["t_off"])
