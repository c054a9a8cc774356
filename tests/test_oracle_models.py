"""Pins for the oracle's ionic models: sizes and stiffness against the
paper's table, the classical HH resting gate values, gate ranges and
removable singularities."""
import json
import os

import numpy as np
import pytest

from oracle.ionic import HH, CRNSurrogate, TTPSurrogate, hh_core_rates

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


@pytest.mark.parametrize("model,key", [(HH(), "HH"), (CRNSurrogate(), "CRN"), (TTPSurrogate(), "TTP")])
def test_sizes_match_table(model, key):
    assert model.n_gates + model.n_slow == GOLDEN["ionic_model_sizes"]["value"][key]
    assert model.rest().size == 1 + GOLDEN["ionic_model_sizes"]["value"][key]


def test_hh_resting_gates_textbook_values():
    """m, h, n steady states at -65 mV of the classical HH model."""
    r = HH().rest()
    assert r[0] == -65.0
    assert r[1] == pytest.approx(0.0529, abs=2e-4)
    assert r[2] == pytest.approx(0.5961, abs=2e-4)
    assert r[3] == pytest.approx(0.3177, abs=2e-4)


def test_hh_removable_singularities():
    """alpha_m(-40) = 1/ms and alpha_n(-55) = 0.1/ms, continuous around."""
    for V0, idx, val in [(-40.0, 0, 1.0), (-55.0, 2, 0.1)]:
        Vs = V0 + np.array([-1e-5, -1e-8, 0.0, 1e-8, 1e-5])
        a = hh_core_rates(Vs, 1.0)[idx][0]
        assert a[2] == pytest.approx(val, rel=1e-15)
        assert np.all(np.abs(a - val) < 1e-5 * val)


def single_cell(model, T=60.0, dt=0.01, amp=20.0):
    """Rush-Larsen single-cell run with a 2 ms stimulus; returns the final
    state, the peak V and the largest of |Lambda_E| and |d i_ion/dV| seen."""
    y = model.rest().astype(float)
    ng = model.n_gates
    vmax = -1e9
    stiff = 0.0
    for it in range(int(T / dt)):
        V = y[:1]
        zE = y[1:1 + ng, None]
        zS = y[1 + ng:, None]
        lam, zinf = model.gates(V)
        dI = (model.i_ion(V + 1e-4, zE, zS) - model.i_ion(V - 1e-4, zE, zS)) / 2e-4
        stiff = max(stiff, np.abs(lam).max(), abs(dI[0]))
        zE1 = zE + np.expm1(dt * lam) * (zE - zinf)
        gS = model.g_S(V, zE1, zS)
        Is = amp if it * dt <= 2.0 else 0.0
        V1 = V + dt * (Is - model.i_ion(V, zE1, zS + dt * gS))
        y = np.concatenate([V1, zE1[:, 0], (zS + dt * gS)[:, 0]])
        vmax = max(vmax, y[0])
    return y, vmax, stiff


@pytest.mark.parametrize("model,key", [(HH(), "HH"), (CRNSurrogate(), "CRN"), (TTPSurrogate(), "TTP")])
def test_single_cell_action_potential_and_stiffness(model, key):
    """A 2 ms stimulus fires an action potential, the state returns towards
    rest with bounded slow variables, gates stay in [0, 1], and the largest
    rate met along the way (gate rates and the V self-coupling) is within a
    factor 2 of the table's rho_max."""
    y, vmax, stiff = single_cell(model)
    assert vmax > 20.0
    assert -80.0 < y[0] < -55.0
    assert np.all(np.isfinite(y))
    g = y[1:1 + model.n_gates]
    assert np.all((g >= 0) & (g <= 1))
    ratio = stiff / GOLDEN["ionic_model_rho_max"]["value"][key]
    assert 0.5 < ratio < 2.0, ratio
