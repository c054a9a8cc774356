"""Practical stability limit (section "Practical stability limit"): the
monodomain equation on a 20 mm cable with dx = 0.025 mm and the TTP-shaped
surrogate, T = 100 ms, stimulus 50 uA/mm^3 on x <= 1.5 mm for t <= 2 ms,
solved with emRKC for growing dt (radii estimated once at rest), against a
reference from EXEX-RL at dt = 1e-3 ms.  The cable is a 2-D grid of 801 x 2
nodes with no transverse conduction (the solution is uniform across it).
Prints the table of relative norms and stage counts (run with -s)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DTS = [0.01, 0.05, 0.1, 0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 5.0, 6.0]


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


def cable_config():
    return dict(name="cable_1d", kind="grid", dim=2, n=(801, 2), h=(0.025, 0.025), sigma=(0.17, 0.0, 0.0),
                chi=140.0, Cm=0.01, model="TTP_SURR",
                stim=dict(kind="box", width=1.5, amp=50.0 / 140.0, t_on=0.0, t_off=2.0), dt=0.05, T=100.0,
                precision="fp64")


def _final_V(E, cfg, dt, method):
    import torch
    sim = E.simulation_from_config(cfg)
    E.emrkc_init_state(sim.ctx, sim.state)
    n = int(round(cfg["T"] / dt))
    stages = None
    if method == "emrkc":
        E.emrkc_estimate_rho(sim.ctx, sim.state, allow_noconv=True)
        stages = E.emrkc_stages(sim.ctx, dt)[:2]
        E.emrkc_step(sim.ctx, sim.state, dt, n)
    else:
        E.emrkc_exexrl_step(sim.ctx, sim.state, dt, n)
    torch.cuda.synchronize()
    V = sim.V.cpu().numpy().copy()
    sim.close()
    return V, stages


def test_practical_stability_limit(E):
    cfg = cable_config()
    Vref, _ = _final_V(E, cfg, 1e-3, "exexrl")
    assert np.all(np.isfinite(Vref))
    nref = np.linalg.norm(Vref)
    rows = []
    for dt in DTS:
        V, (s, m) = _final_V(E, cfg, dt, "emrkc")
        rel = np.linalg.norm(V) / nref if np.all(np.isfinite(V)) else float("inf")
        rows.append((dt, rel, s, m))
    print("\n  dt [ms]   ||V_N||/||V*||   s   m")
    for dt, rel, s, m in rows:
        print("  %7.3f   %14.4g   %2d  %2d" % (dt, rel, s, m))
    # bounded through the step sizes used in practice and well beyond
    for dt, rel, s, m in rows:
        if dt <= 1.0:
            assert 0.5 < rel < 2.0, (dt, rel)
    # the diffusion needs inner stages from the smallest steps on; outer
    # stages appear only for large steps (f_S is mildly stiff)
    assert rows[0][3] > 1 and rows[0][2] == 1
    assert max(r[2] for r in rows) > 1
    # the explicit scheme's limit is near 2/rho_F = 2.6e-3 ms
    Vx, _ = _final_V(E, cfg, 4e-3, "exexrl")
    assert not np.all(np.isfinite(Vx)) or np.linalg.norm(Vx) > 1e3 * nref
