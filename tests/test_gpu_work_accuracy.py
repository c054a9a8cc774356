"""Work against accuracy (the comparison of the numerical experiments, on
the GPU): the 3-D cuboid workload (201 x 71 x 31 Q1 nodes, CRN surrogate)
run to T = 10 ms with emRKC (FP64 and mixed), mRKC and IMEX-RL for several
dt, errors of V at T against EXEX-RL at dt = 2e-4 ms, and the wall time of
each run (context creation excluded; resting state, spectral radii and
steps included).  Prints the table (run with -s)."""
import time

import numpy as np
import pytest

from gpu_util import rel_errors
from workloads.configs import get_config

pytestmark = pytest.mark.gpu

T = 10.0
DTS = [0.1, 0.05, 0.025, 0.0125, 0.00625, 0.003125]
METHODS = [("emRKC", "emrkc", "fp64"), ("emRKC mixed", "emrkc", "mixed"), ("mRKC", "mrkc", "fp64"),
           ("IMEX-RL", "imexrl", "fp64")]


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


def _run(E, sim, method, dt, n):
    import torch
    E.emrkc_init_state(sim.ctx, sim.state)
    info = None
    if method == "imexrl":
        E.emrkc_imexrl_step(sim.ctx, sim.state, dt, n)
        info = E.emrkc_imexrl_iterations(sim.ctx) / max(n, 1)
    elif method == "exexrl":
        E.emrkc_exexrl_step(sim.ctx, sim.state, dt, n)
    else:
        E.emrkc_estimate_rho(sim.ctx, sim.state)
        E.emrkc_step(sim.ctx, sim.state, dt, n)
        info = E.emrkc_stages(sim.ctx, dt)[:2]
    torch.cuda.synchronize()
    return info


def test_work_against_accuracy(E):
    import torch
    cfg = get_config("c2_3d_crn")
    ref = E.simulation_from_config(cfg)
    _run(E, ref, "exexrl", 2e-4, int(round(T / 2e-4)))
    Vref = ref.V.cpu().numpy().copy()
    ref.close()
    assert Vref.max() > -40.0  # excited tissue inside the slab at T
    rows = []
    for label, method, prec in METHODS:
        sim = E.simulation_from_config(cfg, precision=prec, method="mrkc" if method == "mrkc" else "emrkc")
        _run(E, sim, method, DTS[0], 4)  # first launches, graph capture
        for dt in DTS:
            n = int(round(T / dt))
            t0 = time.perf_counter()
            info = _run(E, sim, method, dt, n)
            el = time.perf_counter() - t0
            V = sim.V.cpu().numpy()
            err = rel_errors(V, Vref)[0] if np.all(np.isfinite(V)) else float("inf")
            rows.append((label, dt, err, el, info))
        sim.close()
    print("\n  method        dt [ms]   rel L2 err of V   wall [ms]   stages (s, m) / CG its per step")
    for label, dt, err, el, info in rows:
        print("  %-12s  %6.4f   %14.3e   %9.2f   %s" % (label, dt, err, 1e3 * el, info))
    by = {}
    for label, dt, err, el, info in rows:
        by.setdefault(label, []).append((dt, err, el, info))
    for label in ("emRKC", "emRKC mixed", "IMEX-RL"):
        errs = [x[1] for x in by[label]]
        assert all(np.isfinite(errs)), (label, errs)
        # first order once dt is small enough (the error curves of emRKC and
        # IMEX-RL have a pre-asymptotic bump near dt = 0.025 ms, where the
        # errors of the wave front's timing partly cancel)
        assert errs[-3] > errs[-2] > errs[-1], (label, errs)
        assert 1.4 < errs[-2] / errs[-1] < 2.6, (label, errs)
    # emRKC is cheaper than IMEX-RL at every step size, and more accurate at
    # the small ones (IMEX-RL's explicit ionic current against its implicit
    # diffusion line carries a larger splitting error)
    for (dt, e1, t1, _), (_, e2, t2, _) in zip(by["emRKC"], by["IMEX-RL"]):
        assert t1 < t2, (dt, t1, t2)
        if dt <= 0.0125:
            assert e1 < e2, (dt, e1, e2)
    # the mixed form's error is the FP64 form's
    for (dt, e1, _, _), (_, e2, _, _) in zip(by["emRKC"], by["emRKC mixed"]):
        assert abs(e1 - e2) < 1e-3 + 0.05 * e1, (dt, e1, e2)
