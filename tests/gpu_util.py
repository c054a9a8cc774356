"""Helpers shared by the GPU tests: run the oracle and the library on the
same workload and compare."""
import numpy as np

from oracle.emrkc import emrkc_run
from oracle.monodomain import build_grid_problem
from oracle.powiter import compute_rho, random_unit_interval


def oracle_rho(prob, y, t=0.0, safety=1.05, seed=0):
    v0 = random_unit_interval(y.size, seed)
    _, rF, itF, _ = compute_rho(t, y, prob.f_F, v0.copy())
    _, rS, itS, _ = compute_rho(t, y, prob.f_S, v0.copy())
    return safety * rF, safety * rS, itF, itS


def gpu_run(cfg, nsteps, rho, precision="fp64", flags=0, chunks=None, model_kw=None, variants=None):
    import torch
    from paper_2401_01745_amd import emrkc as E
    sim = E.simulation_from_config(cfg, precision=precision, rho=rho, flags=flags, **(model_kw or {}))
    if variants is not None:
        E.emrkc_set_variants(sim.ctx, variants)
    E.emrkc_init_state(sim.ctx, sim.state)
    for n in (chunks or [nsteps]):
        E.emrkc_step(sim.ctx, sim.state, cfg["dt"], n)
    torch.cuda.synchronize()
    out = sim.V.cpu().numpy().copy(), sim.z.cpu().numpy().astype(np.float64), E.emrkc_last_stats(sim.ctx)
    sim.close()
    return out


def oracle_run(cfg, nsteps, rho, model_kw=None, y0=None, track=None):
    """Oracle run; ``track`` (a list) receives max V after every step."""
    prob = build_grid_problem(cfg, model_kw=model_kw)
    y = prob.uniform_state() if y0 is None else y0
    cb = None if track is None else (lambda n, yy: track.append(float(yy[:prob.N].max())))
    y = emrkc_run(prob, y, 0.0, cfg["dt"], nsteps, rho[0], rho[1], callback=cb)
    return prob, y


def rel_errors(a, b):
    """(relative L2, relative max) of a against the reference b."""
    d = a - b
    return float(np.linalg.norm(d) / np.linalg.norm(b)), float(np.abs(d).max() / np.abs(b).max())
