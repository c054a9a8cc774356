"""Batched ensemble (uneven 2-D and 3-D instances in one context, one launch
per stage): each instance against the oracle, against its own
single-instance run (bitwise), graph against eager, and the per-instance
power iteration."""
import numpy as np
import pytest

from gpu_util import oracle_rho, rel_errors
from oracle.emrkc import emrkc_run, stage_counts
from oracle.monodomain import build_grid_problem
from workloads.ensemble import small_ensemble

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ens():
    cfgs = small_ensemble()
    probs = [build_grid_problem(c, stim_mask=c["mask"]) for c in cfgs]
    rhos = [oracle_rho(p, p.uniform_state()) for p in probs]
    return cfgs, probs, rhos


def run_batch(cfgs, rho, nsteps, precision="fp64", flags=0, chunks=None, shape=None):
    import torch
    from paper_2401_01745_amd import emrkc as E
    sim = E.simulation_from_batch(cfgs, precision=precision, rho=rho, flags=flags)
    if shape is not None:
        E.emrkc_set_variants(sim.ctx, shape if isinstance(shape, tuple) else (shape, 0, 0, 0, 0))
    E.emrkc_init_state(sim.ctx, sim.state)
    for n in (chunks or [nsteps]):
        E.emrkc_step(sim.ctx, sim.state, cfgs[0]["dt"], n)
    torch.cuda.synchronize()
    # the layout the calls stepped with: blocks when asked for (these
    # ensembles are small enough to keep the planes otherwise)
    assert E.emrkc_last_stats(sim.ctx).z_blocks == (1 if flags & E.EMRKC_Z_BLOCKS else 0)
    off, m, rF, rS = E.emrkc_batch_info(sim.ctx, cfgs[0]["dt"])
    out = sim.V.cpu().numpy().copy(), sim.z.cpu().numpy().astype(np.float64), off, m
    sim.close()
    return out


def test_batch_matches_oracle_per_instance(ens):
    cfgs, probs, rhos = ens
    rF = [r[0] for r in rhos]
    rS = [r[1] for r in rhos]
    rSmax = max(rS)
    nsteps = 80
    V, z, off, m = run_batch(cfgs, (rF, rS), nsteps)
    for k, (cfg, prob) in enumerate(zip(cfgs, probs)):
        s_k, m_k, _ = stage_counts(cfg["dt"], rF[k], rSmax)
        assert m[k] == m_k and s_k == 1
        y = emrkc_run(prob, prob.uniform_state(), 0.0, cfg["dt"], nsteps, rF[k], rSmax)
        Y = y.reshape(prob.nv, prob.N)
        sl = slice(off[k], off[k + 1])
        l2, mx = rel_errors(V[sl], Y[0])
        assert l2 <= 1e-10 and mx <= 1e-10, (k, l2, mx)
        for c in range(1, prob.nv):
            zl2, zmx = rel_errors(z[c - 1, sl], Y[c])
            assert zl2 <= 1e-10 and zmx <= 1e-10, (k, c, zl2, zmx)


def test_batch_equals_single_runs_bitwise_and_graph_equals_eager(ens):
    from paper_2401_01745_amd import emrkc as E
    cfgs, probs, rhos = ens
    rF = [r[0] for r in rhos]
    rS = [max(r[1] for r in rhos)] * len(rhos)
    V, z, off, m = run_batch(cfgs, (rF, rS), 41)
    V2, z2, _, _ = run_batch(cfgs, (rF, rS), 41, flags=E.EMRKC_EAGER)
    V3, z3, _, _ = run_batch(cfgs, (rF, rS), 41, chunks=[3, 32, 6])
    assert np.array_equal(V, V2) and np.array_equal(z, z2)
    assert np.array_equal(V, V3) and np.array_equal(z, z3)
    # every tile shape of the batched kernels, the flat batched head,
    # z-marching columns for the 3-D instances' inner stages (11 planes:
    # ragged columns of 4 and 3 planes, whole columns) and two tiles per
    # block for the inner stages give the same bits
    for shape in (1, 2, (0, 1, 0, 0, 0), (2, 1, 0, 0, 0), (1, 1, 1, 4, 0), (0, 0, 1, 64, 0), (2, 1, 1, 3, 0),
                  (1, 1, 2, 0, 0), (0, 0, 2, 0, 0), (2, 1, 2, 0, 0)):
        V4, z4, _, _ = run_batch(cfgs, (rF, rS), 41, shape=shape)
        assert np.array_equal(V, V4) and np.array_equal(z, z4), shape
    # z in blocks of 256 nodes while stepping (an ensemble this small keeps
    # the component planes by default): tiled and flat batched heads, eager
    # launches and a call split (a conversion each way per call)
    ZB = E.EMRKC_Z_BLOCKS
    for shape, fl, ch in [(None, ZB, None), ((1, 1, 0, 0, 0), ZB, None), ((2, 1, 2, 0, 0), ZB, None),
                          ((0, 0, 1, 4, 0), ZB | E.EMRKC_EAGER, None), (None, ZB, [3, 32, 6])]:
        V5, z5, _, _ = run_batch(cfgs, (rF, rS), 41, shape=shape, flags=fl, chunks=ch)
        assert np.array_equal(V, V5) and np.array_equal(z, z5), (shape, fl, ch)
    # single-instance contexts with the same masks
    import torch
    for k, cfg in enumerate(cfgs):
        sim = E.simulation_from_config(cfg, rho=(rF[k], rS[k]), stim_mask=cfg["mask"])
        E.emrkc_init_state(sim.ctx, sim.state)
        E.emrkc_step(sim.ctx, sim.state, cfg["dt"], 41)
        torch.cuda.synchronize()
        sl = slice(off[k], off[k + 1])
        assert np.array_equal(sim.V.cpu().numpy(), V[sl]), k
        assert np.array_equal(sim.z.cpu().numpy().astype(np.float64), z[:, sl]), k
        sim.close()


def test_batch_estimate_rho_per_instance(ens):
    import torch  # noqa: F401
    from paper_2401_01745_amd import emrkc as E
    cfgs, probs, rhos = ens
    sim = E.simulation_from_batch(cfgs)
    E.emrkc_init_state(sim.ctx, sim.state)
    gF, gS, itF, itS, _ = E.emrkc_estimate_rho(sim.ctx, sim.state)
    off, m, rF, rS = E.emrkc_batch_info(sim.ctx, cfgs[0]["dt"])
    for k, r in enumerate(rhos):
        assert rF[k] == pytest.approx(r[0], rel=1e-6) and rS[k] == pytest.approx(r[1], rel=1e-6)
    assert gF == pytest.approx(max(r[0] for r in rhos), rel=1e-6)
    assert gS == pytest.approx(max(r[1] for r in rhos), rel=1e-6)
    sim.close()


def test_batch_mixed_precision_against_oracle_per_instance(ens):
    """The mixed form of the ensemble, every instance against its own FP64
    oracle run: 1e-4 relative L2 in V (ten times that on the maximum, which
    sits at the front), and the float-stored ionic state within 1e-3 of each
    component's range."""
    from paper_2401_01745_amd import emrkc as E
    cfgs, probs, rhos = ens
    rF = [r[0] for r in rhos]
    rSmax = max(r[1] for r in rhos)
    rS = [rSmax] * len(rhos)
    nsteps = 80
    V, z, off, m = run_batch(cfgs, (rF, rS), nsteps, precision="mixed")
    # the same bits with float z in blocks of 256 nodes while stepping
    Vb, zb, _, _ = run_batch(cfgs, (rF, rS), nsteps, precision="mixed", flags=E.EMRKC_Z_BLOCKS)
    assert np.array_equal(V, Vb) and np.array_equal(z, zb)
    for k, (cfg, prob) in enumerate(zip(cfgs, probs)):
        y = emrkc_run(prob, prob.uniform_state(), 0.0, cfg["dt"], nsteps, rF[k], rSmax)
        Y = y.reshape(prob.nv, prob.N)
        sl = slice(off[k], off[k + 1])
        l2, mx = rel_errors(V[sl], Y[0])
        print("instance %d (%d nodes, m=%d): mixed V rel L2 %.3e, rel max %.3e" % (k, prob.N, m[k], l2, mx))
        assert l2 <= 1e-4 and mx <= 1e-3, (k, l2, mx)
        for c in range(1, prob.nv):
            dz = np.abs(z[c - 1, sl] - Y[c]).max()
            assert dz <= 1e-3 * np.abs(Y[c]).max() + 1e-6, (k, c, dz)


def test_batch_refuses_more_than_one_outer_stage(ens):
    """The instances advance with one common outer stage count, which the
    batched kernels support for s = 1 only: a dt whose radii need s >= 2 is
    refused, the state is left as it was, and the error names the reason."""
    import torch
    from paper_2401_01745_amd import emrkc as E
    cfgs, probs, rhos = ens
    rF = [r[0] for r in rhos]
    rS = [max(r[1] for r in rhos)] * len(rhos)
    dt = 0.5                                   # dt rho_S well above beta: s >= 2
    assert E.emrkc_stage_counts(dt, rF[0], rS[0])[0] >= 2
    sim = E.simulation_from_batch(cfgs, rho=(rF, rS))
    E.emrkc_init_state(sim.ctx, sim.state)
    V0, z0 = sim.V.clone(), sim.z.clone()
    with pytest.raises(E.EmrkcError) as ei:
        E.emrkc_step(sim.ctx, sim.state, dt, 3)
    assert ei.value.code == E.EMRKC_EUNSUPPORTED
    assert "s = 1" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.equal(sim.V, V0) and torch.equal(sim.z, z0)
    assert sim.state.step == 0
    # the supported dt still runs on the same context
    E.emrkc_step(sim.ctx, sim.state, cfgs[0]["dt"], 2)
    assert sim.state.step == 2
    sim.close()


def test_batch_autotune(ens):
    """The batch autotuner picks one of the three tile shapes and the tiled
    or flat head, keeps the state, and the run with its choice equals the
    default bit for bit."""
    import torch
    from paper_2401_01745_amd import emrkc as E
    cfgs, probs, rhos = ens
    rF = [r[0] for r in rhos]
    rS = [max(r[1] for r in rhos)] * len(rhos)
    V, z, _, _ = run_batch(cfgs, (rF, rS), 20)
    sim = E.simulation_from_batch(cfgs, rho=(rF, rS))
    E.emrkc_init_state(sim.ctx, sim.state)
    V0, z0 = sim.V.clone(), sim.z.clone()
    v = E.emrkc_autotune(sim.ctx, sim.state, cfgs[0]["dt"], reps=2)
    assert v[0] in (0, 1, 2) and v[1] in (0, 1) and v[4] == 0
    assert (v[2], v[3]) in ((0, 0), (2, 0), (1, 4), (1, 8), (1, 64))
    assert torch.equal(sim.V, V0) and torch.equal(sim.z, z0)
    E.emrkc_step(sim.ctx, sim.state, cfgs[0]["dt"], 20)
    torch.cuda.synchronize()
    assert np.array_equal(sim.V.cpu().numpy(), V)
    for bad in [(3, 0, 0, 0, 0), (0, 2, 0, 0, 0), (0, 0, 1, 0, 0), (0, 0, 0, 4, 0), (0, 0, 1, 65, 0),
                (0, 0, 2, 4, 0), (0, 0, 3, 0, 0)]:
        with pytest.raises(E.EmrkcError):
            E.emrkc_set_variants(sim.ctx, bad)
    sim.close()


def test_full_ensemble_in_the_bench_configuration():
    """The 64-instance ensemble at full size (7.0 M nodes) in the shapes the
    benchmark times (flat batched head, 32x4x2 / 32x8 tiles for the inner
    stage), radii from the library's own power iteration: every instance
    equals its own single-context run bit for bit (a property at any size),
    and the three smallest instances, sampled, equal their oracle runs to
    1e-10."""
    import torch
    from paper_2401_01745_amd import emrkc as E
    from workloads.ensemble import ensemble
    cfgs = ensemble()
    dt, nsteps = cfgs[0]["dt"], 20
    print("full ensemble:", len(cfgs), "instances", flush=True)
    sim = E.simulation_from_batch(cfgs)
    E.emrkc_set_variants(sim.ctx, (1, 1, 0, 0, 0))
    E.emrkc_init_state(sim.ctx, sim.state)
    E.emrkc_estimate_rho(sim.ctx, sim.state)
    off, m, rF, rS = E.emrkc_batch_info(sim.ctx, dt)
    rSmax = max(rS)
    E.emrkc_step(sim.ctx, sim.state, dt, nsteps)
    torch.cuda.synchronize()
    assert E.emrkc_last_stats(sim.ctx).z_blocks == 1  # 1.0 GB of z: stepped in blocks
    V = sim.V.cpu().numpy().copy()
    assert off[-1] == V.size and V.size > 6_900_000
    # the 3-D instances' inner stages in z-marching columns, and two tiles
    # per block for the inner stages: the same bits
    for v in [(1, 1, 1, 64, 0), (1, 1, 2, 0, 0)]:
        sim2 = E.simulation_from_batch(cfgs, rho=(rF, rS))
        E.emrkc_set_variants(sim2.ctx, v)
        E.emrkc_init_state(sim2.ctx, sim2.state)
        E.emrkc_step(sim2.ctx, sim2.state, dt, nsteps)
        torch.cuda.synchronize()
        assert torch.equal(sim2.V, sim.V) and torch.equal(sim2.z, sim.z), v
        sim2.close()
    sizes = [off[k + 1] - off[k] for k in range(len(cfgs))]
    sample = sorted(range(len(cfgs)), key=lambda k: sizes[k])[:3]
    for k, cfg in enumerate(cfgs):
        sl = slice(off[k], off[k + 1])
        zk = sim.z[:, sl].cpu().numpy().astype(np.float64)
        one = E.simulation_from_config(cfg, rho=(rF[k], rSmax), stim_mask=cfg["mask"])
        E.emrkc_init_state(one.ctx, one.state)
        E.emrkc_step(one.ctx, one.state, dt, nsteps)
        torch.cuda.synchronize()
        assert np.array_equal(one.V.cpu().numpy(), V[sl]), k
        assert np.array_equal(one.z.cpu().numpy().astype(np.float64), zk), k
        one.close()
        if k in sample:
            prob = build_grid_problem(cfg, stim_mask=cfg["mask"])
            y = emrkc_run(prob, prob.uniform_state(), 0.0, dt, nsteps, rF[k], rSmax)
            Y = y.reshape(prob.nv, prob.N)
            l2, mx = rel_errors(V[sl], Y[0])
            assert l2 <= 1e-10 and mx <= 1e-10, (k, l2, mx)
            assert np.abs(zk - Y[1:]).max() <= 1e-10 * np.abs(Y[1:]).max(), k
    sim.close()
