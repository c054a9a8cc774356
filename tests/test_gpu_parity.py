"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded synthetic inputs.  FP64 results must agree to 1e-10
relative in V (spec bound), component kernels to a few ulps."""
import numpy as np
import pytest

from gpu_util import gpu_run, oracle_rho, oracle_run, rel_errors
from oracle.monodomain import build_grid_problem
from workloads.configs import get_config, small_config

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name,model", [("c1_2d_hh", "HH"), ("c2_3d_crn", "CRN_SURR"), ("c2_3d_crn", "TTP_SURR")])
def test_init_state_matches_model_rest(E, name, model):
    import torch
    cfg = small_config(name, (9, 7) if name.startswith("c1") else (9, 7, 5), model=model)
    sim = E.simulation_from_config(cfg, rho=(1.0, 1.0))
    E.emrkc_init_state(sim.ctx, sim.state)
    torch.cuda.synchronize()
    prob = build_grid_problem(cfg)
    y = prob.uniform_state().reshape(prob.nv, prob.N)
    assert np.array_equal(sim.V.cpu().numpy(), y[0])
    assert np.abs(sim.z.cpu().numpy() - y[1:]).max() <= 2e-16 * np.abs(y[1:]).max()
    sim.close()


@pytest.mark.parametrize("n", [(37, 29, 11), (13, 300), (201, 7, 3)])
def test_diffusion_operator(E, n):
    """(chi Cm M_L)^{-1} A V from the stencil kernel against the oracle's
    assembled sparse matrix, random V with a resting offset."""
    import torch
    cfg = small_config("c2_3d_crn" if len(n) == 3 else "c1_2d_hh", n)
    if len(n) == 2:
        cfg["h"] = (0.02, 0.03)
        cfg["sigma"] = (0.17, 0.05, 0.05)
    prob = build_grid_problem(cfg)
    rng = np.random.default_rng(sum(n))
    V = -65.0 + 20.0 * rng.standard_normal(prob.N)
    ref = prob.f_F(0.0, np.concatenate([V, np.zeros(prob.N * (prob.nv - 1))]))[:prob.N]
    sim = E.simulation_from_config(cfg, rho=(1.0, 1.0))
    out = torch.empty(prob.N, dtype=torch.float64, device="cuda")
    E.emrkc_apply_diffusion(sim.ctx, to_dev(V), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    scale = np.abs(prob.A).sum(axis=1).A1 / (prob.chi * prob.Cm * prob.ML) * np.abs(V).max()
    assert np.all(np.abs(got - ref) <= 1e-14 * scale.max()), np.abs(got - ref).max() / scale.max()
    # constant states are in the kernel of the operator: exactly zero
    E.emrkc_apply_diffusion(sim.ctx, to_dev(np.full(prob.N, -65.0)), out)
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 0.0)
    sim.close()


@pytest.mark.parametrize("model", ["HH", "CRN_SURR", "TTP_SURR", "LINEAR"])
def test_slow_rhs(E, model):
    """f_S(t, y) at perturbed states from the ionic kernel's model code."""
    import torch
    kw = dict(a=0.7, lam_E=-3.0) if model == "LINEAR" else {}
    cfg = small_config("c2_3d_crn", (11, 9, 7), model=model)
    prob = build_grid_problem(cfg, model_kw=kw)
    rng = np.random.default_rng(4)
    y = prob.uniform_state().reshape(prob.nv, prob.N)
    y[0] += rng.uniform(-20, 90, prob.N)
    y[1:1 + prob.nE] = np.clip(y[1:1 + prob.nE] + rng.uniform(-0.2, 0.2, (prob.nE, prob.N)), 0, 1)
    if prob.nS:
        y[1 + prob.nE:] *= rng.uniform(0.9, 1.1, (prob.nS, prob.N))
    yf = y.reshape(-1)
    for t in (0.5, 3.0):
        ref = prob.f_S(t, yf).reshape(prob.nv, prob.N)
        sim = E.simulation_from_config(cfg, rho=(1.0, 1.0), **kw)
        sim.V.copy_(to_dev(y[0]))
        sim.z.copy_(to_dev(y[1:]))
        out = torch.empty(prob.nv * prob.N, dtype=torch.float64, device="cuda")
        E.emrkc_eval_rhs_slow(sim.ctx, sim.state, t, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(prob.nv, prob.N)
        for c in range(prob.nv):
            scale = max(np.abs(ref[c]).max(), 1e-300)
            assert np.abs(got[c] - ref[c]).max() <= 1e-12 * scale, (c, np.abs(got[c] - ref[c]).max() / scale)
        sim.close()


def _compare_full(cfg, nsteps, rho, tol=FP64_TOL, model_kw=None, track=None, **kw):
    prob, y = oracle_run(cfg, nsteps, rho, model_kw=model_kw, track=track)
    assert np.all(np.isfinite(y)), "oracle run not finite: pick a stable case"
    V, z, stats = gpu_run(cfg, nsteps, rho, model_kw=model_kw, **kw)
    Y = y.reshape(prob.nv, prob.N)
    l2, mx = rel_errors(V, Y[0])
    assert l2 <= tol and mx <= tol, (l2, mx)
    for c in range(1, prob.nv):
        zl2, zmx = rel_errors(z[c - 1], Y[c])
        assert zl2 <= tol and zmx <= tol, (c, zl2, zmx)
    return prob, Y, V, stats


@pytest.mark.parametrize("variants", [None, (0, 0, 2, 0, 0), (0, 0, 3, 0, 0), (0, 0, 4, 0, 0)])
def test_c1_full_run_fp64(E, variants):
    """Unit-square HH workload (65 x 65, 100 steps of 0.05 ms) with the
    oracle's own spectral radii: s = 1, m = 7; separate inner-stage launches
    and all six inner stages in one launch (16 x 16 tiles with reflected
    halos of up to 6 nodes)."""
    cfg = get_config("c1_2d_hh")
    prob = build_grid_problem(cfg)
    rF, rS, _, _ = oracle_rho(prob, prob.uniform_state())
    _, _, _, stats = _compare_full(cfg, 100, (rF, rS), variants=variants)
    assert (stats.s, stats.m) == (1, 7)
    assert stats.kernels_per_step == (7 if variants is None else 1 if variants[2] == 4 else 2)


@pytest.mark.parametrize("rho,sm", [((900.0, 100.0), (2, 3)), ((1600.0, 300.0), (3, 3)), ((2900.0, 4.4), (1, 9)),
                                    ((5000.0, 4.4), (1, 12))])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_inner_stages_in_one_launch(E, rho, sm, precision):
    """2-D grids: all inner stages of a stage in one launch equal the
    separate launches bit for bit for s >= 2 (its buffer rule, with the
    final copy for s = 3), up to the largest stage count it takes (m = 9),
    and beyond it (m = 12: separate launches), in both precisions; FP64 also
    against the oracle."""
    cfg = small_config("c2_3d_crn", (37, 29))
    cfg["dim"] = 2
    V1, z1, st1 = gpu_run(cfg, 30, rho, precision=precision)
    shape = 4 if sm[0] == 1 else 2 + (sm[0] % 2)
    V2, z2, st2 = gpu_run(cfg, 30, rho, precision=precision, variants=(0, 0, shape, 0, 0), chunks=[3, 27])
    assert (st1.s, st1.m) == sm and (st2.s, st2.m) == sm
    s, m = sm
    assert st2.kernels_per_step == ((1 if shape == 4 else 2 * s + (1 if s > 1 and s % 2 else 0)) if m <= 9
                                    else s * m)
    assert np.array_equal(V1, V2) and np.array_equal(z1, z2)
    if precision == "fp64":
        _, y = oracle_run(cfg, 30, rho)
        l2, mx = rel_errors(V2, y[:V2.size])
        assert l2 < FP64_TOL and mx < FP64_TOL, (l2, mx)


@pytest.mark.parametrize("model,n", [("CRN_SURR", (37, 29, 11)), ("TTP_SURR", (41, 19, 9))])
def test_3d_wave_fp64(E, model, n):
    """3-D slab with a propagating wave (200 steps = 10 ms): excitation,
    propagation through the slab and recovery."""
    cfg = small_config("c2_3d_crn", n, model=model)
    prob = build_grid_problem(cfg)
    rF, rS, _, _ = oracle_rho(prob, prob.uniform_state())
    vmax = []
    _, Y, V, stats = _compare_full(cfg, 200, (rF, rS), track=vmax)
    assert (stats.s, stats.m) == (1, 2)
    assert max(vmax) > 20.0  # an action potential fired


def test_2d_wave_fp64(E):
    cfg = small_config("c2_3d_crn", (61, 45), model="TTP_SURR")
    cfg["dim"] = 2
    cfg["h"] = (0.1, 0.1)
    _compare_full(cfg, 120, (51.0, 9.0))


@pytest.mark.parametrize("rho,dt,sm", [((51.0, 100.0), 0.05, (2, 1)), ((2000.0, 300.0), 0.05, (3, 3)),
                                       ((51.0, 4.4), 0.025, (1, 1)), ((51.0, 700.0), 0.05, (5, 1)),
                                       ((5000.0, 100.0), 0.05, (2, 6)), ((150.0, 30.0), 0.1, (2, 2))])
def test_stage_plans(E, rho, dt, sm):
    """Outer stages s >= 2 and single inner stages m = 1 (buffer rotation
    and the final copy) against the oracle.  Radii are over-estimates of the
    true ones (rho_F = 48.6, rho_S = 4.2), which keeps every case stable.
    Plans with m >= 2 also run the split stage (pointwise head, two-stage
    inner kernel; its own buffer rule for s >= 2): the same bits."""
    cfg = small_config("c2_3d_crn", (23, 17, 7), dt=dt)
    _, _, V, stats = _compare_full(cfg, 60, rho)
    assert (stats.s, stats.m) == sm
    if sm[1] >= 2:
        for v in [(7, 3, 1, 4, 0), (8, 0, 1, 4, 0)]:
            for fl in (E.EMRKC_Z_BLOCKS, E.EMRKC_Z_PLANES):  # z in blocks (z_1 too, for s >= 2) and in planes
                V7, _, st7 = gpu_run(cfg, 60, rho, variants=v, flags=fl)
                assert (st7.s, st7.m) == sm
                assert st7.z_blocks == (1 if fl == E.EMRKC_Z_BLOCKS else 0)
                assert np.array_equal(V7, V), (v, fl)


@pytest.mark.parametrize("rho,dt,sm", [((51.0, 100.0), 0.05, (2, 1)), ((2000.0, 300.0), 0.05, (3, 3)),
                                       ((51.0, 700.0), 0.05, (5, 1)), ((150.0, 30.0), 0.1, (2, 2))])
def test_stage_plans_mixed(E, rho, dt, sm):
    """The mixed precision through s >= 2 outer stages against the FP64
    oracle: its first-stage gate update is a float FMA and its later stages
    recur in double; both stay within the mixed-precision bound (FP32
    ionic state: a few 1e-6 relative over 60 steps)."""
    cfg = small_config("c2_3d_crn", (23, 17, 7), dt=dt)
    _, _, V, stats = _compare_full(cfg, 60, rho, tol=2e-5, precision="mixed")
    assert (stats.s, stats.m) == sm
    # float z (and z_1 for s >= 2, read back as z_{j-2}) in blocks and in
    # planes, with the flat head and with the split stage: the same bits
    for v in [None, (7, 3, 1, 4, 0), (8, 0, 1, 4, 0)] if sm[1] >= 2 else [None]:
        runs = [gpu_run(cfg, 60, rho, precision="mixed", variants=v, flags=fl)
                for fl in (E.EMRKC_Z_BLOCKS, E.EMRKC_Z_PLANES)]
        assert runs[0][2].z_blocks == 1 and runs[1][2].z_blocks == 0
        for Vr, zr, _ in runs:
            assert np.array_equal(Vr, V), v
        assert np.array_equal(runs[0][1], runs[1][1]), v


def test_linear_model_closed_form_on_gpu(E):
    """LINEAR model from a cosine mode: V_{n} = P_s(dt Phi_m(eta lF)(lF + lS))^n V0
    (the scalar stability analysis applied per eigenmode)."""
    import torch
    from test_oracle_emrkc import P_cheb, Phi, cosine_mode, phi
    from oracle.emrkc import stage_counts
    n, h, sig = (33, 17, 9), (0.1, 0.1, 0.1), (0.17, 0.019, 0.019)
    cfg = small_config("c2_3d_crn", n, model="LINEAR")
    cfg["stim"]["amp"] = 0.0
    a, lamE = 2.0, -40.0
    ks = (5, 3, 2)
    th = [np.pi * k / (nn - 1) for k, nn in zip(ks, n)]
    lam = [(2 - 2 * np.cos(t)) / hh ** 2 for t, hh in zip(th, h)]
    mu = [(2 + np.cos(t)) / 3 for t in th]
    eig = sig[0] * lam[0] * mu[1] * mu[2] + sig[1] * mu[0] * lam[1] * mu[2] + sig[2] * mu[0] * mu[1] * lam[2]
    lF = -eig / (cfg["chi"] * cfg["Cm"])
    rho = (51.0, 2.1)
    s, m, eta = stage_counts(cfg["dt"], *rho)
    amp = P_cheb(s, cfg["dt"] * Phi(m, eta * lF) * (lF - a))
    ampz = P_cheb(s, cfg["dt"] * phi(eta * lamE) * lamE)
    V0 = cosine_mode(n, ks)
    sim = E.simulation_from_config(cfg, rho=rho, a=a, lam_E=lamE)
    sim.V.copy_(to_dev(V0))
    sim.z.fill_(0.5)
    E.emrkc_step(sim.ctx, sim.state, cfg["dt"], 25)
    torch.cuda.synchronize()
    assert np.abs(sim.V.cpu().numpy() - amp ** 25 * V0).max() < 1e-13
    assert np.abs(sim.z.cpu().numpy() - 0.5 * ampz ** 25).max() < 1e-14
    sim.close()


@pytest.mark.parametrize("n,rho,precision", [((29, 23, 9), (51.0, 4.4), "fp64"), ((29, 23, 9), (51.0, 4.4), "mixed"),
                                              ((37, 11), (900.0, 4.4), "fp64"), ((19, 13, 7), (150.0, 4.4), "fp64")])
def test_graph_eager_fused_split_and_repeat_are_bitwise_identical(E, n, rho, precision):
    """HIP-graph replay, eager launches, the fused tail+head kernel, the
    LDS-tiled, z-marching (ragged 4-plane columns) and flat kernels,
    arbitrary call splits and repeated runs all give the same bits (m = 2,
    2-D with m = 5, and m = 3)."""
    cfg = small_config("c2_3d_crn", n)
    if len(n) == 2:
        cfg["dim"] = 2
    V1, z1, st1 = gpu_run(cfg, 80, rho, precision=precision)
    V2, z2, st2 = gpu_run(cfg, 80, rho, precision=precision, flags=E.EMRKC_EAGER)
    V3, z3, _ = gpu_run(cfg, 80, rho, precision=precision, chunks=[1, 33, 7, 39])
    V4, z4, _ = gpu_run(cfg, 80, rho, precision=precision)
    V5, z5, st5 = gpu_run(cfg, 80, rho, precision=precision, flags=E.EMRKC_FUSE)
    V6, z6, _ = gpu_run(cfg, 80, rho, precision=precision, flags=E.EMRKC_FLAT)
    V7, z7, _ = gpu_run(cfg, 80, rho, precision=precision, flags=E.EMRKC_FLAT | E.EMRKC_EAGER)
    # the flat switch covers every grid kernel: with it the fused request
    # falls back to separate flat head and inner launches
    V8, z8, st8 = gpu_run(cfg, 80, rho, precision=precision, flags=E.EMRKC_FLAT | E.EMRKC_FUSE)
    runs = [(V2, z2), (V3, z3), (V4, z4), (V5, z5), (V6, z6), (V7, z7), (V8, z8)]
    # z in blocks of 256 nodes while stepping (the runs above keep these
    # small z arrays in component planes), with the default, fused and flat
    # kernels, eager launches and an odd call split (a conversion each way
    # per call)
    ZB = E.EMRKC_Z_BLOCKS
    assert st1.z_blocks == 0
    for fl in (ZB, ZB | E.EMRKC_FUSE, ZB | E.EMRKC_FLAT, ZB | E.EMRKC_EAGER):
        Vb, zb, stb = gpu_run(cfg, 80, rho, precision=precision, flags=fl)
        assert stb.z_blocks == 1, fl
        runs.append((Vb, zb))
    runs.append(gpu_run(cfg, 80, rho, precision=precision, flags=ZB, chunks=[1, 33, 7, 39])[:2])
    if len(n) == 3:
        # z-marching head (register and LDS-staged) and inner kernels with
        # ragged columns and plane counts that do not divide n[2]
        for v in [(1, 4, 1, 4, 0), (2, 4, 1, 4, 0), (2, 2, 1, 3, 0), (1, n[2], 1, n[2], 0), (2, 5, 0, 0, 0),
                  (0, 0, 1, 2, 0), (2, 3, 1, 4, 1), (3, 0, 1, 4, 0), (4, 0, 0, 0, 1), (5, 0, 1, 4, 0),
                  (5, 0, 0, 0, 1), (5, 0, 1, 3, 0), (0, 0, 0, 0, 0),
                  # the split stage: pointwise head with the two-stage inner
                  # kernel in ragged columns of 4, 2, 3 and all planes (7),
                  # or with u_1 as a launch of the inner kernel (8)
                  (7, 4, 1, 4, 0), (7, 2, 0, 0, 0), (7, 3, 1, 2, 0), (7, n[2], 1, 3, 0),
                  (8, 0, 1, 4, 0), (8, 0, 0, 0, 0), (8, 0, 1, 2, 0)]:
            runs.append(gpu_run(cfg, 80, rho, precision=precision, variants=v)[:2])
            if v[0] not in (1, 2):  # every head but the z-marching ones also with z in blocks
                runs.append(gpu_run(cfg, 80, rho, precision=precision, variants=v, flags=ZB)[:2])
        if precision == "mixed":  # the 7-wave flat head exists in the mixed precision only
            for v in [(6, 0, 1, 3, 0), (6, 0, 0, 0, 0), (6, 0, 0, 0, 1)]:
                runs.append(gpu_run(cfg, 80, rho, precision=precision, variants=v)[:2])
                runs.append(gpu_run(cfg, 80, rho, precision=precision, variants=v, flags=ZB)[:2])
    assert st1.used_graph == 1 and st2.used_graph == 0
    assert st1.kernels_per_step == st1.m and st5.kernels_per_step == st5.m - 1
    assert st8.kernels_per_step == st8.m
    if len(n) == 2:  # all inner stages in one launch, also over an odd call split
        runs.append(gpu_run(cfg, 80, rho, precision=precision, variants=(0, 0, 2, 0, 0))[:2])
        runs.append(gpu_run(cfg, 80, rho, precision=precision, variants=(0, 0, 3, 0, 0))[:2])
        V11, z11, st11 = gpu_run(cfg, 80, rho, precision=precision, chunks=[1, 33, 7, 39], variants=(0, 0, 4, 0, 0))
        assert st11.kernels_per_step == 1
        runs.append((V11, z11))
        V10, z10, st10 = gpu_run(cfg, 80, rho, precision=precision, chunks=[1, 33, 7, 39], variants=(0, 0, 2, 0, 0))
        assert st10.kernels_per_step == 2
        assert np.array_equal(V10, V1) and np.array_equal(z10, z1)
    if len(n) == 3:  # the split stage with z in blocks over an odd call split
        for v in [(8, 0, 1, 4, 0), (7, 3, 1, 4, 0)]:
            runs.append(gpu_run(cfg, 80, rho, precision=precision, flags=ZB, variants=v, chunks=[1, 33, 7, 39])[:2])
    if len(n) == 3:  # the split stage with an odd call split (ping-pong and the final copy)
        V9, z9, st9 = gpu_run(cfg, 80, rho, precision=precision, chunks=[1, 33, 7, 39], variants=(7, 3, 1, 4, 0))
        assert st9.kernels_per_step == st9.m
        assert np.array_equal(V9, V1) and np.array_equal(z9, z1)
    for V, z in runs:
        assert np.array_equal(V, V1) and np.array_equal(z, z1)


def test_autotune_keeps_state_and_results(E):
    """The autotuner leaves the state untouched, picks valid shapes, and the
    run with its choice equals the default run bit for bit."""
    import torch
    cfg = small_config("c2_3d_crn", (41, 19, 33))
    rho = (51.0, 4.4)
    V1, z1, _ = gpu_run(cfg, 30, rho)
    sim = E.simulation_from_config(cfg, rho=rho)
    E.emrkc_init_state(sim.ctx, sim.state)
    V0, z0 = sim.V.clone(), sim.z.clone()
    v = E.emrkc_autotune(sim.ctx, sim.state, cfg["dt"], reps=2)
    assert torch.equal(sim.V, V0) and torch.equal(sim.z, z0)
    assert v == E.emrkc_get_variants(sim.ctx)
    assert len(v) == 5 and v[0] in range(9) and v[2] in (0, 1) and v[4] in (0, 1)
    assert (v[0] in (1, 2, 7)) == (v[1] > 0) and (v[2] == 0) == (v[3] == 0)
    E.emrkc_step(sim.ctx, sim.state, cfg["dt"], 30)
    torch.cuda.synchronize()
    assert np.array_equal(sim.V.cpu().numpy(), V1)
    assert np.array_equal(sim.z.cpu().numpy().astype(np.float64), z1)
    with pytest.raises(E.EmrkcError):
        E.emrkc_set_variants(sim.ctx, (3, 4, 0, 0, 0))
    with pytest.raises(E.EmrkcError):
        E.emrkc_set_variants(sim.ctx, (1, 34, 0, 0, 0))
    with pytest.raises(E.EmrkcError):
        E.emrkc_set_variants(sim.ctx, (0, 0, 0, 0, 2))
    with pytest.raises(E.EmrkcError):  # the 7-wave flat head is a mixed-precision kernel
        E.emrkc_set_variants(sim.ctx, (6, 0, 0, 0, 0))
    sim.close()


@pytest.mark.parametrize("model,n", [("HH", (65, 65)), ("CRN_SURR", (37, 29, 11)), ("TTP_SURR", (21, 17, 9))])
def test_estimate_rho_matches_oracle(E, model, n):
    """Power iteration on the GPU against the oracle's Compute_Rho from the
    same splitmix64 start: same iteration counts, radii within the
    finite-difference noise of delta = 1e-8 ||y|| (about 1e-8 relative per
    evaluation; 1e-6 allowed)."""
    import torch
    base = "c1_2d_hh" if len(n) == 2 else "c2_3d_crn"
    cfg = small_config(base, n, model=model)
    prob = build_grid_problem(cfg)
    y = prob.uniform_state()
    rF, rS, itF, itS = oracle_rho(prob, y)
    sim = E.simulation_from_config(cfg)
    E.emrkc_init_state(sim.ctx, sim.state)
    gF, gS, gitF, gitS, rc = E.emrkc_estimate_rho(sim.ctx, sim.state)
    assert (gitF, gitS) == (itF, itS)
    assert gF == pytest.approx(rF, rel=1e-6) and gS == pytest.approx(rS, rel=1e-6)
    # warm restart converges at once to the same values
    gF2, gS2, it2F, it2S, _ = E.emrkc_estimate_rho(sim.ctx, sim.state)
    assert it2F <= 2 and it2S <= 2
    assert gF2 == pytest.approx(gF, rel=2e-2) and gS2 == pytest.approx(gS, rel=2e-2)
    sim.close()


def test_check_finite_reports_nan(E):
    import torch
    cfg = small_config("c2_3d_crn", (9, 7, 5))
    sim = E.simulation_from_config(cfg, rho=(51.0, 4.4), flags=E.EMRKC_CHECK_FINITE)
    E.emrkc_init_state(sim.ctx, sim.state)
    E.emrkc_step(sim.ctx, sim.state, 0.05, 3)
    sim.V[17] = float("nan")
    with pytest.raises(E.EmrkcError) as ei:
        E.emrkc_step(sim.ctx, sim.state, 0.05, 1)
    assert ei.value.code == E.EMRKC_ENONFINITE
    sim.close()


def test_step_without_radii_is_rejected(E):
    cfg = small_config("c2_3d_crn", (9, 7, 5))
    sim = E.simulation_from_config(cfg)
    E.emrkc_init_state(sim.ctx, sim.state)
    with pytest.raises(E.EmrkcError) as ei:
        E.emrkc_step(sim.ctx, sim.state, 0.05, 1)
    assert ei.value.code == E.EMRKC_EINVAL
    sim.close()


@pytest.mark.slow
def test_c2_full_size_prefix_fp64(E):
    """The benchmark workload itself (201 x 71 x 31, CRN surrogate) for the
    first 10 steps (stimulus on), every node compared."""
    cfg = get_config("c2_3d_crn")
    prob = build_grid_problem(cfg)
    rF, rS, _, _ = oracle_rho(prob, prob.uniform_state())
    _compare_full(cfg, 10, (rF, rS))



@pytest.mark.parametrize("n,rho", [((2, 2, 2), (200.0, 4.4)), ((2, 3), (1600.0, 0.9)), ((3, 2, 5), (300.0, 4.4)),
                                   ((2, 2, 9), (60.0, 4.4))])
def test_minimal_grids(E, n, rho):
    """Grids with two nodes along an axis (every neighbour on that axis is a
    mirrored boundary node, and one tile or column covers the grid with
    most threads outside it) against the oracle; on 3-D grids every kernel
    shape gives the same bits."""
    base = "c1_2d_hh" if len(n) == 2 else "c2_3d_crn"
    cfg = small_config(base, n)
    if len(n) == 2:
        cfg["h"] = (0.2, 0.2)
    cfg["stim"]["width"] = 0.5 * min(cfg["h"][:len(n)])  # the corner node only: V varies over the grid
    nsteps = 30
    prob, y = oracle_run(cfg, nsteps, rho)
    assert np.ptp(y[:prob.N]) > 0.1
    V, z, _ = gpu_run(cfg, nsteps, rho)
    Y = y.reshape(prob.nv, prob.N)
    l2, mx = rel_errors(V, Y[0])
    assert l2 <= 1e-10 and mx <= 1e-10, (l2, mx)
    assert np.abs(z - Y[1:]).max() <= 1e-10 * np.abs(Y[1:]).max()
    if len(n) == 2:  # all inner stages in one launch: reflected halos reach across the whole grid
        for v in [(0, 0, 2, 0, 0), (0, 0, 3, 0, 0), (0, 0, 4, 0, 0)]:
            V2, z2, st2 = gpu_run(cfg, nsteps, rho, variants=v)
            assert st2.kernels_per_step == (1 if v[2] == 4 else 2)
            assert np.array_equal(V2, V) and np.array_equal(z2, z), v
    if len(n) == 3:
        for v in [(1, 1, 1, 1, 0), (2, n[2], 1, n[2], 0), (2, 1, 0, 0, 1), (3, 0, 1, 2, 0), (0, 0, 0, 0, 0),
                  (5, 0, 1, 1, 0), (5, 0, 0, 0, 0), (7, 1, 0, 0, 0), (7, n[2], 1, 1, 0), (8, 0, 0, 0, 0)]:
            V2, z2, _ = gpu_run(cfg, nsteps, rho, variants=v)
            assert np.array_equal(V2, V) and np.array_equal(z2, z), v


def test_zero_conductivity_decouples_the_cells(E):
    """sigma = 0, a degenerate case of the method: f_F = 0, the power
    iteration reports rho_F = 0 and the stage plan has one inner stage; every
    node then follows its own cell ODE.  The run equals the oracle's with the
    same radii to 1e-10, and all stimulated nodes (and all others) stay equal."""
    import torch
    from oracle.emrkc import emrkc_run
    from oracle.monodomain import build_grid_problem
    from workloads.configs import stim_mask
    cfg = small_config("c2_3d_crn", (9, 7, 5))
    cfg["sigma"] = (0.0, 0.0, 0.0)
    cfg["stim"]["width"] = 0.25   # a corner of 3 x 3 x 3 nodes
    sim = E.simulation_from_config(cfg)
    E.emrkc_init_state(sim.ctx, sim.state)
    rF, rS, _, _, _ = E.emrkc_estimate_rho(sim.ctx, sim.state)
    assert rF == 0.0 and rS > 1.0
    s, m, _ = E.emrkc_stages(sim.ctx, cfg["dt"])[:3]
    assert (s, m) == (1, 1)
    nsteps = 40
    E.emrkc_step(sim.ctx, sim.state, cfg["dt"], nsteps)
    torch.cuda.synchronize()
    V = sim.V.cpu().numpy().copy()
    z = sim.z.cpu().numpy().astype(np.float64)
    sim.close()
    prob = build_grid_problem(cfg)
    y = emrkc_run(prob, prob.uniform_state(), 0.0, cfg["dt"], nsteps, rF, rS)
    Y = y.reshape(prob.nv, prob.N)
    l2, mx = rel_errors(V, Y[0])
    assert l2 <= 1e-10 and mx <= 1e-10, (l2, mx)
    assert np.abs(z - Y[1:]).max() <= 1e-10 * np.abs(Y[1:]).max()
    mask = stim_mask(cfg).astype(bool)
    assert 0 < mask.sum() < mask.size
    assert np.ptp(V[mask]) == 0.0 and np.ptp(V[~mask]) == 0.0 and V[mask][0] > V[~mask][0] + 10.0


@pytest.mark.parametrize("method", ["emrkc", "exexrl"])
def test_step_size_change_continues_the_clock(E, method):
    """A state advanced with one step size and then stepped with another
    continues from its own time: the second call's stage times and the end
    of the stimulus window are those of the oracle started at t1 = n1 dt1
    with dt2 (without the rebase the window would close 0.36 ms late)."""
    import torch
    from oracle.emrkc import emrkc_run
    from oracle.exexrl import exexrl_step
    cfg = small_config("c2_3d_crn", (21, 11, 7))
    cfg["stim"] = dict(cfg["stim"], t_off=1.21)  # no stage time within 1e-3 of it
    rho = (51.0, 4.4)
    # EXEX-RL's explicit diffusion needs dt < 2 / rho_F (about 0.04 ms here)
    dt1, n1, dt2, n2 = (0.05, 12, 0.02, 40) if method == "emrkc" else (0.03, 20, 0.02, 40)
    sim = E.simulation_from_config(cfg, rho=rho)
    E.emrkc_init_state(sim.ctx, sim.state)
    step = E.emrkc_step if method == "emrkc" else E.emrkc_exexrl_step
    step(sim.ctx, sim.state, dt1, n1)
    step(sim.ctx, sim.state, dt2, n2)
    torch.cuda.synchronize()
    V = sim.V.cpu().numpy()
    assert sim.state.step == n1 + n2
    assert abs(sim.state.t - (n1 * dt1 + n2 * dt2)) < 1e-13
    sim.close()
    prob = build_grid_problem(cfg)
    y = prob.uniform_state()
    if method == "emrkc":
        y = emrkc_run(prob, y, 0.0, dt1, n1, *rho)
        y = emrkc_run(prob, y, n1 * dt1, dt2, n2, *rho)
    else:
        for n in range(n1):
            y = exexrl_step(n * dt1, y, dt1, prob)
        for n in range(n2):
            y = exexrl_step(n1 * dt1 + n * dt2, y, dt2, prob)
    l2, mx = rel_errors(V, y[:prob.N])
    assert l2 < FP64_TOL and mx < FP64_TOL, (l2, mx)
