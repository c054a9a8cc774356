"""Pins for the oracle's stepping variants: stability condition A of the
stability lemma, the progressive splitting of the remark after eq. auxp_exp,
and the periodic warm-started re-estimation of the radii (appendix)."""
import numpy as np
import pytest

from oracle.emrkc import emrkc_run, emrkc_step, stage_counts
from oracle.monodomain import build_grid_problem
from oracle.powiter import compute_rho, random_unit_interval
from oracle.rkc import beta_of
from workloads.configs import small_config

from test_oracle_emrkc import P_cheb, Phi, ScalarTest, phi

BETA = beta_of(0.05)


def test_cond_a_stage_counts_definition():
    """Condition A: dt rho_S <= beta s^2 (s minimal), eta = 6 dt/(beta s^2)
    m^2/(m^2-1) and eta rho_F <= beta m^2 with m >= 2 minimal."""
    rng = np.random.default_rng(3)
    for _ in range(400):
        dt = 10 ** rng.uniform(-3, 1)
        rF = 10 ** rng.uniform(-1, 5)
        rS = 10 ** rng.uniform(-2, 3)
        s, m, eta = stage_counts(dt, rF, rS, cond="A")
        assert dt * rS <= BETA * s * s * (1 + 1e-12)
        assert s == 1 or dt * rS > BETA * (s - 1) ** 2
        assert m >= 2
        assert eta == pytest.approx(6 * dt / (BETA * s * s) * m * m / (m * m - 1.0), rel=1e-15)
        assert eta * rF <= BETA * m * m
        if m > 2:
            e1 = 6 * dt / (BETA * s * s) * (m - 1) ** 2 / ((m - 1) ** 2 - 1.0)
            assert e1 * rF > BETA * (m - 1) ** 2
        sb, mb, etab = stage_counts(dt, rF, rS)
        assert sb == s and eta > etab


def test_cond_a_general_stability():
    """The stability lemma under condition A: for any lam_F in [-rho_F, 0] and
    lam_S in [-rho_S, 0] (no scale separation assumed) the mRKC/emRKC
    amplification P_s(dt Phi_m(eta lam_F)(lam_F + lam_S)) stays in [-1, 1]."""
    rng = np.random.default_rng(5)
    for _ in range(60):
        dt = 10 ** rng.uniform(-2, 0.5)
        rF = 10 ** rng.uniform(0, 4)
        rS = 10 ** rng.uniform(-1, 2)
        s, m, eta = stage_counts(dt, rF, rS, cond="A")
        lF, lS = np.meshgrid(-np.linspace(0, rF, 301), -np.linspace(0, rS, 61), indexing="ij")
        amp = P_cheb(s, dt * Phi(m, eta * lF) * (lF + lS))
        assert np.abs(amp).max() <= 1.0 + 1e-10


def test_cond_a_scalar_closed_form():
    """The condition-A step is the same emRKC step with the other (m, eta):
    y_{n+1} = P_s(dt lam_bar) y_n."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        dt = 10 ** rng.uniform(-2, 0.5)
        rF = 10 ** rng.uniform(0, 4)
        rS = 10 ** rng.uniform(-1, 2)
        s, m, eta = stage_counts(dt, rF, rS, cond="A")
        k = 32
        lF, lS = -rng.uniform(0, rF, k), -rng.uniform(0, rS, k)
        lE = -10 ** rng.uniform(-2, 3, k)
        y0 = rng.uniform(0.5, 1.5, k)
        y1 = emrkc_step(0.0, y0, dt, ScalarTest(lF, lS, lE), rF, rS, cond="A")
        lbar = Phi(m, eta * lF) * (lF + lS) * np.exp(eta * lE) + phi(eta * lE) * lE
        ref = P_cheb(s, dt * lbar) * y0
        assert np.abs(y1 - ref).max() <= 1e-12 * np.abs(ref).max() + 1e-14


def test_progressive_scalar_closed_form():
    """Progressive splitting on y' = (lam_F + lam_S + lam_E) y (all three on
    one component): the inner problem u' = lam_F u + c, u(0) = y, with the
    constant c = lam_S y_E + (y_E - y)/eta gives
    lam_bar = Phi_m(eta lam_F)(lam_F + lam_S e^{eta lam_E} + phi(eta lam_E) lam_E),
    which differs from the standard splitting whenever lam_F lam_E != 0."""
    rng = np.random.default_rng(9)
    for _ in range(20):
        dt = 10 ** rng.uniform(-2, 0.5)
        rF = 10 ** rng.uniform(0, 4)
        rS = 10 ** rng.uniform(-1, 2)
        s, m, eta = stage_counts(dt, rF, rS)
        k = 32
        lF, lS = -rng.uniform(0, rF, k), -rng.uniform(0, rS, k)
        lE = -10 ** rng.uniform(-2, 3, k)
        y0 = rng.uniform(0.5, 1.5, k)
        prob = ScalarTest(lF, lS, lE)
        y1 = emrkc_step(0.0, y0, dt, prob, rF, rS, progressive=True)
        lbar = Phi(m, eta * lF) * (lF + lS * np.exp(eta * lE) + phi(eta * lE) * lE)
        ref = P_cheb(s, dt * lbar) * y0
        # the reference's Phi = (P_m(z) - 1)/z cancels for small |z|: 1e-11
        assert np.abs(y1 - ref).max() <= 1e-11 * np.abs(ref).max() + 1e-14
        std = emrkc_step(0.0, y0, dt, prob, rF, rS)
        assert np.abs(std - ref).max() > 1e-6 * np.abs(ref).max()


def test_progressive_equals_standard_on_the_monodomain_split():
    """On the monodomain split f_F acts on V only and f_E on the gates only,
    so the gate forcing of the progressive inner problem is constant and its
    end value z + c'_m (z_E - z) equals z_E up to the rounding of c'_m = 1:
    both splittings give the same step to ~1e-13."""
    cfg = small_config("c2_3d_crn", (9, 7, 5))
    prob = build_grid_problem(cfg)
    y = prob.uniform_state()
    rng = np.random.default_rng(1)
    y = y + 1e-3 * rng.standard_normal(y.size) * np.abs(y)
    for rho in [(51.0, 4.4), (700.0, 4.4), (150.0, 30.0)]:
        a = emrkc_step(0.5, y, cfg["dt"], prob, *rho)
        b = emrkc_step(0.5, y, cfg["dt"], prob, *rho, progressive=True)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_rho_every_linear_model_warm_start():
    """With the linear test model both Jacobians are constant: warm-started
    re-estimates reach the same radii in at most two iterations, and the
    run equals the run with fixed radii bit for bit (same stage counts)."""
    cfg = small_config("c1_2d_hh", (17, 13), model="LINEAR")
    kw = dict(a=2.0, lam_E=-3.0)
    prob = build_grid_problem(cfg, model_kw=kw)
    y0 = prob.uniform_state()
    y0 = y0 + np.cos(np.arange(y0.size) * 0.37)
    v0 = random_unit_interval(y0.size, 0)
    vF, rF, _, _ = compute_rho(0.0, y0, prob.f_F, v0.copy())
    vS, rS, _, _ = compute_rho(0.0, y0, prob.f_S, v0.copy())
    state = dict(vF=vF, vS=vS, rF=rF, rS=rS)
    seen = []
    ya = emrkc_run(prob, y0, 0.0, cfg["dt"], 30, 1.05 * rF, 1.05 * rS, rho_every=10, rho_state=state,
                   on_estimate=lambda n, a, b, i, j: seen.append((n, a, b, i, j)))
    yb = emrkc_run(prob, y0, 0.0, cfg["dt"], 30, 1.05 * rF, 1.05 * rS)
    assert [e[0] for e in seen] == [10, 20]
    for n, a, b, i, j in seen:
        assert i <= 2 and j <= 2
        assert a == pytest.approx(1.05 * rF, rel=2e-2) and b == pytest.approx(1.05 * rS, rel=2e-2)
    assert np.array_equal(ya, yb)


def _fS_blocks(prob, t, y):
    """Per-node Jacobian blocks of f_S at (t, y) by central differences (f_S
    is pointwise: perturbing one component at every node at once gives each
    node's column of its own block)."""
    N, nv = prob.N, prob.nv
    J = np.zeros((N, nv, nv))
    for k in range(nv):
        h = 1e-6 * max(1.0, np.abs(y[k * N:(k + 1) * N]).max())
        e = np.zeros_like(y)
        e[k * N:(k + 1) * N] = h
        J[:, :, k] = ((prob.f_S(t, y + e) - prob.f_S(t, y - e)) / (2 * h)).reshape(nv, N).T
    return J


def test_rho_every_estimates_at_the_scheduled_states():
    """CRN surrogate on a stimulated 5 x 4 x 3 grid, K = 15 over 40 steps:
    estimates happen before steps 15 and 30 (positive multiples of K), and
    * the run equals three plain runs with the reported radii in force
      (15, 15 and 10 steps), so the radii change exactly there;
    * the diffusion is linear, so every rho_F is the largest eigenvalue
      magnitude of the assembled operator (dense eigensolver) within the
      iteration's tolerance, and the warm start from the previous
      eigenvector needs one iteration;
    * Compute_Rho on f_S at each scheduled state (the state after n steps,
      time n dt), run from a fresh vector to a tight tolerance, reaches the
      largest eigenvalue magnitude of f_S's Jacobian there (dense eigensolver
      on the nodes' blocks; by step 30 the stimulated nodes are in the
      upstroke, whose radius differs from the resting one), and the
      scheduled warm estimate
      is within 10% of it (its stop at a 1% change per iteration can leave
      it a few percent above: f_S's Jacobian is far from normal)."""
    cfg = small_config("c2_3d_crn", (5, 4, 3))
    prob = build_grid_problem(cfg)
    dt = cfg["dt"]
    y0 = prob.uniform_state()
    v0 = random_unit_interval(y0.size, 0)
    vF, rF, _, _ = compute_rho(0.0, y0, prob.f_F, v0.copy())
    vS, rS, _, _ = compute_rho(0.0, y0, prob.f_S, v0.copy())
    seen, states = [], {}
    ya = emrkc_run(prob, y0, 0.0, dt, 40, 1.05 * rF, 1.05 * rS, rho_every=15,
                   rho_state=dict(vF=vF, vS=vS, rF=rF, rS=rS),
                   on_estimate=lambda n, a, b, i, j: seen.append((n, a, b, i, j)),
                   callback=lambda n, y: states.__setitem__(n, y.copy()))
    assert [e[0] for e in seen] == [15, 30]
    y = emrkc_run(prob, y0, 0.0, dt, 15, 1.05 * rF, 1.05 * rS)
    y = emrkc_run(prob, y, 15 * dt, dt, 15, seen[0][1], seen[0][2])
    y = emrkc_run(prob, y, 30 * dt, dt, 10, seen[1][1], seen[1][2])
    assert np.array_equal(ya, y)
    lamF = np.abs(np.linalg.eigvals(prob.A.toarray() / (prob.chi * prob.Cm * prob.ML)[:, None])).max()
    lam_rest = max(np.abs(np.linalg.eigvals(B)).max() for B in _fS_blocks(prob, 0.0, y0))
    shift = 0.0
    for n, rho_F, rho_S, itF, itS in seen:
        assert itF == 1
        assert abs(rho_F / 1.05 - lamF) <= 1e-2 * lamF, (n, rho_F, lamF)
        yn = states[n]
        lam = max(np.abs(np.linalg.eigvals(B)).max() for B in _fS_blocks(prob, n * dt, yn))
        shift = max(shift, abs(lam - lam_rest) / lam_rest)
        _, r, _, _ = compute_rho(n * dt, yn, prob.f_S, random_unit_interval(yn.size, 1), tol=1e-10, max_iter=20000)
        assert abs(r - lam) <= 1e-4 * lam, (n, r, lam)
        assert abs(rho_S / 1.05 - lam) <= 0.1 * lam, (n, rho_S, lam)
    assert shift > 0.02, shift
