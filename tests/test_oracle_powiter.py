"""Pins for the oracle's nonlinear power iteration (appendix) and its
random start vector."""
import numpy as np
import pytest

from oracle import fem
from oracle.ionic import HH, LinearTest
from oracle.monodomain import Monodomain, build_grid_problem
from oracle.powiter import compute_rho, random_unit_interval, splitmix64
from workloads.configs import get_config


def test_splitmix64_published_first_output():
    """splitmix64 from state 0: first output 0xE220A8397B1DCDAF."""
    assert int(splitmix64(1, 0)[0]) == 0xE220A8397B1DCDAF


def test_random_vector_range_and_mean():
    v = random_unit_interval(200000, 0)
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(v.mean()) < 0.01
    assert abs((v ** 2).mean() - 1.0 / 3.0) < 0.01
    assert not np.array_equal(v, random_unit_interval(200000, 1))


def test_rho_F_converges_to_closed_form_max_eigenvalue():
    """With a tight tolerance the iteration converges to the largest
    eigenvalue of (chi Cm M_L)^{-1} K, 4 sigma_x/(h^2 chi Cm) on a grid."""
    n, h, sig, chi, Cm = (6, 5), (0.1, 0.1), (0.17, 0.019), 1.4, 0.5
    K, ML, _ = fem.assemble_q1_grid(list(n), list(h), list(sig))
    prob = Monodomain(K, ML, chi, Cm, LinearTest())
    y = np.concatenate([np.linspace(-80, 20, prob.N), np.zeros(prob.N)])
    v0 = random_unit_interval(y.size, 0)
    # finite differences at delta = 1e-8 |y| limit the attainable tolerance
    _, rho, it, ok = compute_rho(0.0, y, prob.f_F, v0, tol=1e-7, max_iter=100000)
    assert ok
    assert rho == pytest.approx(4 * sig[0] / h[0] ** 2 / (chi * Cm), rel=1e-5)


def test_rho_F_default_tolerance_on_c1_is_a_lower_estimate():
    cfg = get_config("c1_2d_hh")
    prob = build_grid_problem(cfg)
    y = prob.uniform_state()
    _, rho, it, ok = compute_rho(0.0, y, prob.f_F, random_unit_interval(y.size, 0))
    exact = 4 * 0.1 * 64 ** 2
    assert ok and 0.8 * exact < rho < exact * (1 + 1e-6)


def test_rho_S_hh_closed_form():
    """f_S of HH has a single nonzero Jacobian row per node, so
    rho_S = (g_Na m^3 h + g_K n^4 + g_L) at the state (per capacitance)."""
    K, ML, _ = fem.assemble_q1_grid([4, 3], [0.1, 0.1], [0.1, 0.1])
    prob = Monodomain(K, ML, 1.0, 1.0, HH())
    y = prob.uniform_state()
    V, zE, _ = prob.split(y)
    m, h, n = zE
    # vary the state a little per node so that one node dominates
    y = y.copy()
    y[0] = -60.0
    V, zE, _ = prob.split(y)
    m, h, n = zE
    g = 120 * m ** 3 * h + 36 * n ** 4 + 0.3
    _, rho, it, ok = compute_rho(0.0, y, prob.f_S, random_unit_interval(y.size, 0), tol=1e-10, max_iter=200)
    assert ok
    assert rho == pytest.approx(g.max(), rel=1e-6)


def test_rho_S_linear_model_is_a():
    K, ML, _ = fem.assemble_q1_grid([4, 3], [0.1, 0.1], [0.1, 0.1])
    prob = Monodomain(K, ML, 1.0, 2.0, LinearTest(a=3.25, lam_E=-7.0))
    y = np.concatenate([np.linspace(1, 2, prob.N), np.zeros(prob.N)])
    _, rho, it, ok = compute_rho(0.0, y, prob.f_S, random_unit_interval(y.size, 0))
    assert ok and rho == pytest.approx(3.25, rel=1e-7)


def test_max_iter_reports_non_convergence_and_zero_state_uses_eps():
    K, ML, _ = fem.assemble_q1_grid([5, 5], [0.1, 0.1], [0.1, 0.1])
    prob = Monodomain(K, ML, 1.0, 1.0, LinearTest())
    y = np.zeros(2 * prob.N)
    v, rho, it, ok = compute_rho(0.0, y, prob.f_F, random_unit_interval(y.size, 0), max_iter=1)
    assert it == 1 and not ok and rho > 0
    v2, rho2, it2, ok2 = compute_rho(0.0, y, prob.f_F, v, rho)
    assert ok2 and it2 >= 1


@pytest.mark.parametrize("name", ["CRN_SURR", "TTP_SURR"])
def test_rho_S_surrogates_against_jacobian_eigenvalues(name):
    """The nonlinear power iteration on f_S of the surrogates (whose slow
    variables couple back into V) estimates the spectral radius of f_S's
    Jacobian within its tolerance (1e-2): against the largest eigenvalue
    magnitude of a central-difference Jacobian from numpy's dense
    eigensolver.  Two nodes at different potentials: f_S is pointwise, so
    the radius is the larger of the two nodes' blocks."""
    import scipy.sparse as sp
    from oracle.ionic import make_model
    model = make_model(name)
    prob = Monodomain(sp.csr_matrix((2, 2)), np.ones(2), 140.0, 0.01, model)
    y = prob.uniform_state().copy()
    y[0], y[1] = -40.0, 10.0
    n = y.size
    J = np.zeros((n, n))
    for j in range(n):
        h = 1e-6 * max(1.0, abs(y[j]))
        e = np.zeros(n)
        e[j] = h
        J[:, j] = (prob.f_S(0.0, y + e) - prob.f_S(0.0, y - e)) / (2 * h)
    lam = np.abs(np.linalg.eigvals(J)).max()
    _, rho, it, ok = compute_rho(0.0, y, prob.f_S, random_unit_interval(n, 0))
    assert ok and it < 20
    assert abs(rho - lam) <= 1e-2 * lam, (rho, lam)
