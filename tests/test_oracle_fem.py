"""Pins for the oracle's finite-element assembly (section "Space
discretization"): symmetry, K.1 = 0, semidefiniteness, lumped mass sums to
the volume, the tensor-product form of Q1 on a grid, the closed form of one
P1 tetrahedron, the patch test, and the closed-form Neumann spectrum of
M_L^{-1} K on Q1 grids."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem


def one_d(n, h):
    K = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil() / h
    K[0, 0] = 1.0 / h
    K[n - 1, n - 1] = 1.0 / h
    M = sp.diags([np.ones(n - 1) / 6, 2 * np.ones(n) / 3, np.ones(n - 1) / 6], [-1, 0, 1]).tolil() * h
    M[0, 0] = h / 3
    M[n - 1, n - 1] = h / 3
    return K.tocsr(), M.tocsr()


@pytest.mark.parametrize("n,h,sig", [((5, 4), (0.25, 1 / 3), (0.1, 0.1)),
                                     ((6, 3), (0.1, 0.2), (0.17, 0.019)),
                                     ((4, 3, 5), (0.1, 0.2, 0.3), (0.17, 0.019, 0.03)),
                                     ((3, 3, 3), (0.1, 0.1, 0.1), (1.0, 1.0, 1.0))])
def test_q1_invariants_and_tensor_form(n, h, sig):
    K, ML, M = fem.assemble_q1_grid(list(n), list(h), list(sig))
    N = int(np.prod(n))
    Kd = K.toarray()
    assert np.abs(Kd - Kd.T).max() < 1e-14 * np.abs(Kd).max()
    assert np.abs(K @ np.ones(N)).max() < 1e-13 * np.abs(Kd).max()
    assert np.linalg.eigvalsh(Kd).min() > -1e-12 * np.abs(Kd).max()
    vol = np.prod([(nn - 1) * hh for nn, hh in zip(n, h)])
    assert ML.sum() == pytest.approx(vol, rel=1e-14)
    assert np.all(ML > 0)
    # tensor-product identity, x fastest: K = sum_d sig_d (... x K_d x ...)
    ones = [one_d(nn, hh) for nn, hh in zip(n, h)]
    d = len(n)
    Kt = 0
    Mt = None
    for k in range(d):
        fac = None
        for axis in range(d):
            mat = ones[axis][0] if axis == k else ones[axis][1]
            fac = mat if fac is None else sp.kron(mat, fac)
        Kt = Kt + sig[k] * fac
    for axis in range(d):
        Mt = ones[axis][1] if Mt is None else sp.kron(ones[axis][1], Mt)
    assert np.abs(Kt.toarray() - Kd).max() < 1e-13 * np.abs(Kd).max()
    assert np.abs(Mt.toarray() - M.toarray()).max() < 1e-15


def test_p1_single_reference_tet():
    xs = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    Ke, Me, vol = fem.p1_tet_element(xs, np.eye(3))
    ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    assert vol == pytest.approx(1 / 6)
    assert np.abs(Ke - ref).max() < 1e-15
    assert Me.sum() == pytest.approx(1 / 6)
    assert np.abs(Me.sum(axis=1) - vol / 4).max() < 1e-16


def test_p1_skewed_tet_against_barycentric_interpolation():
    """A skewed tetrahedron (non-symmetric edge matrix): the element
    stiffness equals |T| g_a . D g_b with the barycentric gradients g_a
    obtained independently, as the linear parts of the affine functions
    that interpolate the unit vectors at the vertices (solve of the 4x4
    system [1 x y z]); the vectorised assembly of the one-element mesh gives
    the same matrix, and K reproduces a linear field's flux exactly."""
    xs = np.array([[0.1, -0.2, 0.05], [1.3, 0.4, -0.1], [0.2, 0.9, 0.3], [-0.1, 0.35, 1.1]])
    D = fem.conductivity_from_fibre([0.8, -0.3, 0.5], 0.17, 0.019)
    A = np.hstack([np.ones((4, 1)), xs])
    coef = np.linalg.solve(A, np.eye(4))          # column a: lambda_a = c0 + g . x
    g = coef[1:].T                                # row a: gradient of lambda_a
    vol = abs(np.linalg.det(xs[1:] - xs[0])) / 6.0
    ref = vol * g @ D @ g.T
    Ke, _, v = fem.p1_tet_element(xs, D)
    assert v == pytest.approx(vol, rel=1e-14)
    assert np.abs(Ke - ref).max() <= 1e-14 * np.abs(ref).max()
    K, _, _ = fem.assemble_p1_tets(xs, np.array([[0, 1, 2, 3]]), np.array([[0.8, -0.3, 0.5]]), 0.17, 0.019)
    assert np.abs(K.toarray() - ref).max() <= 1e-14 * np.abs(ref).max()
    grad = np.array([0.7, -1.2, 0.4])
    assert np.abs(K @ (xs @ grad) - vol * g @ D @ grad).max() <= 1e-14


def test_p1_fibre_conductivity():
    D = fem.conductivity_from_fibre([2.0, 0, 0], 0.17, 0.019)
    assert np.allclose(D, np.diag([0.17, 0.019, 0.019]), atol=1e-16)
    a = np.array([1.0, 2.0, -0.5])
    D = fem.conductivity_from_fibre(a, 0.2, 0.05)
    an = a / np.linalg.norm(a)
    assert D @ an == pytest.approx(0.2 * an)
    perp = np.cross(an, [0, 0, 1.0])
    assert D @ perp == pytest.approx(0.05 * perp)


def kuhn_cube_mesh(n, h, jitter=0.0, seed=0):
    """Structured cube split into 6 Kuhn tetrahedra per cell (test-local)."""
    idx = lambda i, j, k: i + n * (j + n * k)
    coords = np.array([[i * h, j * h, k * h] for k in range(n) for j in range(n) for i in range(n)], float)
    tets = []
    for k, j, i in itertools.product(range(n - 1), repeat=3):
        c = [idx(i + a, j + b, k + cc) for cc in (0, 1) for b in (0, 1) for a in (0, 1)]
        for p in itertools.permutations(range(3)):
            path = [0]
            cur = [0, 0, 0]
            for axis in p:
                cur[axis] = 1
                path.append(cur[0] + 2 * cur[1] + 4 * cur[2])
            tets.append([c[q] for q in path])
    coords = coords.copy()
    if jitter:
        rng = np.random.default_rng(seed)
        interior = np.all((coords > 1e-12) & (coords < (n - 1) * h - 1e-12), axis=1)
        coords[interior] += rng.uniform(-jitter, jitter, (interior.sum(), 3)) * h
    return coords, np.array(tets, dtype=np.int64)


def test_p1_mesh_invariants_and_patch_test():
    coords, tets = kuhn_cube_mesh(4, 0.5, jitter=0.1, seed=3)
    fib = np.tile([1.0, 0.3, 0.2], (tets.shape[0], 1))
    K, ML, M = fem.assemble_p1_tets(coords, tets, fib, 0.17, 0.019)
    Kd = K.toarray()
    N = coords.shape[0]
    assert np.abs(Kd - Kd.T).max() < 1e-14
    assert np.abs(K @ np.ones(N)).max() < 1e-14
    assert np.linalg.eigvalsh(Kd).min() > -1e-13
    assert ML.sum() == pytest.approx(1.5 ** 3, rel=1e-13)
    # patch test: a linear field has zero discrete flux at interior nodes
    interior = np.all((coords > 1e-12) & (coords < 1.5 - 1e-12), axis=1)
    for g in ([1.0, 0, 0], [0.3, -2.0, 0.7]):
        u = coords @ np.array(g)
        assert np.abs((K @ u)[interior]).max() < 1e-13


def neumann_spectrum(n, h, sig):
    """Closed-form eigenvalues of M_L^{-1}K for Q1 on a grid with Neumann
    boundary: cosine modes theta_d = k pi/(n_d - 1),
    eig = sum_d sig_d lam_d prod_{e != d} mu_e,
    lam_d = (2 - 2 cos theta_d)/h_d^2, mu_e = (2 + cos theta_e)/3."""
    thetas = [np.pi * np.arange(nn) / (nn - 1) for nn in n]
    out = []
    for ks in itertools.product(*[range(nn) for nn in n]):
        th = [thetas[d][k] for d, k in enumerate(ks)]
        lam = [(2 - 2 * np.cos(t)) / hh ** 2 for t, hh in zip(th, h)]
        mu = [(2 + np.cos(t)) / 3 for t in th]
        e = 0.0
        for d in range(len(n)):
            e += sig[d] * lam[d] * np.prod([mu[q] for q in range(len(n)) if q != d])
        out.append(e)
    return np.sort(out)


@pytest.mark.parametrize("n,h,sig", [((7, 5), (0.1, 0.1), (0.17, 0.019)),
                                     ((9, 9), (1 / 8, 1 / 8), (0.1, 0.1)),
                                     ((5, 4, 3), (0.1, 0.1, 0.1), (0.17, 0.019, 0.019))])
def test_q1_lumped_neumann_spectrum_closed_form(n, h, sig):
    K, ML, _ = fem.assemble_q1_grid(list(n), list(h), list(sig))
    # M_L^{-1} K is similar to the symmetric M^{-1/2} K M^{-1/2}
    s = 1.0 / np.sqrt(ML)
    ev = np.sort(np.linalg.eigvalsh((K.toarray() * s).T * s))
    ref = neumann_spectrum(n, h, sig)
    assert np.abs(ev - ref).max() < 1e-10 * ref.max()


def test_q1_max_eigenvalue_formula():
    """Largest eigenvalue is 4 sigma_x / h^2 when sigma_x dominates
    (corner {pi, 0, 0} of the mode set)."""
    ref = neumann_spectrum((6, 5, 4), (0.1, 0.1, 0.1), (0.17, 0.019, 0.019))
    assert ref.max() == pytest.approx(4 * 0.17 / 0.01, rel=1e-14)
