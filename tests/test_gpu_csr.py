"""The assembled-operator boundary (EMRKC_MESH_CSR: A = -K and the lumped
mass given by the caller, the semi-discrete system of section "Space
discretization" with its matrices supplied).  Input: a seeded random graph
Laplacian (test-local generator) with random lumped masses; the oracle runs
the same matrices.  Parity of emRKC and IMEX-RL, invariance to duplicate and
unsorted entries, and rejection of malformed input."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import rel_errors
from oracle.emrkc import emrkc_run
from oracle.exexrl import imexrl_run
from oracle.ionic import make_model
from oracle.monodomain import Monodomain
from oracle.powiter import compute_rho, random_unit_interval

pytestmark = pytest.mark.gpu

CHI, CM = 140.0, 0.01
STIM = dict(amp=2.0, t_on=0.0, t_off=2.0)
# HH runs in the scaled units of the unit-square workload
UNITS = {"HH": (1.0, 1.0, dict(amp=100.0, t_on=0.0, t_off=1.0))}


def random_laplacian(n, deg, seed):
    """A = W - diag(W 1) for a random symmetric W >= 0 (each node linked to
    `deg` random others), and lumped masses in [0.5, 1.5] * 1e-3."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), deg)
    cols = rng.integers(0, n, n * deg)
    keep = rows != cols
    w = rng.uniform(0.002, 0.01, keep.sum())
    W = sp.coo_matrix((w, (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    W = W + W.T
    A = (W - sp.diags(np.asarray(W.sum(axis=1)).ravel())).tocsr()
    ML = rng.uniform(0.5, 1.5, n) * 1e-3
    mask = np.zeros(n, np.uint8)
    mask[rng.choice(n, n // 20, replace=False)] = 1
    return A, ML, mask


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


def _units(model):
    return UNITS.get(model, (CHI, CM, STIM))


def _oracle(A, ML, mask, model):
    chi, cm, st = _units(model)
    return Monodomain(-A, ML, chi, cm, make_model(model), mask, st["amp"], st["t_on"], st["t_off"])


def _rho(prob):
    y = prob.uniform_state()
    v0 = random_unit_interval(y.size, 0)
    _, rF, _, _ = compute_rho(0.0, y, prob.f_F, v0.copy())
    _, rS, _, _ = compute_rho(0.0, y, prob.f_S, v0.copy())
    return 1.05 * rF, 1.05 * rS


def _run(E, A, ML, mask, model, rho, dt, nsteps, method="emrkc", precision="fp64"):
    import torch
    chi, cm, st = _units(model)
    sim = E.simulation_from_csr(A, ML, chi, cm, model, mask, st, precision=precision, rho=rho)
    E.emrkc_init_state(sim.ctx, sim.state)
    if method == "imexrl":
        E.emrkc_imexrl_step(sim.ctx, sim.state, dt, nsteps)
    else:
        E.emrkc_step(sim.ctx, sim.state, dt, nsteps)
    torch.cuda.synchronize()
    out = sim.V.cpu().numpy().copy(), sim.z.cpu().numpy().astype(np.float64)
    sim.close()
    return out


def _check(prob, y, V, z, tol=1e-10):
    Y = y.reshape(prob.nv, prob.N)
    l2, mx = rel_errors(V, Y[0])
    assert l2 <= tol and mx <= tol, (l2, mx)
    assert np.abs(z - Y[1:]).max() <= tol * np.abs(Y[1:]).max()


@pytest.mark.parametrize("model,n,deg", [("CRN_SURR", 3000, 6), ("TTP_SURR", 2000, 9), ("HH", 1500, 4)])
def test_csr_emrkc_parity(E, model, n, deg):
    A, ML, mask = random_laplacian(n, deg, seed=n)
    prob = _oracle(A, ML, mask, model)
    rho = _rho(prob)
    dt, nsteps = 0.05, 60
    y = emrkc_run(prob, prob.uniform_state(), 0.0, dt, nsteps, *rho)
    assert np.all(np.isfinite(y)) and np.ptp(y[:prob.N]) > 0.1
    V, z = _run(E, A, ML, mask, model, rho, dt, nsteps)
    _check(prob, y, V, z)


def test_csr_emrkc_mixed(E):
    """The mixed precision on an assembled operator (float ELL weights and
    products, float ionic state) against the FP64 oracle."""
    A, ML, mask = random_laplacian(3000, 6, seed=3000)
    prob = _oracle(A, ML, mask, "CRN_SURR")
    rho = _rho(prob)
    dt, nsteps = 0.05, 60
    y = emrkc_run(prob, prob.uniform_state(), 0.0, dt, nsteps, *rho)
    V, z = _run(E, A, ML, mask, "CRN_SURR", rho, dt, nsteps, precision="mixed")
    Y = y.reshape(prob.nv, prob.N)
    l2, mx = rel_errors(V, Y[0])
    assert l2 <= 1e-5 and mx <= 1e-4, (l2, mx)
    assert np.abs(z - Y[1:]).max() <= 1e-4 * np.abs(Y[1:]).max()


def test_csr_imexrl_parity(E):
    A, ML, mask = random_laplacian(2500, 6, seed=7)
    prob = _oracle(A, ML, mask, "CRN_SURR")
    dt, nsteps = 0.1, 30
    y = imexrl_run(prob, prob.uniform_state(), 0.0, dt, nsteps)
    V, z = _run(E, A, ML, mask, "CRN_SURR", None, dt, nsteps, method="imexrl")
    _check(prob, y, V, z)


def test_csr_duplicates_unsorted_and_explicit_diagonal(E):
    """Each entry split into two halves (exact), the rows shuffled, the
    diagonal kept: the same operator, so the same run to rounding."""
    A, ML, mask = random_laplacian(1800, 5, seed=11)
    prob = _oracle(A, ML, mask, "CRN_SURR")
    rho = _rho(prob)
    V0, z0 = _run(E, A, ML, mask, "CRN_SURR", rho, 0.05, 40)
    C = A.tocoo()
    rng = np.random.default_rng(3)
    r = np.concatenate([C.row, C.row])
    c = np.concatenate([C.col, C.col])
    v = np.concatenate([0.5 * C.data, 0.5 * C.data])
    perm = rng.permutation(r.size)
    order = np.argsort(r[perm], kind="stable")
    r, c, v = r[perm][order], c[perm][order], v[perm][order]
    row_ptr = np.zeros(A.shape[0] + 1, np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    B = sp.csr_matrix((v, c.astype(np.int32), row_ptr), shape=A.shape)
    B.has_sorted_indices = False
    V1, z1 = _run(E, B, ML, mask, "CRN_SURR", rho, 0.05, 40)
    assert rel_errors(V1, V0)[1] <= 1e-13 and np.abs(z1 - z0).max() <= 1e-13 * np.abs(z0).max()


def test_csr_malformed_input_rejected(E):
    A, ML, mask = random_laplacian(400, 4, seed=5)
    bad_sum = A.tolil()
    bad_sum[3, 3] += 1e-6
    with pytest.raises(E.EmrkcError):
        E.simulation_from_csr(bad_sum.tocsr(), ML, CHI, CM, "CRN_SURR", mask, STIM)
    bad_mass = ML.copy()
    bad_mass[7] = 0.0
    with pytest.raises(E.EmrkcError):
        E.simulation_from_csr(A, bad_mass, CHI, CM, "CRN_SURR", mask, STIM)
    wide = random_laplacian(200, 60, seed=9)[0]   # rows with more than 64 neighbours
    assert np.diff(wide.indptr).max() > 65
    with pytest.raises(E.EmrkcError):
        E.simulation_from_csr(wide, np.full(200, 1e-3), CHI, CM, "CRN_SURR")
