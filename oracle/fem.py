"""Conforming P1/Q1 finite elements: stiffness matrix K (so that the paper's
A = -K), consistent mass and row-sum lumped mass (section "Space
discretization", eq. sd_sys).  FP64 numpy/scipy, element by element.
Test infrastructure only.

Readings: A is the negative semidefinite operator -K; the lumped mass is the
row sum of the consistent mass; Q1 integrals use the exact tensor 2-point
Gauss rule; the P1 conductivity of an element is built from its fibre
direction a_l as D = sigma_l a_l a_l^T + sigma_t (I - a_l a_l^T)
(eq. def_D with sigma_n = sigma_t).
"""
import itertools

import numpy as np
import scipy.sparse as sp

_GAUSS_1D = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))


def q1_element_matrices(h, D):
    """Stiffness and consistent mass of one axis-aligned Q1 element with edge
    lengths h (length d) and constant conductivity tensor D (d x d).
    Local node a has reference coordinates bits(a), x fastest."""
    d = len(h)
    corners = [tuple((a >> k) & 1 for k in range(d)) for a in range(2 ** d)]
    nloc = len(corners)
    Ke = np.zeros((nloc, nloc))
    Me = np.zeros((nloc, nloc))
    detJ = float(np.prod(h))
    for qp in itertools.product(_GAUSS_1D, repeat=d):
        w = (0.5 ** d) * detJ
        phi = np.empty(nloc)
        grad = np.empty((nloc, d))
        for a, c in enumerate(corners):
            fac = [qp[k] if c[k] else 1.0 - qp[k] for k in range(d)]
            phi[a] = np.prod(fac)
            for k in range(d):
                dk = (1.0 if c[k] else -1.0) / h[k]
                other = [fac[l] for l in range(d) if l != k]
                grad[a, k] = dk * (np.prod(other) if other else 1.0)
        Ke += w * grad @ D @ grad.T
        Me += w * np.outer(phi, phi)
    return Ke, Me, corners


def q1_grid_connectivity(n):
    """Global node indices of every element's local nodes (x fastest)."""
    d = len(n)
    ne = [nn - 1 for nn in n]
    # element multi-indices, x fastest
    grids = np.meshgrid(*[np.arange(v) for v in ne], indexing="ij")
    e_idx = [g.reshape(-1, order="F") for g in grids]
    strides = [1]
    for k in range(1, d):
        strides.append(strides[-1] * n[k - 1])
    corners = [tuple((a >> k) & 1 for k in range(d)) for a in range(2 ** d)]
    conn = np.empty((e_idx[0].size, len(corners)), dtype=np.int64)
    for a, c in enumerate(corners):
        g = np.zeros(e_idx[0].size, dtype=np.int64)
        for k in range(d):
            g += (e_idx[k] + c[k]) * strides[k]
        conn[:, a] = g
    return conn


def assemble_q1_grid(n, h, sigma):
    """K (csr) and lumped mass for a Q1 grid with n nodes per axis, spacing h
    and D = diag(sigma) (fibres along x)."""
    d = len(n)
    D = np.diag(np.asarray(sigma[:d], dtype=np.float64))
    Ke, Me, _ = q1_element_matrices(list(h[:d]), D)
    conn = q1_grid_connectivity(list(n))
    N = int(np.prod(n))
    nloc = conn.shape[1]
    rows = np.repeat(conn, nloc, axis=1).reshape(-1)
    cols = np.tile(conn, (1, nloc)).reshape(-1)
    K = sp.coo_matrix((np.tile(Ke.reshape(-1), conn.shape[0]), (rows, cols)), shape=(N, N)).tocsr()
    M = sp.coo_matrix((np.tile(Me.reshape(-1), conn.shape[0]), (rows, cols)), shape=(N, N)).tocsr()
    ML = np.asarray(M.sum(axis=1)).reshape(-1)
    return K, ML, M


def p1_tet_element(xs, D):
    """Stiffness |T| G D G^T and consistent mass of one P1 tetrahedron with
    vertex coordinates xs (4 x 3)."""
    B = np.stack([xs[1] - xs[0], xs[2] - xs[0], xs[3] - xs[0]], axis=1)
    vol = abs(np.linalg.det(B)) / 6.0
    Binv = np.linalg.inv(B)          # rows: gradients of lambda_1..lambda_3
    G = np.vstack([-Binv.sum(axis=0), Binv])
    Ke = vol * G @ D @ G.T
    Me = vol / 20.0 * (np.ones((4, 4)) + np.eye(4))
    return Ke, Me, vol


def conductivity_from_fibre(a, sigma_l, sigma_t):
    a = np.asarray(a, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return sigma_l * np.outer(a, a) + sigma_t * (np.eye(3) - np.outer(a, a))


def assemble_p1_tets(coords, tets, fibres, sigma_l, sigma_t):
    """K (csr), lumped mass and consistent mass for a P1 tetrahedral mesh.
    Element by element, vectorised over elements: the same formulas as
    p1_tet_element and conductivity_from_fibre applied to every element."""
    N = coords.shape[0]
    X = coords[tets]                                   # E x 4 x 3
    B = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)  # columns
    vol = np.abs(np.linalg.det(B)) / 6.0
    Binv = np.linalg.inv(B)                            # rows: gradients of lambda_1..3
    G = np.concatenate([-Binv.sum(axis=1, keepdims=True), Binv], axis=1)   # E x 4 x 3
    a = fibres / np.linalg.norm(fibres, axis=1)[:, None]
    aa = np.einsum("ei,ej->eij", a, a)
    D = sigma_l * aa + sigma_t * (np.eye(3)[None] - aa)
    Ke = vol[:, None, None] * np.einsum("eai,eij,ebj->eab", G, D, G)
    Me = (vol / 20.0)[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None]
    rows = np.repeat(tets, 4, axis=1).reshape(-1)
    cols = np.tile(tets, (1, 4)).reshape(-1)
    K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(N, N)).tocsr()
    M = sp.coo_matrix((Me.reshape(-1), (rows, cols)), shape=(N, N)).tocsr()
    ML = np.asarray(M.sum(axis=1)).reshape(-1)
    return K, ML, M
