"""Nonlinear power iteration for spectral radii (appendix "Nonlinear power
iteration", Compute_Rho).  FP64 numpy.  Test infrastructure only.

Readings: the norm is the Euclidean norm over every component of the state;
delta = eps*||y|| falls back to eps when ||y|| = 0; the loop stops after
max_iter iterations even if the tolerance test has not been met (reported as
not converged); the caller multiplies the result by the safety factor.
The initial vector is the splitmix64 generator (Steele, Lea and Flood, 2014),
one 64-bit output per component index, mapped to [-1, 1).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(n, seed=0):
    """The i-th output (i = 0..n-1) of splitmix64 started at state ``seed``:
    state_i = seed + (i+1)*golden, then the published mixing function."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(n, dtype=np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def random_unit_interval(n, seed=0):
    """splitmix64 outputs mapped to [-1, 1): 2*(z >> 11)*2^-53 - 1."""
    z = splitmix64(n, seed)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def compute_rho(t, y, f, v, rho=0.0, tol=1e-2, eps=1e-8, max_iter=100):
    """Compute_Rho of the appendix.  Returns (v, rho, iterations, converged)."""
    ny = float(np.sqrt(np.dot(y, y)))
    nv = float(np.sqrt(np.dot(v, v)))
    delta = ny * eps if ny > 0.0 else eps
    q = delta / nv
    rho_old = 0.0
    fy = f(t, y)
    it = 0
    while abs(rho - rho_old) >= tol * rho:
        if it >= max_iter:
            return v, rho, it, False
        rho_old = rho
        v_old = v
        z = y + q * v_old
        v = f(t, z) - fy
        nv = float(np.sqrt(np.dot(v, v)))
        it += 1
        if nv == 0.0:
            return v, 0.0, it, True
        q = delta / nv
        rho = nv / delta
    return v, rho, it, True
