"""IMEX-RL, the implicit-explicit Rush-Larsen step of the section "Numerical
experiments", and EXEX-RL, the same step with its implicit diffusion solve
replaced by an explicit update (the fine reference method of the error
measurements).  FP64 numpy.  Test infrastructure only.

EXEX-RL:
  z_E^{n+1} = z_E + (e^{dt Lambda_E(V_n)} - 1)(z_E - z_inf(V_n))
  z_S^{n+1} = z_S + dt g_S(V_n, z_E^{n+1}, z_S^n)
  V^{n+1}   = V_n + dt [ (chi Cm M_L)^{-1} A V_n
                          + Cm^{-1}(I_stim(t_n) - I_ion(V_n, z_E^{n+1}, z_S^{n+1})) ]
"""
import numpy as np


def exexrl_step(tn, y, dt, prob):
    V, zE, zS = prob.split(y)
    LE, zinf = prob.model.gates(V)
    zE1 = zE + np.expm1(dt * LE) * (zE - zinf)
    zS1 = zS + dt * prob.model.g_S(V, zE1, zS) if prob.nS else zS
    diff = (prob.A @ V) / (prob.chi * prob.Cm * prob.ML)
    I_ion = prob.Cm * prob.model.i_ion(V, zE1, zS1)
    V1 = V + dt * (diff + (prob.I_stim(tn) - I_ion) / prob.Cm)
    return np.concatenate([V1, zE1.reshape(-1), np.asarray(zS1).reshape(-1)])


def exexrl_run(prob, y0, t0, dt, nsteps):
    y = np.array(y0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        y = exexrl_step(t0 + n * dt, y, dt, prob)
    return y


def imexrl_matrix(dt, prob):
    """I - dt F with F = (chi Cm M_L)^{-1} A (sparse, CSC)."""
    import scipy.sparse as sp
    Fm = sp.diags(1.0 / (prob.chi * prob.Cm * prob.ML)) @ prob.A
    return (sp.identity(prob.N, format="csr") - dt * Fm).tocsc()


def imexrl_step(tn, y, dt, prob, solve=None):
    """IMEX-RL (algorithm "One step of the IMEX-RL method"): the gates and
    the other ionic variables as in EXEX-RL, then V^{n+1} from the linear
    system Cm M (V^{n+1} - V^n)/dt = chi^{-1} A V^{n+1} + M (I_stim(t_n) -
    I_ion(V^n, z^{n+1})), i.e. (I - dt F) V^{n+1} = V^n + dt S with the
    lumped mass, F = (chi Cm M_L)^{-1} A and S = Cm^{-1}(I_stim - I_ion);
    solved with a sparse direct solver (`solve`, a factorisation of
    I - dt F for this dt, else a fresh solve)."""
    import scipy.sparse.linalg as spla
    V, zE, zS = prob.split(y)
    LE, zinf = prob.model.gates(V)
    zE1 = zE + np.expm1(dt * LE) * (zE - zinf)
    zS1 = zS + dt * prob.model.g_S(V, zE1, zS) if prob.nS else zS
    I_ion = prob.Cm * prob.model.i_ion(V, zE1, zS1)
    rhs = V + dt * (prob.I_stim(tn) - I_ion) / prob.Cm
    V1 = solve(rhs) if solve is not None else spla.spsolve(imexrl_matrix(dt, prob), rhs)
    return np.concatenate([V1, zE1.reshape(-1), np.asarray(zS1).reshape(-1)])


def imexrl_cg_solver(dt, prob, rtol=1e-13):
    """A solve of (I - dt F) x = rhs by scipy's conjugate gradients on the
    equivalent symmetric positive definite system
    (M_L - dt (chi Cm)^{-1} A) x = M_L rhs, Jacobi preconditioned, started
    from zero (for meshes where a sparse LU is too slow)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    K = (sp.diags(prob.ML) - (dt / (prob.chi * prob.Cm)) * prob.A).tocsr()
    dinv = 1.0 / K.diagonal()
    M = spla.LinearOperator(K.shape, matvec=lambda v: dinv * v, dtype=np.float64)

    def solve(rhs):
        x, info = spla.cg(K, prob.ML * rhs, rtol=rtol, atol=0.0, M=M, maxiter=10000)
        if info != 0:
            raise RuntimeError("IMEX-RL CG did not converge (info=%d)" % info)
        return x
    return solve


def imexrl_run(prob, y0, t0, dt, nsteps):
    """nsteps IMEX-RL steps; I - dt F is factorised once (sparse LU)."""
    import scipy.sparse.linalg as spla
    solve = spla.splu(imexrl_matrix(dt, prob)).solve
    y = np.array(y0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        y = imexrl_step(t0 + n * dt, y, dt, prob, solve)
    return y
