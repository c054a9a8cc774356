"""Seeded ensemble of independent monodomain instances (batched workload).

Instance i (seed 1745, numpy default_rng):
  * size N_i = exp(U[ln 32k, ln 260k]); even i -> 2-D square-ish slab
    n0 x n1 with n0 n1 ~ N_i, odd i -> 3-D slab n0 x n1 x 11;
    spacing h = 0.1 mm;
  * sigma_l ~ U[0.1, 0.25] mS/mm, sigma_t = sigma_l * U[0.08, 0.2], fibres
    along x;
  * stimulus: the nodes within a 1.5 mm infinity-ball around a site drawn
    uniformly by length/area on the slab's outer boundary, 50/chi uA/mm^2
    for 2 ms;
  * TTP surrogate, chi = 140/mm, Cm = 0.01 uF/mm^2, dt = 0.05 ms, T = 20 ms.
Masks are built from integer indices as for the single workloads.
"""
import math

import numpy as np

H = 0.1


def _slab_dims(N, three_d):
    if three_d:
        a = N / 11.0
        n0 = max(8, int(round(math.sqrt(a * 1.6))))
        n1 = max(8, int(round(a / n0)))
        return (n0, n1, 11)
    n0 = max(16, int(round(math.sqrt(N * 1.25))))
    n1 = max(16, int(round(N / n0)))
    return (n0, n1)


def _boundary_site(rng, n):
    """A node index on the boundary of the box of node counts n, drawn
    uniformly over its faces (edges in 2-D) by measure."""
    d = len(n)
    ext = [(k - 1) * H for k in n]
    faces = []
    for ax in range(d):
        area = float(np.prod([ext[b] for b in range(d) if b != ax])) if d > 1 else 1.0
        faces += [(ax, 0, area), (ax, n[ax] - 1, area)]
    w = np.array([f[2] for f in faces])
    ax, side, _ = faces[rng.choice(len(faces), p=w / w.sum())]
    idx = [int(rng.integers(0, k)) for k in n]
    idx[ax] = side
    return idx


def _ball_mask(n, centre, width):
    km = int(math.floor(width / H + 1e-9))
    axes = [np.abs(np.arange(k) - c) <= km for k, c in zip(n, centre)]
    m = axes[0]
    for a in axes[1:]:
        m = np.logical_and.outer(a, m)
    return np.ascontiguousarray(m.reshape(-1)).astype(np.uint8)


def ensemble(n_inst=64, seed=1745, nmin=32_000, nmax=260_000):
    """List of instance dictionaries in the format of workloads.configs."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        N = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        n = _slab_dims(N, three_d=(i % 2 == 1))
        sl = rng.uniform(0.1, 0.25)
        st = sl * rng.uniform(0.08, 0.2)
        site = _boundary_site(rng, n)
        cfg = dict(name="c4_inst%02d" % i, kind="grid", dim=len(n), n=n, h=(H,) * len(n),
                   sigma=(sl, st, st), chi=140.0, Cm=0.01, model="TTP_SURR",
                   stim=dict(kind="mask", width=1.5, amp=50.0 / 140.0, t_on=0.0, t_off=2.0),
                   dt=0.05, T=20.0, precision="fp64")
        cfg["mask"] = _ball_mask(n, site, 1.5)
        out.append(cfg)
    return out


def small_ensemble(n_inst=6, seed=1745):
    """A few small instances (a few thousand nodes each) for parity tests."""
    return ensemble(n_inst, seed, nmin=1500, nmax=6000)
