"""Seeded unstructured P1 mesh of a truncated prolate-ellipsoidal shell
(stand-in for the paper's left-atrium mesh, which is not available).

The shell is described in index space (t, p, q): t transmural (endocardium
t = 0 to epicardium t = 1), p circumferential (periodic), q longitudinal
between two truncation angles.  Every index-space cell is split into the six
Kuhn tetrahedra along its main diagonal, a conforming triangulation with at
most 14 neighbours per node.  Interior nodes are jittered by
U[-0.1, 0.1] * h_local per coordinate (seeded); a tetrahedron with
non-positive volume halves the jitter and retries.  Fibres rotate in the
tangent plane from -60 degrees at the endocardium to +60 degrees at the
epicardium (rule-based helical fibres).

Node index: t + nt * (p + np * q) (t fastest), which keeps every
neighbour within nt * np of a node.  Only geometry and connectivity live
here; no assembly.
"""
import numpy as np


def shell_mesh(nt=19, npr=360, nq=150, r_endo=20.0, r_epi=28.0, c_endo=40.0, c_epi=48.0,
               q0=0.8, q1=2.34, jitter=0.1, seed=2401):
    """Returns dict(coords [N,3] float64, tets [E,4] int64, fibres [E,3],
    t [N] transmural coordinate, dims (nt, np, nq))."""
    T, P, Q = np.meshgrid(np.linspace(0.0, 1.0, nt), np.arange(npr) * (2 * np.pi / npr),
                          np.linspace(q0, q1, nq), indexing="ij")
    # flatten with t fastest
    t = T.reshape(-1, order="F")
    p = P.reshape(-1, order="F")
    q = Q.reshape(-1, order="F")
    a = r_endo + t * (r_epi - r_endo)
    c = c_endo + t * (c_epi - c_endo)
    coords = np.stack([a * np.sin(q) * np.cos(p), a * np.sin(q) * np.sin(p), c * np.cos(q)], axis=1)

    def nid(it, ip, iq):
        return it + nt * ((ip % npr) + npr * iq)

    it, ip, iq = np.meshgrid(np.arange(nt - 1), np.arange(npr), np.arange(nq - 1), indexing="ij")
    it, ip, iq = (v.reshape(-1, order="F") for v in (it, ip, iq))
    corner = lambda a_, b_, c_: nid(it + a_, ip + b_, iq + c_)
    v = [corner((k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1) for k in range(8)]
    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        cur = 0
        path = [0]
        for axis in perm:
            cur |= 1 << axis
            path.append(cur)
        tets.append(np.stack([v[k] for k in path], axis=1))
    tets = np.concatenate(tets, axis=0).astype(np.int64)

    # local spacing for the jitter: shortest distance to an index neighbour
    h_t = (r_epi - r_endo) / (nt - 1)
    h_p = a * np.sin(q) * (2 * np.pi / npr)
    h_q = np.sqrt((a * np.cos(q)) ** 2 + (c * np.sin(q)) ** 2) * (q1 - q0) / (nq - 1)
    h_loc = np.minimum(np.minimum(h_t, h_p), h_q)
    interior = (t > 0) & (t < 1) & (q > q0) & (q < q1)
    rng = np.random.default_rng(seed)
    disp = rng.uniform(-1.0, 1.0, size=coords.shape) * (jitter * h_loc)[:, None]
    disp[~interior] = 0.0
    scale = 1.0
    for _ in range(20):
        X = coords + scale * disp
        if min_volume(X, tets) > 0:
            coords = X
            break
        scale *= 0.5
    else:
        raise RuntimeError("jittered shell has inverted elements")

    # helical fibres at element centroids: angle -60 deg (endo) .. +60 deg (epi)
    tc = t[tets].mean(axis=1)
    pc = np.angle(np.exp(1j * p[tets]).mean(axis=1))
    qc = q[tets].mean(axis=1)
    ac = r_endo + tc * (r_epi - r_endo)
    cc = c_endo + tc * (c_epi - c_endo)
    e_p = np.stack([-np.sin(pc), np.cos(pc), np.zeros_like(pc)], axis=1)
    e_q = np.stack([ac * np.cos(qc) * np.cos(pc), ac * np.cos(qc) * np.sin(pc), -cc * np.sin(qc)], axis=1)
    e_q /= np.linalg.norm(e_q, axis=1)[:, None]
    ang = np.deg2rad(-60.0 + 120.0 * tc)
    fib = np.cos(ang)[:, None] * e_p + np.sin(ang)[:, None] * e_q
    fib /= np.linalg.norm(fib, axis=1)[:, None]
    return dict(coords=np.ascontiguousarray(coords), tets=np.ascontiguousarray(tets),
                fibres=np.ascontiguousarray(fib), t=t, dims=(nt, npr, nq))


def signed_volumes(X, tets):
    a = X[tets[:, 1]] - X[tets[:, 0]]
    b = X[tets[:, 2]] - X[tets[:, 0]]
    c = X[tets[:, 3]] - X[tets[:, 0]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def min_volume(X, tets):
    """Smallest signed volume relative to each element's orientation in index
    space (the Kuhn tetrahedra of one permutation share an orientation; odd
    permutations are mirrored).  Positive for a valid mesh."""
    v = signed_volumes(X, tets)
    E6 = tets.shape[0] // 6
    sign = np.repeat(np.array([1, -1, -1, 1, 1, -1], dtype=np.float64), E6)
    s = v * sign
    return float(s.min()) if s.sum() > 0 else float((-s).min())


def endo_patch_mask(mesh, radius=1.5, seed=2401):
    """uint8 mask: nodes within `radius` mm of a seeded endocardial node."""
    t = mesh["t"]
    endo = np.nonzero(t == 0.0)[0]
    rng = np.random.default_rng(seed + 1)
    centre = mesh["coords"][endo[rng.integers(len(endo))]]
    d = np.linalg.norm(mesh["coords"] - centre, axis=1)
    return (d <= radius).astype(np.uint8)


def shell_config(dims=(19, 360, 150), model="TTP_SURR", **kw):
    """Workload dictionary of the unstructured shell (dt 0.05 ms, T 100 ms,
    sigma of the cuboid workload, chi = 140/mm, Cm = 0.01 uF/mm^2)."""
    cfg = dict(name="c3_shell_%dx%dx%d" % dims, kind="tet", dims=tuple(dims), sigma=(0.17, 0.019),
               chi=140.0, Cm=0.01, model=model,
               stim=dict(kind="endo_patch", width=1.5, amp=50.0 / 140.0, t_on=0.0, t_off=2.0),
               dt=0.05, T=100.0, precision="fp64")
    cfg.update(kw)
    return cfg


def build_shell(cfg):
    nt, npr, nq = cfg["dims"]
    mesh = shell_mesh(nt, npr, nq)
    mask = endo_patch_mask(mesh, cfg["stim"]["width"])
    return mesh, mask


def small_shell_config(dims=(5, 48, 24), model="TTP_SURR", radius=4.0, **kw):
    """A coarse shell for parity tests (about 6k nodes); the stimulus ball is
    widened so that it covers several nodes of the coarse mesh."""
    cfg = shell_config(dims, model, **kw)
    cfg["stim"]["width"] = radius
    cfg["name"] = "c3_shell_small_%dx%dx%d" % tuple(dims)
    return cfg
