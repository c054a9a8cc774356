"""ctypes binding of the C ABI in include/emrkc.h (argument marshalling only).

Every function here forwards to the function of the same name in
libemrkc.so; device buffers are torch tensors on the current HIP device and
streams are torch streams.  Importing this module fails loudly when the
library has not been built.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemrkc.so")

EMRKC_OK = 0
EMRKC_EINVAL = -1
EMRKC_ENOMEM = -2
EMRKC_EHIP = -3
EMRKC_ENONFINITE = -4
EMRKC_ENOCONV = -5
EMRKC_EUNSUPPORTED = -6
ERROR_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENONFINITE", -5: "ENOCONV",
               -6: "EUNSUPPORTED"}

EMRKC_MESH_Q1_GRID = 1
EMRKC_MESH_P1_TET = 2
EMRKC_MESH_CSR = 3
MODELS = {"HH": 1, "LINEAR": 2, "CRN_SURR": 3, "TTP_SURR": 4}
EMRKC_FP64 = 0
EMRKC_MIXED32 = 1
PRECISIONS = {"fp64": EMRKC_FP64, "mixed": EMRKC_MIXED32}
EMRKC_CHECK_FINITE = 1
EMRKC_PROGRESSIVE = 0x100  # progressive splitting of the auxiliary problem
METHODS = {"emrkc": 0, "mrkc": 1}
EMRKC_COND_A = 0x200       # stage counts from stability condition A
EMRKC_EAGER = 2          # diagnostic flag: no HIP-graph replay
EMRKC_FUSE = 4           # diagnostic flag: fused tail+head kernel
EMRKC_FLAT = 8           # diagnostic flag: flat (untiled) grid kernels
EMRKC_Z_PLANES = 0x400   # diagnostic flag: z stays in component planes while stepping
EMRKC_Z_BLOCKS = 0x800   # diagnostic flag: z in blocks of 256 nodes also for small z arrays


class Mesh(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("n", C.c_int64 * 3), ("h", C.c_double * 3),
                ("n_nodes", C.c_int64), ("n_elems", C.c_int64), ("coords", C.c_void_p),
                ("tets", C.c_void_p), ("fibres", C.c_void_p), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("values", C.c_void_p), ("lumped_mass", C.c_void_p)]


class Conductivity(C.Structure):
    _fields_ = [("sigma_l", C.c_double), ("sigma_t", C.c_double), ("sigma_n", C.c_double)]


class Params(C.Structure):
    _fields_ = [("chi", C.c_double), ("Cm", C.c_double), ("eps", C.c_double), ("rho_safety", C.c_double),
                ("precision", C.c_int32), ("flags", C.c_uint32), ("stim_mask", C.c_void_p),
                ("stim_amp", C.c_double), ("stim_t_on", C.c_double), ("stim_t_off", C.c_double),
                ("rho_F", C.c_double), ("rho_S", C.c_double), ("powiter_tol", C.c_double),
                ("powiter_eps", C.c_double), ("powiter_max_iter", C.c_int32), ("rho_every", C.c_int32),
                ("powiter_seed", C.c_uint64), ("linear_a", C.c_double), ("linear_lambda_E", C.c_double),
                ("method", C.c_int32), ("reserved1", C.c_int32)]


class State(C.Structure):
    _fields_ = [("t0", C.c_double), ("step", C.c_int64), ("t", C.c_double), ("V", C.c_void_p),
                ("z", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("s", C.c_int32), ("m", C.c_int32), ("eta", C.c_double), ("kernels_per_step", C.c_int64),
                ("used_graph", C.c_int32), ("z_blocks", C.c_int32)]


EXPORTS = {
    "emrkc_default_params": (None, [C.POINTER(Params)]),
    "emrkc_model_num_vars": (C.c_int, [C.c_int]),
    "emrkc_model_num_gates": (C.c_int, [C.c_int]),
    "emrkc_rkc_coeffs": (C.c_int, [C.c_int, C.c_double] + [C.POINTER(C.c_double)] * 4),
    "emrkc_stage_counts": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "emrkc_stage_counts_a": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "emrkc_eval_elementary": (C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "emrkc_eval_mrkc_terms": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_int, C.c_void_p]),
    "emrkc_exexrl_step": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_int64]),
    "emrkc_imexrl_step": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_int64]),
    "emrkc_imexrl_iterations": (C.c_int64, [C.c_void_p]),
    "emrkc_profile_imexrl": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_int64,
                                       C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "emrkc_autotune": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_int, C.POINTER(C.c_int)]),
    "emrkc_get_variants": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "emrkc_set_variants": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "emrkc_create": (C.c_int, [C.POINTER(Mesh), C.POINTER(Conductivity), C.c_int, C.POINTER(Params),
                               C.POINTER(C.c_void_p)]),
    "emrkc_destroy": (None, [C.c_void_p]),
    "emrkc_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "emrkc_num_nodes": (C.c_int64, [C.c_void_p]),
    "emrkc_num_vars": (C.c_int, [C.c_void_p]),
    "emrkc_ell_width": (C.c_int, [C.c_void_p]),
    "emrkc_last_error": (C.c_char_p, [C.c_void_p]),
    "emrkc_init_state": (C.c_int, [C.c_void_p, C.POINTER(State)]),
    "emrkc_estimate_rho": (C.c_int, [C.c_void_p, C.POINTER(State), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "emrkc_set_rho": (C.c_int, [C.c_void_p, C.c_double, C.c_double]),
    "emrkc_get_rho": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "emrkc_stages": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_double)]),
    "emrkc_step": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_int64]),
    "emrkc_step_noalloc": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_int64]),
    "emrkc_last_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "emrkc_profile_step": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_int64, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64)]),
    "emrkc_apply_diffusion": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "emrkc_create_batch": (C.c_int, [C.c_int, C.POINTER(Mesh), C.POINTER(Conductivity), C.c_int, C.POINTER(Params),
                                     C.POINTER(C.c_void_p)]),
    "emrkc_batch_size": (C.c_int, [C.c_void_p]),
    "emrkc_batch_info": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_int64), C.POINTER(C.c_int),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "emrkc_batch_set_rho": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "emrkc_eval_rhs_slow": (C.c_int, [C.c_void_p, C.POINTER(State), C.c_double, C.c_void_p]),
}

_lib = None


def lib():
    """The loaded libemrkc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libemrkc.so not found at %s: build it with "
                               "`python -m paper_2401_01745_amd.build`" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class EmrkcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, msg))
        self.code = code


def _check(rc, ctx=None):
    if rc != EMRKC_OK:
        msg = lib().emrkc_last_error(ctx).decode() if ctx else ""
        raise EmrkcError(rc, msg)
    return rc


# ---- thin wrappers with the ABI's names --------------------------------------
def emrkc_default_params():
    p = Params()
    lib().emrkc_default_params(C.byref(p))
    return p


def emrkc_model_num_vars(model):
    return lib().emrkc_model_num_vars(MODELS.get(model, model) if isinstance(model, str) else model)


def emrkc_model_num_gates(model):
    return lib().emrkc_model_num_gates(MODELS.get(model, model) if isinstance(model, str) else model)


def emrkc_rkc_coeffs(s, eps=0.05):
    arrs = [(C.c_double * (s + 1))() for _ in range(4)]
    _check(lib().emrkc_rkc_coeffs(s, eps, *arrs))
    return [list(a) for a in arrs]


def emrkc_stage_counts(dt, rho_F, rho_S, eps=0.05, cond="B"):
    s, m, eta = C.c_int(), C.c_int(), C.c_double()
    fn = lib().emrkc_stage_counts_a if cond == "A" else lib().emrkc_stage_counts
    _check(fn(dt, rho_F, rho_S, eps, C.byref(s), C.byref(m), C.byref(eta)))
    return s.value, m.value, eta.value


def emrkc_stage_counts_a(dt, rho_F, rho_S, eps=0.05):
    """(s, m, eta) under stability condition A."""
    return emrkc_stage_counts(dt, rho_F, rho_S, eps, cond="A")


def emrkc_num_nodes(ctx):
    return lib().emrkc_num_nodes(ctx)


def emrkc_num_vars(ctx):
    return lib().emrkc_num_vars(ctx)


def emrkc_ell_width(ctx):
    return lib().emrkc_ell_width(ctx)


def emrkc_batch_size(ctx):
    return lib().emrkc_batch_size(ctx)


def emrkc_last_error(ctx):
    """The context's last error message ('' when none)."""
    msg = lib().emrkc_last_error(ctx)
    return msg.decode() if msg else ""


ELEMENTARY = {"exp": 0, "expm1": 1, "log": 2}


def emrkc_eval_elementary(fn, x, precision="fp64", stream=None):
    """y = f(x) on the device as the kernels evaluate it (x: CUDA float64 tensor)."""
    import torch
    x = x.contiguous()
    if x.dtype != torch.float64 or not x.is_cuda:
        raise ValueError("x must be a CUDA float64 tensor")
    y = torch.empty_like(x)
    st = stream if stream is not None else torch.cuda.current_stream(x.device).cuda_stream
    _check(lib().emrkc_eval_elementary(ELEMENTARY[fn], PRECISIONS.get(precision, precision), x.data_ptr(),
                                       y.data_ptr(), x.numel(), st))
    return y


def emrkc_create(mesh, cond, model, params):
    ctx = C.c_void_p()
    rc = lib().emrkc_create(C.byref(mesh), C.byref(cond) if cond is not None else None,
                            MODELS.get(model, model) if isinstance(model, str) else model,
                            C.byref(params), C.byref(ctx))
    if rc != EMRKC_OK:
        raise EmrkcError(rc, "emrkc_create failed")
    return ctx


def emrkc_destroy(ctx):
    lib().emrkc_destroy(ctx)


def emrkc_set_stream(ctx, stream_ptr):
    _check(lib().emrkc_set_stream(ctx, C.c_void_p(stream_ptr)), ctx)


def emrkc_init_state(ctx, state):
    _check(lib().emrkc_init_state(ctx, C.byref(state)), ctx)


def emrkc_estimate_rho(ctx, state, allow_noconv=False):
    rf, rs, itf, its = C.c_double(), C.c_double(), C.c_int(), C.c_int()
    rc = lib().emrkc_estimate_rho(ctx, C.byref(state), C.byref(rf), C.byref(rs), C.byref(itf), C.byref(its))
    if rc != EMRKC_OK and not (allow_noconv and rc == EMRKC_ENOCONV):
        _check(rc, ctx)
    return rf.value, rs.value, itf.value, its.value, rc


def emrkc_set_rho(ctx, rho_F, rho_S):
    _check(lib().emrkc_set_rho(ctx, rho_F, rho_S), ctx)


def emrkc_get_rho(ctx):
    rf, rs = C.c_double(), C.c_double()
    _check(lib().emrkc_get_rho(ctx, C.byref(rf), C.byref(rs)), ctx)
    return rf.value, rs.value


def emrkc_stages(ctx, dt):
    s, m, eta = C.c_int(), C.c_int(), C.c_double()
    _check(lib().emrkc_stages(ctx, dt, C.byref(s), C.byref(m), C.byref(eta)), ctx)
    return s.value, m.value, eta.value


def emrkc_step(ctx, state, dt, nsteps):
    return _check(lib().emrkc_step(ctx, C.byref(state), dt, int(nsteps)), ctx)


def emrkc_step_noalloc(ctx, state, dt, nsteps):
    """emrkc_step with the work buffers in the library's static scratch
    array (allocates nothing)."""
    return _check(lib().emrkc_step_noalloc(ctx, C.byref(state), dt, int(nsteps)), ctx)


PROFILE_CLASSES = ("head", "inner", "fused")


def emrkc_profile_step(ctx, state, dt, nsteps):
    """{class: (mean ms, launches)} for the head, inner and fused kernels."""
    ms = (C.c_double * 3)()
    cnt = (C.c_int64 * 3)()
    _check(lib().emrkc_profile_step(ctx, C.byref(state), dt, int(nsteps), ms, cnt), ctx)
    return {k: (ms[i], cnt[i]) for i, k in enumerate(PROFILE_CLASSES)}


def emrkc_eval_mrkc_terms(ctx, state, t, which, out):
    """out (CUDA float64 tensor of n_v N entries) = f~_F (which 0) or f~_S (1)."""
    return _check(lib().emrkc_eval_mrkc_terms(ctx, C.byref(state), t, which, out.data_ptr()), ctx)


def emrkc_exexrl_step(ctx, state, dt, nsteps):
    return _check(lib().emrkc_exexrl_step(ctx, C.byref(state), dt, int(nsteps)), ctx)


def emrkc_imexrl_step(ctx, state, dt, nsteps):
    return _check(lib().emrkc_imexrl_step(ctx, C.byref(state), dt, int(nsteps)), ctx)


def emrkc_imexrl_iterations(ctx):
    return int(lib().emrkc_imexrl_iterations(ctx))


IMEXRL_KERNELS = ("pointwise", "cg_init", "cg_apply", "cg_update")


def emrkc_profile_imexrl(ctx, state, dt, nsteps):
    """Mean kernel durations (ms) and launch counts of IMEX-RL steps, by
    kernel class."""
    ms = (C.c_double * 4)()
    cnt = (C.c_int64 * 4)()
    _check(lib().emrkc_profile_imexrl(ctx, C.byref(state), dt, int(nsteps), ms, cnt), ctx)
    return {k: (ms[i], int(cnt[i])) for i, k in enumerate(IMEXRL_KERNELS)}


def emrkc_autotune(ctx, state, dt, reps=3):
    """Times the kernel shapes and keeps the fastest; returns the chosen
    (head, head planes, inner, inner planes, fused)."""
    v = (C.c_int * 5)()
    _check(lib().emrkc_autotune(ctx, C.byref(state), dt, int(reps), v), ctx)
    return tuple(v)


def emrkc_get_variants(ctx):
    v = (C.c_int * 5)()
    _check(lib().emrkc_get_variants(ctx, v), ctx)
    return tuple(v)


def emrkc_set_variants(ctx, variants):
    if len(variants) != 5:
        raise ValueError("variants has 5 entries")
    v = (C.c_int * 5)(*variants)
    _check(lib().emrkc_set_variants(ctx, v), ctx)


def emrkc_last_stats(ctx):
    st = Stats()
    _check(lib().emrkc_last_stats(ctx, C.byref(st)), ctx)
    return st


def emrkc_apply_diffusion(ctx, V, out):
    _check(lib().emrkc_apply_diffusion(ctx, C.c_void_p(V.data_ptr()), C.c_void_p(out.data_ptr())), ctx)


def emrkc_eval_rhs_slow(ctx, state, t, out):
    _check(lib().emrkc_eval_rhs_slow(ctx, C.byref(state), t, C.c_void_p(out.data_ptr())), ctx)


# ---- convenience: mesh/params structs from workload dictionaries -------------
def grid_mesh(n, h):
    m = Mesh()
    m.kind = EMRKC_MESH_Q1_GRID
    m.dim = len(n)
    for d in range(3):
        m.n[d] = int(n[d]) if d < len(n) else 1
        m.h[d] = float(h[d]) if d < len(n) else 1.0
    return m


def tet_mesh(coords, tets, fibres):
    """P1 mesh struct; the numpy arrays must stay alive during emrkc_create."""
    import numpy as np
    m = Mesh()
    m.kind = EMRKC_MESH_P1_TET
    m.dim = 3
    m.n_nodes = coords.shape[0]
    m.n_elems = tets.shape[0]
    assert coords.dtype == np.float64 and coords.flags.c_contiguous
    assert tets.dtype == np.int64 and tets.flags.c_contiguous
    assert fibres.dtype == np.float64 and fibres.flags.c_contiguous
    m.coords = coords.ctypes.data
    m.tets = tets.ctypes.data
    m.fibres = fibres.ctypes.data
    return m


def emrkc_create_batch(meshes, conds, model, params):
    n = len(meshes)
    M = (Mesh * n)(*meshes)
    Cd = (Conductivity * n)(*conds)
    P = (Params * n)(*params)
    ctx = C.c_void_p()
    rc = lib().emrkc_create_batch(n, M, Cd, MODELS.get(model, model) if isinstance(model, str) else model, P,
                                  C.byref(ctx))
    if rc != EMRKC_OK:
        raise EmrkcError(rc, "emrkc_create_batch failed")
    return ctx


def emrkc_batch_info(ctx, dt):
    n = lib().emrkc_batch_size(ctx)
    off = (C.c_int64 * (n + 1))()
    m = (C.c_int * n)()
    rf = (C.c_double * n)()
    rs = (C.c_double * n)()
    _check(lib().emrkc_batch_info(ctx, dt, off, m, rf, rs), ctx)
    return list(off), list(m), list(rf), list(rs)


def emrkc_batch_set_rho(ctx, rho_F, rho_S):
    n = len(rho_F)
    _check(lib().emrkc_batch_set_rho(ctx, (C.c_double * n)(*rho_F), (C.c_double * n)(*rho_S)), ctx)


class Simulation:
    """Owns one context and the caller-side state tensors (V, z) on the
    current HIP device.  All numerical work is done by the library."""

    def __init__(self, mesh, cond, model, params, keep=(), batch=None):
        import torch
        self._keep = keep
        if batch is not None:
            self.ctx = emrkc_create_batch(batch[0], batch[1], model, batch[2])
        else:
            self.ctx = emrkc_create(mesh, cond, model, params)
        self.N = lib().emrkc_num_nodes(self.ctx)
        self.nv = lib().emrkc_num_vars(self.ctx)
        zdt = torch.float32 if params.precision == EMRKC_MIXED32 else torch.float64
        self.V = torch.empty(self.N, dtype=torch.float64, device="cuda")
        self.z = torch.empty((self.nv - 1, self.N), dtype=zdt, device="cuda")
        self.state = State()
        self.state.t0 = 0.0
        self.state.step = 0
        self.state.t = 0.0
        self.state.V = self.V.data_ptr()
        self.state.z = self.z.data_ptr()

    def close(self):
        if self.ctx:
            emrkc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulation_from_config(cfg, precision=None, rho=None, flags=0, stim_mask=None, rho_every=0, method="emrkc",
                           **model_kw):
    """Simulation for a structured-grid workload dictionary (see the
    workloads package).  ``rho`` = (rho_F, rho_S) fixes the spectral radii;
    otherwise call ``estimate_rho``.  ``rho_every`` > 0 re-estimates them
    every that many steps."""
    import numpy as np
    from workloads.configs import stim_mask as make_mask
    prec = PRECISIONS[precision or cfg.get("precision", "fp64")]
    d = cfg["dim"]
    mesh = grid_mesh(cfg["n"][:d], cfg["h"][:d])
    sig = list(cfg["sigma"]) + [cfg["sigma"][-1]] * (3 - len(cfg["sigma"]))
    cond = Conductivity(sig[0], sig[1], sig[2])
    p = emrkc_default_params()
    p.chi = cfg["chi"]
    p.Cm = cfg["Cm"]
    p.precision = prec
    p.flags = flags
    mask = make_mask(cfg) if stim_mask is None else np.ascontiguousarray(stim_mask, dtype=np.uint8)
    p.stim_mask = mask.ctypes.data
    st = cfg["stim"]
    p.stim_amp = st["amp"]
    p.stim_t_on = st["t_on"]
    p.stim_t_off = st["t_off"]
    if rho is not None:
        p.rho_F, p.rho_S = rho
    p.rho_every = rho_every
    p.method = METHODS[method]
    p.linear_a = model_kw.get("a", 0.0)
    p.linear_lambda_E = model_kw.get("lam_E", 0.0)
    return Simulation(mesh, cond, cfg["model"], p, keep=(mask,))


def csr_mesh(row_ptr, col_idx, values, lumped_mass):
    """CSR mesh struct (A = -K and M_L given); the numpy arrays must stay
    alive during emrkc_create."""
    import numpy as np
    m = Mesh()
    m.kind = EMRKC_MESH_CSR
    m.n_nodes = lumped_mass.shape[0]
    assert row_ptr.dtype == np.int64 and col_idx.dtype == np.int32
    assert values.dtype == np.float64 and lumped_mass.dtype == np.float64
    for a in (row_ptr, col_idx, values, lumped_mass):
        assert a.flags.c_contiguous
    m.row_ptr = row_ptr.ctypes.data
    m.col_idx = col_idx.ctypes.data
    m.values = values.ctypes.data
    m.lumped_mass = lumped_mass.ctypes.data
    return m


def simulation_from_csr(A, ML, chi, Cm, model, stim_mask=None, stim=None, precision="fp64", rho=None, flags=0,
                        method="emrkc"):
    """Simulation for an assembled operator: A = -K (scipy sparse, any
    format) and the lumped mass ML; stim = dict(amp, t_on, t_off)."""
    import numpy as np
    Ac = A.tocsr()
    row_ptr = np.ascontiguousarray(Ac.indptr, dtype=np.int64)
    col_idx = np.ascontiguousarray(Ac.indices, dtype=np.int32)
    values = np.ascontiguousarray(Ac.data, dtype=np.float64)
    ml = np.ascontiguousarray(ML, dtype=np.float64)
    m = csr_mesh(row_ptr, col_idx, values, ml)
    p = emrkc_default_params()
    p.chi = chi
    p.Cm = Cm
    p.precision = PRECISIONS[precision]
    p.flags = flags
    keep = [row_ptr, col_idx, values, ml]
    if stim_mask is not None:
        mask = np.ascontiguousarray(stim_mask, dtype=np.uint8)
        p.stim_mask = mask.ctypes.data
        keep.append(mask)
        p.stim_amp, p.stim_t_on, p.stim_t_off = stim["amp"], stim["t_on"], stim["t_off"]
    if rho is not None:
        p.rho_F, p.rho_S = rho
    p.method = METHODS[method]
    return Simulation(m, None, model, p, keep=tuple(keep))


def simulation_from_tet_config(cfg, mesh, mask, precision=None, rho=None, flags=0, method="emrkc"):
    """Simulation for an unstructured P1 workload (see workloads.tetmesh)."""
    import numpy as np
    prec = PRECISIONS[precision or cfg.get("precision", "fp64")]
    coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
    tets = np.ascontiguousarray(mesh["tets"], dtype=np.int64)
    fib = np.ascontiguousarray(mesh["fibres"], dtype=np.float64)
    m = tet_mesh(coords, tets, fib)
    cond = Conductivity(cfg["sigma"][0], cfg["sigma"][1], cfg["sigma"][1])
    p = emrkc_default_params()
    p.chi = cfg["chi"]
    p.Cm = cfg["Cm"]
    p.precision = prec
    p.flags = flags
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    p.stim_mask = mask.ctypes.data
    st = cfg["stim"]
    p.stim_amp = st["amp"]
    p.stim_t_on = st["t_on"]
    p.stim_t_off = st["t_off"]
    if rho is not None:
        p.rho_F, p.rho_S = rho
    p.method = METHODS[method]
    return Simulation(m, cond, cfg["model"], p, keep=(coords, tets, fib, mask))


def simulation_from_batch(cfgs, precision=None, rho=None, flags=0):
    """One batched Simulation for a list of grid workload dictionaries with
    their own masks (see workloads.ensemble).  rho = (list of rho_F, list of
    rho_S) fixes per-instance radii."""
    import numpy as np
    meshes, conds, params, keep = [], [], [], []
    prec = PRECISIONS[precision or cfgs[0].get("precision", "fp64")]
    for k, cfg in enumerate(cfgs):
        d = cfg["dim"]
        meshes.append(grid_mesh(cfg["n"][:d], cfg["h"][:d]))
        sig = list(cfg["sigma"]) + [cfg["sigma"][-1]] * (3 - len(cfg["sigma"]))
        conds.append(Conductivity(sig[0], sig[1], sig[2]))
        p = emrkc_default_params()
        p.chi = cfg["chi"]
        p.Cm = cfg["Cm"]
        p.precision = prec
        p.flags = flags
        mask = np.ascontiguousarray(cfg["mask"], dtype=np.uint8)
        keep.append(mask)
        p.stim_mask = mask.ctypes.data
        st = cfg["stim"]
        p.stim_amp = st["amp"]
        p.stim_t_on = st["t_on"]
        p.stim_t_off = st["t_off"]
        if rho is not None:
            p.rho_F, p.rho_S = rho[0][k], rho[1][k]
        params.append(p)
    p0 = params[0]
    return Simulation(None, None, cfgs[0]["model"], p0, keep=tuple(keep), batch=(meshes, conds, params))
