"""CPU checks of the C ABI: the library loads, exports every declared
symbol, its structs match the header's layout, and its host-only paths
(coefficient tables, stage counts, argument validation) behave."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "emrkc.h")

E = pytest.importorskip("paper_2401_01745_amd.emrkc")
if not os.path.exists(E.LIB_PATH):
    pytest.skip("libemrkc.so not built", allow_module_level=True)


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(emrkc_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    L = E.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert n in E.EXPORTS, n
        assert callable(getattr(E, n, None)), n   # the binding has the same names


def test_accessors_on_null_context():
    assert E.emrkc_num_nodes(None) == -1
    assert E.emrkc_num_vars(None) == -1
    assert E.emrkc_ell_width(None) == -1
    assert E.emrkc_batch_size(None) < 0
    assert isinstance(E.emrkc_last_error(None), str)
    s, m, eta = E.emrkc_stage_counts_a(0.05, 51.0, 4.4)
    assert s == 1 and m >= 2 and eta > 0


def test_struct_layout_matches_header(tmp_path):
    """sizeof/offsetof of the ABI structs from a C compiler agree with the
    ctypes mirror used by the Python binding."""
    src = tmp_path / "probe.c"
    structs = {"emrkc_mesh": E.Mesh, "emrkc_conductivity": E.Conductivity, "emrkc_params": E.Params,
               "emrkc_state": E.State, "emrkc_stats": E.Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "emrkc.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.split("\n") if l)
    for cname, py in structs.items():
        assert int(out[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("s", [1, 2, 3, 7, 16, 63, 200])
def test_library_coefficients_against_closed_forms(s):
    """The library's FP64 tables against cosh/sinh closed forms of the
    Chebyshev polynomials (independent of the oracle)."""
    mu, nu, ka, c = E.emrkc_rkc_coeffs(s, 0.05)
    w0 = 1 + 0.05 / s ** 2
    th = math.acosh(w0)
    T = [math.cosh(j * th) for j in range(s + 1)]
    w1 = T[s] / (s * math.sinh(s * th) / math.sinh(th))
    assert mu[1] == pytest.approx(w1 / w0, rel=1e-13)
    for j in range(2, s + 1):
        assert mu[j] == pytest.approx(2 * w1 * T[j - 1] / T[j], rel=1e-12)
        assert nu[j] == pytest.approx(2 * w0 * T[j - 1] / T[j], rel=1e-12)
        assert ka[j] == pytest.approx(-T[j - 2] / T[j], rel=1e-12)
        assert nu[j] + ka[j] == pytest.approx(1.0, abs=1e-13)
    assert c[s] == pytest.approx(1.0, abs=1e-12)


def test_stage_counts_match_oracle():
    from oracle.emrkc import stage_counts
    rng = np.random.default_rng(3)
    for _ in range(500):
        dt = 10 ** rng.uniform(-3, 0.5)
        rF = 10 ** rng.uniform(-1, 5)
        rS = 10 ** rng.uniform(-2, 3)
        assert E.emrkc_stage_counts(dt, rF, rS) == stage_counts(dt, rF, rS)
        assert E.emrkc_stage_counts(dt, rF, rS, cond="A") == stage_counts(dt, rF, rS, cond="A")


def test_model_sizes():
    assert E.emrkc_model_num_vars("HH") == 4
    assert E.emrkc_model_num_vars("CRN_SURR") == 21
    assert E.emrkc_model_num_vars("TTP_SURR") == 19
    assert E.emrkc_model_num_gates("TTP_SURR") == 12
    assert E.emrkc_model_num_vars(99) == E.EMRKC_EINVAL


def test_invalid_arguments_rejected_before_any_gpu_call():
    L = E.lib()
    p = E.emrkc_default_params()
    cond = E.Conductivity(0.1, 0.1, 0.1)
    ctx = C.c_void_p()
    good = E.grid_mesh((5, 5), (0.1, 0.1))

    def create(mesh, cond, model, params):
        return L.emrkc_create(C.byref(mesh) if mesh is not None else None,
                              C.byref(cond) if cond is not None else None, model,
                              C.byref(params) if params is not None else None, C.byref(ctx))

    assert create(None, cond, 1, p) == E.EMRKC_EINVAL
    assert create(good, cond, 77, p) == E.EMRKC_EINVAL
    assert create(good, None, 1, p) == E.EMRKC_EINVAL
    bad = E.grid_mesh((1, 5), (0.1, 0.1))
    assert create(bad, cond, 1, p) == E.EMRKC_EINVAL
    bad = E.grid_mesh((5, 5), (0.1, -0.1))
    assert create(bad, cond, 1, p) == E.EMRKC_EINVAL
    q = E.emrkc_default_params()
    q.Cm = 0.0
    assert create(good, cond, 1, q) == E.EMRKC_EINVAL
    q = E.emrkc_default_params()
    q.precision = 7
    assert create(good, cond, 1, q) == E.EMRKC_EINVAL
    q = E.emrkc_default_params()
    q.powiter_max_iter = 0
    assert create(good, cond, 1, q) == E.EMRKC_EINVAL
    q = E.emrkc_default_params()
    q.rho_every = -1
    assert create(good, cond, 1, q) == E.EMRKC_EINVAL
    # assembled operators: arrays missing, or fewer than two nodes
    import numpy as np
    rp = np.array([0, 1, 2], np.int64)
    ci = np.array([1, 0], np.int32)
    va = np.array([1.0, 1.0])
    ml = np.array([1.0, 1.0])
    csr = E.csr_mesh(rp, ci, va, ml)
    for field in ("row_ptr", "col_idx", "values", "lumped_mass"):
        m = E.csr_mesh(rp, ci, va, ml)
        setattr(m, field, None)
        assert create(m, None, 3, p) == E.EMRKC_EINVAL
    m = E.csr_mesh(rp, ci, va, ml)
    m.n_nodes = 1
    assert create(m, None, 3, p) == E.EMRKC_EINVAL
    unknown = E.csr_mesh(rp, ci, va, ml)
    unknown.kind = 9
    assert create(unknown, None, 3, p) == E.EMRKC_EINVAL
    assert csr.kind == E.EMRKC_MESH_CSR
    assert ctx.value is None
    # node counts beyond 32-bit device indices, including products that
    # would wrap a 64-bit integer (2^22 * 2^21 * 2^21 = 2^64)
    for n in [(1 << 22, 1 << 21, 1 << 21), (1 << 30, 1 << 30, 1 << 30), (46341, 46341), (1 << 11, 1 << 10, 1 << 10)]:
        huge = E.grid_mesh(n, (0.1,) * len(n))
        assert create(huge, cond, 1, p) == E.EMRKC_EUNSUPPORTED, n
    assert ctx.value is None
    # ensembles: no condition-A stage counts, no periodic re-estimation
    meshes = (E.Mesh * 1)(good)
    conds = (E.Conductivity * 1)(cond)
    for field, value, code in [("flags", E.EMRKC_COND_A, E.EMRKC_EUNSUPPORTED),
                               ("rho_every", 5, E.EMRKC_EUNSUPPORTED)]:
        q = E.emrkc_default_params()
        setattr(q, field, value)
        ps = (E.Params * 1)(q)
        assert L.emrkc_create_batch(1, meshes, conds, 1, ps, C.byref(ctx)) == code
    # ensembles whose instances, or whose total, exceed 32-bit node indices
    ps = (E.Params * 3)(p, p, p)
    big = (E.Mesh * 1)(E.grid_mesh((1 << 22, 1 << 21, 1 << 21), (0.1, 0.1, 0.1)))
    assert L.emrkc_create_batch(1, big, conds, 1, ps, C.byref(ctx)) == E.EMRKC_EUNSUPPORTED
    third = E.grid_mesh((1 << 15, 1 << 15), (0.1, 0.1))  # 2^30 nodes each: three exceed 2^31 - 1
    three = (E.Mesh * 3)(third, third, third)
    assert L.emrkc_create_batch(3, three, (E.Conductivity * 3)(cond, cond, cond), 1, ps, C.byref(ctx)) == \
        E.EMRKC_EUNSUPPORTED
    assert ctx.value is None
    # calls on a null context
    assert L.emrkc_step(None, None, 0.1, 1) == E.EMRKC_EINVAL
    assert L.emrkc_step_noalloc(None, None, 0.1, 1) == E.EMRKC_EINVAL
    assert L.emrkc_set_rho(None, 1.0, 1.0) == E.EMRKC_EINVAL
    assert L.emrkc_num_nodes(None) == -1
    L.emrkc_destroy(None)
    # stage counts argument checks
    s = C.c_int()
    assert L.emrkc_stage_counts(-1.0, 1.0, 1.0, 0.05, C.byref(s), None, None) == E.EMRKC_EINVAL
    assert L.emrkc_stage_counts(0.1, float("nan"), 1.0, 0.05, C.byref(s), None, None) == E.EMRKC_EINVAL
    assert L.emrkc_stage_counts_a(-1.0, 1.0, 1.0, 0.05, C.byref(s), None, None) == E.EMRKC_EINVAL
    assert L.emrkc_rkc_coeffs(0, 0.05, None, None, None, None) == E.EMRKC_EINVAL
