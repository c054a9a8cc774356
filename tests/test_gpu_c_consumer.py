"""The C ABI driven from a plain C11 program (gcc, HIP runtime API only: no
Python, no torch): it allocates the state with hipMalloc, creates a context
on a 3-D grid, runs emRKC steps and writes V back.  Its V must equal, bit for
bit, the run of the same workload through the Python binding."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from workloads.configs import small_config

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GCC = shutil.which("gcc")

PROGRAM = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <hip/hip_runtime_api.h>
#include "emrkc.h"

static int die(const char *what, int code) {
  fprintf(stderr, "%s failed (%d)\n", what, code);
  return 1;
}

/* n0 n1 n2 h chi Cm sigma_l sigma_t sigma_n model amp t_on t_off rho_F rho_S
 * dt nsteps precision mask_file out_file */
int main(int argc, char **argv) {
  if (argc != 21) return die("arguments", argc);
  const long long n0 = atoll(argv[1]), n1 = atoll(argv[2]), n2 = atoll(argv[3]);
  const long long N = n0 * n1 * n2;
  const double h = atof(argv[4]);
  if (hipSetDevice(0) != hipSuccess) return die("hipSetDevice", 0);

  emrkc_mesh mesh;
  memset(&mesh, 0, sizeof mesh);
  mesh.kind = EMRKC_MESH_Q1_GRID;
  mesh.dim = 3;
  mesh.n[0] = n0;
  mesh.n[1] = n1;
  mesh.n[2] = n2;
  mesh.h[0] = mesh.h[1] = mesh.h[2] = h;
  emrkc_conductivity cond = {atof(argv[7]), atof(argv[8]), atof(argv[9])};

  unsigned char *mask = malloc((size_t)N);
  FILE *f = fopen(argv[19], "rb");
  if (!mask || !f || fread(mask, 1, (size_t)N, f) != (size_t)N) return die("mask", 0);
  fclose(f);

  emrkc_params p;
  emrkc_default_params(&p);
  p.chi = atof(argv[5]);
  p.Cm = atof(argv[6]);
  p.stim_mask = mask;
  p.stim_amp = atof(argv[11]);
  p.stim_t_on = atof(argv[12]);
  p.stim_t_off = atof(argv[13]);
  p.rho_F = atof(argv[14]);
  p.rho_S = atof(argv[15]);
  p.precision = atoi(argv[18]);
  emrkc_ctx *ctx = NULL;
  int rc = emrkc_create(&mesh, &cond, atoi(argv[10]), &p, &ctx);
  if (rc != EMRKC_OK) return die("emrkc_create", rc);

  const int nv = emrkc_num_vars(ctx);
  const size_t zb = (size_t)(nv - 1) * (size_t)N * (p.precision == EMRKC_MIXED32 ? 4 : 8);
  void *V = NULL, *z = NULL;
  if (hipMalloc(&V, (size_t)N * 8) != hipSuccess || hipMalloc(&z, zb) != hipSuccess) return die("hipMalloc", 0);
  emrkc_state st;
  memset(&st, 0, sizeof st);
  st.V = V;
  st.z = z;
  if ((rc = emrkc_init_state(ctx, &st)) != EMRKC_OK) return die("emrkc_init_state", rc);
  if ((rc = emrkc_step(ctx, &st, atof(argv[16]), atoll(argv[17]))) != EMRKC_OK) return die("emrkc_step", rc);
  if (hipDeviceSynchronize() != hipSuccess) return die("hipDeviceSynchronize", 0);

  double *out = malloc((size_t)N * 8);
  if (!out || hipMemcpy(out, V, (size_t)N * 8, hipMemcpyDeviceToHost) != hipSuccess) return die("copy", 0);
  f = fopen(argv[20], "wb");
  if (!f || fwrite(out, 8, (size_t)N, f) != (size_t)N) return die("write", 0);
  fclose(f);
  printf("step %lld t %.6f\n", (long long)st.step, st.t);
  emrkc_destroy(ctx);
  (void)hipFree(V);
  (void)hipFree(z);
  free(out);
  free(mask);
  return 0;
}
"""


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


@pytest.fixture(scope="module")
def program(tmp_path_factory):
    if GCC is None:
        pytest.skip("gcc not available")
    from paper_2401_01745_amd import emrkc
    d = tmp_path_factory.mktemp("cabi")
    src, exe = d / "run.c", d / "run"
    src.write_text(PROGRAM)
    libdir = os.path.dirname(emrkc.LIB_PATH)
    cmd = [GCC, "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L", libdir, "-lemrkc",
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + libdir, "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c_program_equals_binding(E, program, tmp_path, precision):
    import torch
    from workloads.configs import stim_mask
    cfg = small_config("c2_3d_crn", (33, 21, 9))
    rho, dt, nsteps = (51.0, 4.4), cfg["dt"], 60
    mask = stim_mask(cfg)
    mfile, ofile = tmp_path / "mask.bin", tmp_path / "V.bin"
    mfile.write_bytes(np.ascontiguousarray(mask, dtype=np.uint8).tobytes())
    prec = E.PRECISIONS[precision]
    st = cfg["stim"]
    args = [str(program), *(str(x) for x in cfg["n"]), repr(cfg["h"][0]), repr(cfg["chi"]), repr(cfg["Cm"]),
            *(repr(x) for x in cfg["sigma"]), str(E.MODELS[cfg["model"]]), repr(st["amp"]), repr(st["t_on"]),
            repr(st["t_off"]), repr(rho[0]), repr(rho[1]), repr(dt), str(nsteps), str(prec), str(mfile), str(ofile)]
    assert len(set(cfg["h"])) == 1 and len(cfg["sigma"]) == 3
    print("c program:", precision, cfg["n"], nsteps, flush=True)
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    Vc = np.fromfile(ofile, dtype=np.float64)

    sim = E.simulation_from_config(cfg, precision=precision, rho=rho)
    E.emrkc_init_state(sim.ctx, sim.state)
    E.emrkc_step(sim.ctx, sim.state, dt, nsteps)
    torch.cuda.synchronize()
    Vp = sim.V.cpu().numpy().copy()
    sim.close()
    assert np.ptp(Vp) > 1.0  # the stimulus started a wave
    assert np.array_equal(Vc, Vp)
