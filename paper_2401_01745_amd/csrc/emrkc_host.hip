// Host runtime and C ABI of the emRKC library: argument validation, the
// RKC coefficient tables, stage selection, buffer planning for one emRKC
// step, HIP-graph replay of steps, and the power-iteration driver.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/emrkc.h"
#include "emrkc_internal.h"

using namespace emrkc;

#define EMRKC_EAGER_FLAG EMRKC_EAGER  // never capture graphs
#define EMRKC_FUSE_FLAG EMRKC_FUSE    // fused tail+head kernel (s == 1, m >= 2, grids)
#define EMRKC_FLAT_FLAG EMRKC_FLAT    // flat global-load kernels on grids

// Largest node count of a context: the kernels index nodes with 32-bit
// unsigned integers and form sums of an index and a plane stride.
constexpr int64_t kMaxNodes = ((int64_t)1 << 31) - 1;

struct GraphKey {
  int s, m, chunk;
  uint64_t dt_bits;
  const void *V, *z;
  bool operator<(const GraphKey &o) const {
    return std::tie(s, m, chunk, dt_bits, V, z) < std::tie(o.s, o.m, o.chunk, o.dt_bits, o.V, o.z);
  }
};

// Stage counts and coefficient tables of one emRKC step.
struct StepPlan {
  int s, m;
  double eta;
  std::vector<double> mu, nu, ka, cc;      // outer, index j
  std::vector<double> mui, nui, kai, cci;  // inner, index k
};

// emrkc_step_noalloc: largest stage counts (its plan arrays are sized when
// the context is created), and the static scratch array every context on a
// device shares for the step's work buffers.
constexpr int kNoAllocMaxStages = 1024;
constexpr size_t kScratchBytes = (size_t)64 << 20;

// One instance of a batched ensemble.
struct Inst {
  Mesh mesh;
  uint32_t off = 0, N = 0;
  double chi = 0, Cm = 0, amp = 0, t_on = 0, t_off = -1;
  double rho_F = 0, rho_S = 0;
  bool have_rho = false;
  bool warm_F = false, warm_S = false;
  int sel_F = 0, sel_S = 0;
  double raw_F = 0, raw_S = 0, nv_F = 0, nv_S = 0;
  int m = 0;  // inner stages of the current plan
};

// Device tables of the batched step for one (dt, radii): per parity of the
// step (V^n in X[n % 2]) one head launch over all instances and one launch
// per inner stage k = 2..m_max over the instances with m_i >= k.
struct BatchLaunch {
  BatchInst *tab = nullptr;
  uint16_t *map = nullptr;
  uint32_t nblocks = 0;
};
struct BatchDev {
  bool valid = false;
  uint64_t dt_bits = 0;
  const void *V = nullptr, *z = nullptr;  // state buffers the tables point into
  int shape = 0;                          // tile shape the tables were built for (+3: flat head)
  int s = 0, m_max = 0;
  double eta = 0;
  BatchLaunch head[2];
  std::vector<BatchLaunch> inner[2];
};

struct emrkc_ctx {
  // problem
  int mesh_kind = 0;
  int dim = 0;
  int64_t n[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int64_t N = 0;
  int model = 0, nv = 0, ng = 0, ns = 0;
  bool mixed = false;
  uint32_t flags = 0;
  double chi = 0, Cm = 0, eps = 0.05, safety = 1.05;
  double stim_amp = 0, t_on = 0, t_off = -1;
  ModelParams mp{0, 0};
  double pi_tol = 1e-2, pi_eps = 1e-8;
  int pi_max_iter = 100;
  uint64_t pi_seed = 0;
  // spectral radii (with safety) and warm-start data of the power iteration
  double rho_F = 0, rho_S = 0;
  bool have_rho = false;
  bool warm_F = false, warm_S = false;
  int sel_F = 0, sel_S = 0;
  double raw_F = 0, raw_S = 0, nv_F = 0, nv_S = 0;
  // batched ensembles (emrkc_create_batch)
  bool batch = false;
  std::vector<struct Inst> inst;
  BatchDev bdev;
  // device data
  Mesh mesh{};
  uint8_t *d_mask = nullptr;
  uint32_t *d_ell_col = nullptr;
  double *d_ell_w64 = nullptr;
  float *d_ell_w32 = nullptr;
  double *d_V1 = nullptr;
  double *d_U[3] = {nullptr, nullptr, nullptr};
  void *d_SV = nullptr;
  void *d_SV2 = nullptr;
  bool use_fused = false;
  bool flat = false;
  bool progressive = false;   // EMRKC_PROGRESSIVE
  bool cond_a = false;        // EMRKC_COND_A
  int rho_every = 0;          // params.rho_every
  int method = EMRKC_METHOD_EMRKC;
  int batch_shape = 0;        // tile shape of the batched kernels (0..2)
  bool batch_flat_head = true;   // batched head: flat kernel (measured faster) instead of the tiles
  int batch_march_zc = 0;        // > 0: inner stages of 3-D instances by z-marching columns of this many planes
  bool batch_pairs = false;      // inner stages with two tiles per block
  double *d_ML = nullptr;     // lumped mass (tets at creation, grids on first IMEX-RL step)
  double *d_cgq = nullptr;    // IMEX-RL: the conjugate gradient's B p
  double *d_Dsum = nullptr;   // IMEX-RL on tets: row sums of the operator's weights
  double grid_dsum = 0.0;     // IMEX-RL on grids: the same sum (one value for every node)
  int64_t cg_iters = 0;       // conjugate-gradient iterations of the last emrkc_imexrl_step
  int cg_guess = 0;           // iterations of the last solve (how many to enqueue ahead)
  double *d_cgp2 = nullptr;   // IMEX-RL: second direction buffer (directions alternate with d_V1)
  double *d_cgpart = nullptr; // IMEX-RL: partial sums
  CgScalars *d_cgs = nullptr; // the solver's device scalars, and a pinned host copy
  CgScalars *h_cgs = nullptr;
  // mRKC: gate-0 inner buffers, and full-state vectors of its power iteration
  double *d_W[2] = {nullptr, nullptr};
  double *d_Y = nullptr, *d_FY = nullptr, *d_Wv = nullptr, *d_FW = nullptr;
  double *d_mv[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  double *d_mpart = nullptr;
  bool m_warm[2] = {false, false};
  int m_sel[2] = {0, 0};
  double m_raw[2] = {0, 0}, m_nv[2] = {0, 0};
  int64_t last_est_step = -1; // state step of the last re-estimate by emrkc_step
  void *d_z1 = nullptr;
  // z in blocks of kZBlock nodes while emrkc_step runs the pointwise head
  // (allocated on first use; zb_run: the enqueued heads address it)
  void *d_zb = nullptr;
  bool zb_run = false;
  Clock *d_clock = nullptr;
  // emrkc_step_noalloc: the device the context was created on, the device
  // address of that device's scratch array (null if it could not be
  // resolved, with the reason in scratch_err), and plan arrays of
  // kNoAllocMaxStages + 1 entries (plus the work space of get_coeffs)
  int device = 0;
  unsigned char *scratch = nullptr;
  std::string scratch_err;
  StepPlan fixed_plan;
  std::vector<double> fixed_work;
  double *d_partials = nullptr;
  double *d_result = nullptr;
  int *d_flag = nullptr;
  double *d_vF[2] = {nullptr, nullptr};
  double *d_vS[2] = {nullptr, nullptr};
  double *d_zV = nullptr;
  // streams and graphs
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;
  std::map<GraphKey, hipGraphExec_t> graphs;
  emrkc_stats last{};
  std::string err;
};

static int fail(emrkc_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
static int fail(emrkc_ctx *c, int code, const char *fmt, ...) {
  if (c != nullptr) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIP_TRY(ctx, call)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail((ctx), EMRKC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));           \
  } while (0)

// ---------------------------------------------------------------------------
// Host-only helpers
// ---------------------------------------------------------------------------
extern "C" void emrkc_default_params(emrkc_params *p) {
  if (p == nullptr) return;
  memset(p, 0, sizeof *p);
  p->chi = 140.0;
  p->Cm = 0.01;
  p->eps = 0.05;
  p->rho_safety = 1.05;
  p->precision = EMRKC_FP64;
  p->stim_t_off = -1.0;
  p->powiter_tol = 1e-2;
  p->powiter_eps = 1e-8;
  p->powiter_max_iter = 100;
  p->powiter_seed = 0;
}

static int model_gates(int m) {
  switch (m) {
    case EMRKC_MODEL_HH: return 3;
    case EMRKC_MODEL_LINEAR: return 1;
    case EMRKC_MODEL_CRN_SURR: return 15;
    case EMRKC_MODEL_TTP_SURR: return 12;
    default: return -1;
  }
}
static int model_slow(int m) {
  switch (m) {
    case EMRKC_MODEL_HH: return 0;
    case EMRKC_MODEL_LINEAR: return 0;
    case EMRKC_MODEL_CRN_SURR: return 5;
    case EMRKC_MODEL_TTP_SURR: return 6;
    default: return -1;
  }
}

extern "C" int emrkc_model_num_vars(int m) {
  return model_gates(m) < 0 ? EMRKC_EINVAL : 1 + model_gates(m) + model_slow(m);
}
extern "C" int emrkc_model_num_gates(int m) { return model_gates(m) < 0 ? EMRKC_EINVAL : model_gates(m); }

// get_coeffs of the RKC algorithm with Chebyshev values by their
// three-term recurrences (T_j and T_j').  Every array holds s + 1 entries;
// mu, nu, kappa and c are overwritten (0 where the algorithm defines no
// value), T, dT and b are work space.
static void rkc_coeffs_into(int s, double eps, double *mu, double *nu, double *kappa, double *c, double *T,
                            double *dT, double *b) {
  for (int j = 0; j <= s; ++j) mu[j] = nu[j] = kappa[j] = c[j] = 0.0;
  const double w0 = 1.0 + eps / ((double)s * (double)s);
  T[0] = 1.0;
  dT[0] = 0.0;
  if (s >= 1) {
    T[1] = w0;
    dT[1] = 1.0;
  }
  for (int j = 2; j <= s; ++j) {
    T[j] = 2.0 * w0 * T[j - 1] - T[j - 2];
    dT[j] = 2.0 * T[j - 1] + 2.0 * w0 * dT[j - 1] - dT[j - 2];
  }
  const double w1 = T[s] / dT[s];
  for (int j = 0; j <= s; ++j) b[j] = 1.0 / T[j];
  mu[1] = w1 / w0;
  c[1] = mu[1];
  for (int j = 2; j <= s; ++j) {
    mu[j] = 2.0 * w1 * b[j] / b[j - 1];
    nu[j] = 2.0 * w0 * b[j] / b[j - 1];
    kappa[j] = -b[j] / b[j - 2];
    c[j] = nu[j] * c[j - 1] + kappa[j] * c[j - 2] + mu[j];
  }
}

static void rkc_coeffs(int s, double eps, std::vector<double> &mu, std::vector<double> &nu,
                       std::vector<double> &kappa, std::vector<double> &c) {
  mu.resize(s + 1);
  nu.resize(s + 1);
  kappa.resize(s + 1);
  c.resize(s + 1);
  std::vector<double> work(3 * (size_t)(s + 1));
  rkc_coeffs_into(s, eps, mu.data(), nu.data(), kappa.data(), c.data(), work.data(), work.data() + (s + 1),
                  work.data() + 2 * (s + 1));
}

extern "C" int emrkc_rkc_coeffs(int s, double eps, double *mu, double *nu, double *kappa, double *c) {
  if (s < 1 || s > 10000 || !(eps > 0) || !mu || !nu || !kappa || !c) return EMRKC_EINVAL;
  std::vector<double> a, b, k, cc;
  rkc_coeffs(s, eps, a, b, k, cc);
  for (int j = 0; j <= s; ++j) {
    mu[j] = a[j];
    nu[j] = b[j];
    kappa[j] = k[j];
    c[j] = cc[j];
  }
  return EMRKC_OK;
}

// get_stages: s = max(1, ceil(sqrt(dt rho / beta))), l_s = beta s^2.
static int get_stages(double dt, double rho, double eps, double *ls) {
  const double beta = 2.0 - 4.0 * eps / 3.0;
  double s = ceil(sqrt(dt * rho / beta));
  if (!(s >= 1.0)) s = 1.0;
  if (s > 1e6) s = 1e6;
  *ls = beta * s * s;
  return (int)s;
}

extern "C" int emrkc_stage_counts_a(double dt, double rho_F, double rho_S, double eps, int *s, int *m,
                                    double *eta) {
  if (!(dt > 0) || !(rho_F >= 0) || !(rho_S >= 0) || !(eps > 0) || !isfinite(dt) || !isfinite(rho_F) ||
      !isfinite(rho_S))
    return EMRKC_EINVAL;
  double ls;
  const int ss = get_stages(dt, rho_S, eps, &ls);
  const double beta = 2.0 - 4.0 * eps / 3.0;
  // eta(m) decreases and beta m^2 grows with m: search upwards from 2
  int mm = 2;
  double e = 0;
  for (;; ++mm) {
    if (mm > 10000) return EMRKC_EUNSUPPORTED;
    const double m2 = (double)mm * (double)mm;
    e = (6.0 * dt / ls) * (m2 / (m2 - 1.0));
    if (e * rho_F <= beta * m2) break;
  }
  if (ss > 10000) return EMRKC_EUNSUPPORTED;
  if (s) *s = ss;
  if (m) *m = mm;
  if (eta) *eta = e;
  return EMRKC_OK;
}

extern "C" int emrkc_stage_counts(double dt, double rho_F, double rho_S, double eps, int *s, int *m, double *eta) {
  if (!(dt > 0) || !(rho_F >= 0) || !(rho_S >= 0) || !(eps > 0) || !isfinite(dt) || !isfinite(rho_F) ||
      !isfinite(rho_S))
    return EMRKC_EINVAL;
  double ls, lm;
  const int ss = get_stages(dt, rho_S, eps, &ls);
  const double e = 2.0 * dt / ls;
  const int mm = get_stages(e, rho_F, eps, &lm);
  if (ss > 10000 || mm > 10000) return EMRKC_EUNSUPPORTED;
  if (s) *s = ss;
  if (m) *m = mm;
  if (eta) *eta = e;
  return EMRKC_OK;
}

extern "C" int emrkc_eval_elementary(int fn, int precision, const double *x, double *y, int64_t n,
                                     void *hip_stream) {
  if (fn < 0 || fn > 2 || (precision != EMRKC_FP64 && precision != EMRKC_MIXED32) || n < 0 ||
      n > (int64_t)UINT32_MAX - 1024 || (n > 0 && (!x || !y)))
    return EMRKC_EINVAL;
  if (n == 0) return EMRKC_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  if (launch_elementary(fn, precision == EMRKC_MIXED32, x, y, (uint32_t)n, st) != hipSuccess) return EMRKC_EHIP;
  return hipStreamSynchronize(st) == hipSuccess ? EMRKC_OK : EMRKC_EHIP;
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
static FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t b = 0;
  while ((1ull << b) < d) ++b;
  f.shift = 31 + b;
  const unsigned __int128 one = 1;
  f.mult = (uint64_t)(((one << f.shift) + d - 1) / d);
  return f;
}

// Weights of (chi Cm M_L)^{-1} A on neighbour differences of the lumped Q1
// operator: sum_d sigma_d L_d(o_d) prod_{e != d} Mh(o_e) with
// L(+-1) = -1/h^2, L(0) = 2/h^2, Mh(+-1) = 1/6, Mh(0) = 2/3, negated and
// divided by chi Cm.
static void grid_weights(int dim, const double *h, const double *sig, double chiCm, double *w) {
  auto L = [&](int d, int o) { return o ? -1.0 / (h[d] * h[d]) : 2.0 / (h[d] * h[d]); };
  auto Mh = [](int o) { return o ? 1.0 / 6.0 : 2.0 / 3.0; };
  auto G = [&](int ox, int oy, int oz) {
    int o[3] = {ox, oy, oz};
    double g = 0.0;
    for (int d = 0; d < dim; ++d) {
      double p = sig[d] * L(d, o[d]);
      for (int e = 0; e < dim; ++e)
        if (e != d) p *= Mh(o[e]);
      g += p;
    }
    return -g / chiCm;
  };
  for (int k = 0; k < 8; ++k) w[k] = 0.0;
  w[0] = G(1, 0, 0);
  w[1] = G(0, 1, 0);
  w[3] = G(1, 1, 0);
  if (dim == 3) {
    w[2] = G(0, 0, 1);
    w[4] = G(1, 0, 1);
    w[5] = G(0, 1, 1);
    w[6] = G(1, 1, 1);
    // the weight of one neighbouring plane's centre difference in the
    // plane-by-plane form of the 3-D stencil
    w[7] = w[2] + 2.0 * (w[4] + w[5]) + 4.0 * w[6];
  }
}

static void free_batch_tables(emrkc_ctx *c) {
  auto rel = [](BatchLaunch &b) {
    if (b.tab) (void)hipFree(b.tab);
    if (b.map) (void)hipFree(b.map);
    b = BatchLaunch{};
  };
  for (int p = 0; p < 2; ++p) {
    rel(c->bdev.head[p]);
    for (auto &b : c->bdev.inner[p]) rel(b);
    c->bdev.inner[p].clear();
  }
  c->bdev.valid = false;
}

static void clear_graphs(emrkc_ctx *c) {
  for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

static void free_ctx(emrkc_ctx *c) {
  if (c->batch) {
    (void)hipDeviceSynchronize();
    free_batch_tables(c);
  }
  for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  void *ptrs[] = {c->d_mask, c->d_ell_col, c->d_ell_w64, c->d_ell_w32, c->d_V1, c->d_U[0], c->d_U[1],
                  c->d_U[2], c->d_SV, c->d_SV2,   c->d_z1,      c->d_zb,      c->d_clock,   c->d_partials, c->d_result, c->d_flag,
                  c->d_vF[0], c->d_vF[1], c->d_vS[0], c->d_vS[1], c->d_zV,
                  c->d_W[0], c->d_W[1], c->d_Y, c->d_FY, c->d_Wv, c->d_FW,
                  c->d_mv[0][0], c->d_mv[0][1], c->d_mv[1][0], c->d_mv[1][1], c->d_mpart, c->d_ML, c->d_cgq, c->d_Dsum, c->d_cgs, c->d_cgp2, c->d_cgpart};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_cgs) (void)hipHostFree(c->h_cgs);
  if (c->capture) (void)hipStreamDestroy(c->capture);
}

static int dalloc(emrkc_ctx *c, void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, e == hipErrorOutOfMemory ? EMRKC_ENOMEM : EMRKC_EHIP, "hipMalloc(%zu) failed: %s", bytes,
                hipGetErrorString(e));
  }
  return EMRKC_OK;
}

static int build_p1(emrkc_ctx *c, const emrkc_mesh *mesh, const emrkc_conductivity *cond);
static int build_csr(emrkc_ctx *c, const emrkc_mesh *mesh);

// Work buffers of emrkc_step_noalloc: one array per device, in the code
// object's zero-initialised device data, so that the call allocates
// nothing.  The name `scratch` is only a host-side handle: host code
// resolves the array's device address once per device (with that device
// current, when the first context on it is created) and passes that
// address to kernels, never the symbol itself.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_addr[kMaxDevices];

// Device address of device dev's scratch array (dev must be current), or
// null with the reason in *why.
static unsigned char *scratch_address(int dev, std::string *why) {
  if (dev < 0 || dev >= kMaxDevices) {
    *why = "device index out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[dev] == nullptr) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      *why = std::string("hipGetSymbolAddress failed: ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_addr[dev] = (unsigned char *)p;
  }
  return g_scratch_addr[dev];
}

// Sets up what emrkc_step_noalloc needs of a single context: its device,
// that device's scratch address and plan arrays for kNoAllocMaxStages.
static int setup_noalloc(emrkc_ctx *c) {
  HIP_TRY(c, hipGetDevice(&c->device));
  c->scratch = scratch_address(c->device, &c->scratch_err);
  StepPlan &P = c->fixed_plan;
  for (std::vector<double> *v : {&P.mu, &P.nu, &P.ka, &P.cc, &P.mui, &P.nui, &P.kai, &P.cci})
    v->assign(kNoAllocMaxStages + 1, 0.0);
  c->fixed_work.assign(3 * (size_t)(kNoAllocMaxStages + 1), 0.0);
  return EMRKC_OK;
}

extern "C" int emrkc_create(const emrkc_mesh *mesh, const emrkc_conductivity *cond, int ionic_model,
                            const emrkc_params *p, emrkc_ctx **out) {
  if (out == nullptr) return EMRKC_EINVAL;
  *out = nullptr;
  if (mesh == nullptr || p == nullptr) return EMRKC_EINVAL;
  if (model_gates(ionic_model) < 0) return EMRKC_EINVAL;
  if (!(p->chi > 0) || !(p->Cm > 0) || !isfinite(p->chi) || !isfinite(p->Cm)) return EMRKC_EINVAL;
  if (!(p->eps > 0) || !(p->eps < 1) || !(p->rho_safety >= 1.0)) return EMRKC_EINVAL;
  if (p->precision != EMRKC_FP64 && p->precision != EMRKC_MIXED32) return EMRKC_EINVAL;
  if (!(p->powiter_tol > 0) || !(p->powiter_eps > 0) || p->powiter_max_iter < 1) return EMRKC_EINVAL;
  if (p->rho_every < 0) return EMRKC_EINVAL;
  if (p->method != EMRKC_METHOD_EMRKC && p->method != EMRKC_METHOD_MRKC) return EMRKC_EINVAL;
  if (p->method == EMRKC_METHOD_MRKC && p->precision != EMRKC_FP64) return EMRKC_EUNSUPPORTED;
  if (!isfinite(p->stim_amp) || !isfinite(p->stim_t_on) || !isfinite(p->stim_t_off)) return EMRKC_EINVAL;
  if (!isfinite(p->rho_F) || !isfinite(p->rho_S)) return EMRKC_EINVAL;
  if (ionic_model == EMRKC_MODEL_LINEAR && (!isfinite(p->linear_a) || !isfinite(p->linear_lambda_E) ||
                                            p->linear_lambda_E > 0))
    return EMRKC_EINVAL;

  int64_t N = 0;
  if (mesh->kind == EMRKC_MESH_Q1_GRID) {
    if (cond == nullptr) return EMRKC_EINVAL;
    if (mesh->dim != 2 && mesh->dim != 3) return EMRKC_EINVAL;
    N = 1;
    for (int d = 0; d < mesh->dim; ++d) {
      if (mesh->n[d] < 2 || mesh->n[d] > (1 << 30) || !(mesh->h[d] > 0) || !isfinite(mesh->h[d]))
        return EMRKC_EINVAL;
      // 32-bit node indices on the device; checked before the product so
      // that it cannot overflow
      if (mesh->n[d] > kMaxNodes / N) return EMRKC_EUNSUPPORTED;
      N *= mesh->n[d];
    }
    const double sg[3] = {cond->sigma_l, cond->sigma_t, cond->sigma_n};
    for (int d = 0; d < mesh->dim; ++d)
      if (!(sg[d] >= 0) || !isfinite(sg[d])) return EMRKC_EINVAL;
  } else if (mesh->kind == EMRKC_MESH_P1_TET) {
    if (cond == nullptr || mesh->n_nodes < 4 || mesh->n_elems < 1 || !mesh->coords || !mesh->tets || !mesh->fibres)
      return EMRKC_EINVAL;
    if (!(cond->sigma_l >= 0) || !(cond->sigma_t >= 0) || !isfinite(cond->sigma_l) || !isfinite(cond->sigma_t))
      return EMRKC_EINVAL;
    N = mesh->n_nodes;
  } else if (mesh->kind == EMRKC_MESH_CSR) {
    if (mesh->n_nodes < 2 || !mesh->row_ptr || !mesh->col_idx || !mesh->values || !mesh->lumped_mass)
      return EMRKC_EINVAL;
    N = mesh->n_nodes;
  } else {
    return EMRKC_EINVAL;
  }
  if (N > kMaxNodes) return EMRKC_EUNSUPPORTED;  // 32-bit node indices on the device

  emrkc_ctx *c = new (std::nothrow) emrkc_ctx();
  if (c == nullptr) return EMRKC_ENOMEM;
  c->mesh_kind = mesh->kind;
  c->N = N;
  c->model = ionic_model;
  c->ng = model_gates(ionic_model);
  c->ns = model_slow(ionic_model);
  c->nv = 1 + c->ng + c->ns;
  c->mixed = p->precision == EMRKC_MIXED32;
  c->flags = p->flags;
  c->use_fused = getenv("EMRKC_FUSE") != nullptr || (p->flags & EMRKC_FUSE_FLAG) != 0;
  c->flat = (p->flags & EMRKC_FLAT_FLAG) != 0;
  c->progressive = (p->flags & EMRKC_PROGRESSIVE) != 0;
  c->cond_a = (p->flags & EMRKC_COND_A) != 0;
  c->rho_every = p->rho_every;
  c->method = p->method;
  c->chi = p->chi;
  c->Cm = p->Cm;
  c->eps = p->eps;
  c->safety = p->rho_safety;
  c->stim_amp = p->stim_amp;
  c->t_on = p->stim_t_on;
  c->t_off = p->stim_t_off;
  c->mp.lin_a = p->linear_a;
  c->mp.lin_lamE = p->linear_lambda_E;
  c->pi_tol = p->powiter_tol;
  c->pi_eps = p->powiter_eps;
  c->pi_max_iter = p->powiter_max_iter;
  c->pi_seed = p->powiter_seed;
  if (p->rho_F > 0 && p->rho_S > 0) {
    c->rho_F = p->rho_F;
    c->rho_S = p->rho_S;
    c->have_rho = true;
  }

  int rc = EMRKC_OK;
  const uint32_t Nu = (uint32_t)N;
  if (mesh->kind == EMRKC_MESH_Q1_GRID) {
    c->dim = mesh->dim;
    for (int d = 0; d < 3; ++d) {
      c->n[d] = d < mesh->dim ? mesh->n[d] : 1;
      c->h[d] = d < mesh->dim ? mesh->h[d] : 1.0;
    }
    Mesh &M = c->mesh;
    M.kind = kGrid;
    Grid &g = M.grid;
    g.n0 = (uint32_t)c->n[0];
    g.n1 = (uint32_t)c->n[1];
    g.n2 = (uint32_t)c->n[2];
    g.N = Nu;
    g.dim = c->dim;
    g.div0 = make_fastdiv(g.n0);
    g.div1 = make_fastdiv(g.n1);
    const double sg[3] = {cond->sigma_l, cond->sigma_t, cond->sigma_n};
    grid_weights(c->dim, c->h, sg, c->chi * c->Cm, g.w);
    // default inner-stage kernel: z-marching columns on 3-D grids, with the
    // number of planes per block chosen for at least ~4 blocks per CU
    {
      const uint32_t cols = ((g.n0 + 31) / 32) * ((g.n1 + 7) / 8);
      uint32_t zc = 16;
      while (zc > 1 && cols * ((g.n2 + zc - 1) / zc) < 2048) zc /= 2;
      g.zc = zc;
      // short columns re-read too much halo: small grids keep 3-D tiles
      g.inner_variant = (c->dim == 3 && zc >= 4) ? 1 : 0;
      // head: the flat kernel on 3-D grids (measured fastest on the 442k- and
      // 36M-node slabs), 2-D tiles otherwise (emrkc_autotune refines both)
      g.head_variant = c->dim == 3 ? 5 : 0;
      g.head_zc = g.zc;
    }
  } else if (mesh->kind == EMRKC_MESH_P1_TET) {
    rc = build_p1(c, mesh, cond);
    if (rc != EMRKC_OK) goto error;
  } else {
    rc = build_csr(c, mesh);
    if (rc != EMRKC_OK) goto error;
  }
  c->mesh.flat = c->flat ? 1 : 0;

  {
    const size_t vb = sizeof(double) * (size_t)N;
    const size_t svb = (c->mixed ? sizeof(float) : sizeof(double)) * (size_t)N;
    if ((rc = dalloc(c, (void **)&c->d_V1, vb)) || (rc = dalloc(c, (void **)&c->d_U[0], vb)) ||
        (rc = dalloc(c, (void **)&c->d_U[1], vb)) || (rc = dalloc(c, (void **)&c->d_U[2], vb)) ||
        (rc = dalloc(c, &c->d_SV, svb)) || (rc = dalloc(c, &c->d_SV2, svb)) ||
        (rc = dalloc(c, (void **)&c->d_clock, sizeof(Clock))) ||
        (rc = dalloc(c, (void **)&c->d_result, 2 * sizeof(double))) ||
        (rc = dalloc(c, (void **)&c->d_flag, sizeof(int))))
      goto error;
    const size_t nparts = std::max<size_t>(reduce_blocks(Nu), 65536);
    if ((rc = dalloc(c, (void **)&c->d_partials, nparts * sizeof(double)))) goto error;
    if (p->stim_mask != nullptr) {
      if ((rc = dalloc(c, (void **)&c->d_mask, (size_t)N))) goto error;
      hipError_t e = hipMemcpy(c->d_mask, p->stim_mask, (size_t)N, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        rc = fail(c, EMRKC_EHIP, "mask upload failed: %s", hipGetErrorString(e));
        goto error;
      }
    }
    hipError_t e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
      rc = fail(c, EMRKC_EHIP, "hipStreamCreate failed: %s", hipGetErrorString(e));
      goto error;
    }
    e = hipMemset(c->d_clock, 0, sizeof(Clock));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      rc = fail(c, EMRKC_EHIP, "initialisation failed: %s", hipGetErrorString(e));
      goto error;
    }
  }
  if ((rc = setup_noalloc(c)) != EMRKC_OK) goto error;
  *out = c;
  return EMRKC_OK;
error:
  free_ctx(c);
  delete c;
  return rc;
}

extern "C" void emrkc_destroy(emrkc_ctx *c) {
  if (c == nullptr) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  (void)hipDeviceSynchronize();
  free_ctx(c);
  delete c;
}

extern "C" int emrkc_set_stream(emrkc_ctx *c, void *s) {
  if (c == nullptr) return EMRKC_EINVAL;
  c->stream = (hipStream_t)s;
  return EMRKC_OK;
}

extern "C" int64_t emrkc_num_nodes(const emrkc_ctx *c) { return c ? c->N : -1; }
extern "C" int emrkc_num_vars(const emrkc_ctx *c) { return c ? c->nv : -1; }
extern "C" int emrkc_ell_width(const emrkc_ctx *c) {
  return c ? (c->mesh.kind == kEll ? (int)c->mesh.ell.width : 0) : -1;
}
extern "C" const char *emrkc_last_error(const emrkc_ctx *c) { return c ? c->err.c_str() : "null context"; }

static bool state_ok(const emrkc_ctx *c, const emrkc_state *s) {
  return s != nullptr && s->V != nullptr && s->z != nullptr && s->V != s->z;
}

static StimArgs stim_args(const emrkc_ctx *c) {
  StimArgs s;
  s.mask = c->d_mask;
  s.amp = c->stim_amp;
  s.t_on = c->t_on;
  s.t_off = c->t_off;
  return s;
}

static double state_time(double t0, int64_t step, double dt) {
#pragma clang fp contract(off)
  return t0 + (double)step * dt;
}

// The clock of a state is t0 + step*dt, and every stepping call writes
// t = t0 + step*dt on return.  A state advanced with one step size and then
// stepped with another no longer satisfies t == t0 + step*dt for the new
// dt: move t0 so that the clock continues from t (step keeps counting).
static void rebase_clock(emrkc_state *st, double dt) {
#pragma clang fp contract(off)
  if (st->step != 0 && state_time(st->t0, st->step, dt) != st->t) st->t0 = st->t - (double)st->step * dt;
}

extern "C" int emrkc_init_state(emrkc_ctx *c, emrkc_state *s) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, s)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  HIP_TRY(c, launch_init_state(c->model, c->mixed, (uint32_t)c->N, (double *)s->V, s->z, c->mp, c->stream));
  s->step = 0;
  s->t = s->t0;
  return EMRKC_OK;
}

extern "C" int emrkc_set_rho(emrkc_ctx *c, double rho_F, double rho_S) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!(rho_F >= 0) || !(rho_S >= 0) || !isfinite(rho_F) || !isfinite(rho_S))
    return fail(c, EMRKC_EINVAL, "invalid spectral radii");
  c->rho_F = rho_F;
  c->rho_S = rho_S;
  c->have_rho = true;
  for (auto &I : c->inst) {
    I.rho_F = rho_F;
    I.rho_S = rho_S;
  }
  if (c->batch) {
    clear_graphs(c);
    c->bdev.valid = false;
  }
  return EMRKC_OK;
}

extern "C" int emrkc_get_rho(const emrkc_ctx *c, double *rho_F, double *rho_S) {
  if (c == nullptr || !c->have_rho) return EMRKC_EINVAL;
  if (rho_F) *rho_F = c->rho_F;
  if (rho_S) *rho_S = c->rho_S;
  return EMRKC_OK;
}

extern "C" int emrkc_stages(const emrkc_ctx *c, double dt, int *s, int *m, double *eta) {
  if (c == nullptr || !c->have_rho) return EMRKC_EINVAL;
  return c->cond_a ? emrkc_stage_counts_a(dt, c->rho_F, c->rho_S, c->eps, s, m, eta)
                   : emrkc_stage_counts(dt, c->rho_F, c->rho_S, c->eps, s, m, eta);
}

extern "C" int emrkc_last_stats(const emrkc_ctx *c, emrkc_stats *out) {
  if (c == nullptr || out == nullptr) return EMRKC_EINVAL;
  *out = c->last;
  return EMRKC_OK;
}

// ---------------------------------------------------------------------------
// emRKC steps as sequences of launches
// ---------------------------------------------------------------------------
struct KernelTimer {
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> cls;        // 0 = head, 1 = inner, 2 = fused
  size_t used = 0;
  int arm(emrkc_ctx *c, int k);
};

// With a timer, the kernel launch itself records the pair of events (its
// dispatch timestamps), so the interval holds the kernel's execution only.
#define TIMED(cls, call)                                                  \
  do {                                                                    \
    if (tm && tm->arm(c, (cls))) return EMRKC_EHIP;                       \
    const hipError_t timed_e_ = (call);                                   \
    if (tm) set_launch_events(nullptr, nullptr);                          \
    if (timed_e_ != hipSuccess)                                           \
      return fail(c, EMRKC_EHIP, "%s failed: %s", #call,                  \
                  hipGetErrorString(timed_e_));                           \
  } while (0)

static HeadArgs make_head(emrkc_ctx *c, const StepPlan &P, double dt, int j, int step_off) {
  HeadArgs h{};
  h.SV = c->d_SV;
  h.clock = c->d_clock;
  h.step_off = step_off;
  h.stim = stim_args(c);
  h.mp = c->mp;
  h.dt = dt;
  h.eta = P.eta;
  h.inv_eta = 1.0 / P.eta;
  h.Cm = c->Cm;
  h.c_prev = P.cc[j - 1];
  h.mu_dt = P.mu[j] * dt;
  h.nu = P.nu[j];
  h.kappa = P.ka[j];
  h.mu1_eta = P.mui[1] * P.eta;
  h.cm_eta = P.cci[P.m] * P.eta;
  h.j1 = j == 1;
  h.m_is_one = P.m == 1;
  h.progressive = c->progressive ? 1 : 0;
  h.cm = P.cci[P.m];
  h.z_aos = c->zb_run ? 1 : 0;
  return h;
}

// The z the enqueued heads address: the caller's, or the block buffer while
// emrkc_step holds z in blocks (the pointwise head only).
static void *zstate(const emrkc_ctx *c, const emrkc_state *st) { return c->zb_run ? c->d_zb : st->z; }

static TailArgs make_stage(const StepPlan &P, double dt, int j, int k) {
  TailArgs t{};
  t.nu = P.nui[k];
  t.kappa = P.kai[k];
  t.mu_eta = P.mui[k] * P.eta;
  t.inv_eta = 1.0 / P.eta;
  t.mu_dt = P.mu[j] * dt;
  t.nu_o = P.nu[j];
  t.kappa_o = P.ka[j];
  t.j1 = j == 1;
  return t;
}

// Head shape 8 (3-D grids, m >= 2): the pointwise head writes z_j and S_V,
// and the first inner stage u_1 = u_0 + mu'_1 eta (f_F(u_0) + S_V) is an
// inner-kernel launch of its own (the grid's inner shape), ahead of the
// usual inner stages; the buffers follow the generic step.
static bool u1_split_mode(const emrkc_ctx *c, const StepPlan &P) {
  return c->method == EMRKC_METHOD_EMRKC && !c->batch && split_supported(c->mesh) &&
         c->mesh.grid.head_variant == 8 && P.m >= 2;
}

// One step, any (s, m), with separate head and inner kernels.
//
// V_j lives in X[j % 2] for j < s (X[0] = the caller's V, X[1] a library
// buffer): V_j may overwrite V_{j-2} because that value is only read at the
// same node.  The last stage writes X[0] unless m == 1 and V_{s-1} is in
// X[0]: then the head kernel that reads V_{s-1} with neighbours must not
// overwrite it, and the step ends with a copy.  z_j follows the same rule
// with Z[0] = the caller's z and always ends in Z[0] (z is pointwise).
// Inner values u_k (k >= 1) rotate through U[(k-1) % 2]; u_0 = V_{j-1}.
// The last kernel of the chunk advances the device clock by tick_by.
static int enqueue_step_generic(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int step_off,
                                int64_t tick_by, hipStream_t strm, KernelTimer *tm) {
  const int s = P.s, m = P.m;
  double *X[2] = {(double *)st->V, c->d_V1};
  void *Z[2] = {zstate(c, st), c->d_z1};
  auto vidx = [&](int j) { return j == 0 ? 0 : (j < s ? j % 2 : 0); };
  auto zidx = [&](int j) { return j == 0 ? 0 : (j < s ? j % 2 : 0); };
  const bool final_copy = (m == 1) && (vidx(s - 1) == 0);
  for (int j = 1; j <= s; ++j) {
    const bool lastj = j == s;
    double *Vin = X[vidx(j - 1)];
    double *Vin2 = j >= 2 ? X[vidx(j - 2)] : nullptr;
    double *Vdst = (lastj && final_copy) ? X[1] : X[vidx(j)];
    HeadArgs h = make_head(c, P, dt, j, step_off);
    h.Vin = Vin;
    h.Vin2 = Vin2;
    h.zin = Z[zidx(j - 1)];
    h.zin2 = j >= 2 ? Z[zidx(j - 2)] : nullptr;
    h.zout = Z[zidx(j)];
    h.uout = m >= 2 ? c->d_U[0] : Vdst;
    if (u1_split_mode(c, P)) {
      // head shape 8: the pointwise head, then u_1 by the inner kernel
      h.uout = nullptr;
      TIMED(0, launch_head_pw(c->model, c->mixed, c->mesh, h, strm));
      InnerArgs a{};
      a.t = make_stage(P, dt, j, 1);
      a.t.mu_eta = P.mui[1] * P.eta;
      a.t.uprev = Vin;
      a.t.uprev2 = Vin;
      a.t.SV = c->d_SV;
      a.first = 1;
      a.out = c->d_U[0];
      TIMED(1, launch_inner(c->mixed, c->mesh, a, strm));
    } else {
      TIMED(0, launch_head(c->model, c->mixed, c->mesh, h, strm));
    }
    for (int k = 2; k <= m; ++k) {
      InnerArgs a{};
      a.t = make_stage(P, dt, j, k);
      a.t.uprev = c->d_U[(k - 2) % 2];
      a.t.uprev2 = k == 2 ? Vin : c->d_U[(k - 3) % 2];
      a.t.SV = c->d_SV;
      a.t.Vin = Vin;
      a.t.Vin2 = Vin2;
      a.last = k == m;
      a.out = a.last ? Vdst : c->d_U[(k - 1) % 2];
      a.tick = (lastj && k == m && tick_by > 0) ? c->d_clock : nullptr;
      a.tick_by = tick_by;
      TIMED(1, launch_inner(c->mixed, c->mesh, a, strm));
    }
  }
  if (m == 1 && (final_copy || tick_by > 0)) {
    HIP_TRY(c, launch_copy_tick(final_copy ? X[1] : nullptr, X[0], (uint32_t)c->N, tick_by > 0 ? c->d_clock : nullptr,
                                tick_by, strm));
  }
  return EMRKC_OK;
}

// The split stage (3-D grids, head shape 7, m >= 2): the pointwise head
// writes z_j and S_V only, and k_inner12_march forms u_1 and u_2 in one
// pass (for m == 2 with the outer V update).  That kernel reads V_{j-1} with
// a halo, so with m == 2 it cannot write V_j over V_{j-1}: the buffers
// follow the rule of the m == 1 path (the last stage writes X[1] and copies
// when V_{s-1} is in X[0]); with m >= 3 the last inner stage reads u with a
// halo and V pointwise, as in the generic step.
static bool split_mode(const emrkc_ctx *c, const StepPlan &P) {
  return c->method == EMRKC_METHOD_EMRKC && !c->batch && split_supported(c->mesh) &&
         c->mesh.grid.head_variant == 7 && P.m >= 2;
}

static Inner12Args make_inner12(emrkc_ctx *c, const StepPlan &P, double dt, int j, const double *Vin,
                                const double *Vin2) {
  Inner12Args a{};
  a.t = make_stage(P, dt, j, 2);
  a.V = Vin;
  a.Vin2 = Vin2;
  a.SV = c->d_SV;
  a.mu1_eta = P.mui[1] * P.eta;
  a.last = P.m == 2;
  a.out = P.m == 2 ? nullptr : c->d_U[1];
  a.u1out = P.m == 2 ? nullptr : c->d_U[0];
  return a;
}

static int enqueue_step_split(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int step_off,
                              int64_t tick_by, hipStream_t strm, KernelTimer *tm) {
  const int s = P.s, m = P.m;
  double *X[2] = {(double *)st->V, c->d_V1};
  void *Z[2] = {zstate(c, st), c->d_z1};
  auto vidx = [&](int j) { return j == 0 ? 0 : (j < s ? j % 2 : 0); };
  const bool final_copy = m == 2 && vidx(s - 1) == 0;
  for (int j = 1; j <= s; ++j) {
    const bool lastj = j == s;
    double *Vin = X[vidx(j - 1)];
    double *Vin2 = j >= 2 ? X[vidx(j - 2)] : nullptr;
    double *Vdst = (lastj && final_copy) ? X[1] : X[vidx(j)];
    HeadArgs h = make_head(c, P, dt, j, step_off);
    h.Vin = Vin;
    h.Vin2 = Vin2;
    h.zin = Z[vidx(j - 1)];
    h.zin2 = j >= 2 ? Z[vidx(j - 2)] : nullptr;
    h.zout = Z[vidx(j)];
    h.uout = nullptr;
    TIMED(0, launch_head_pw(c->model, c->mixed, c->mesh, h, strm));
    Inner12Args a = make_inner12(c, P, dt, j, Vin, Vin2);
    if (m == 2) a.out = Vdst;
    a.tick = (lastj && m == 2 && tick_by > 0 && !final_copy) ? c->d_clock : nullptr;
    a.tick_by = tick_by;
    TIMED(1, launch_inner12(c->mixed, c->mesh, a, strm));
    for (int k = 3; k <= m; ++k) {
      InnerArgs b{};
      b.t = make_stage(P, dt, j, k);
      b.t.uprev = c->d_U[(k - 2) % 2];
      b.t.uprev2 = c->d_U[(k - 3) % 2];
      b.t.SV = c->d_SV;
      b.t.Vin = Vin;
      b.t.Vin2 = Vin2;
      b.last = k == m;
      b.out = b.last ? Vdst : c->d_U[(k - 1) % 2];
      b.tick = (lastj && k == m && tick_by > 0) ? c->d_clock : nullptr;
      b.tick_by = tick_by;
      TIMED(1, launch_inner(c->mixed, c->mesh, b, strm));
    }
  }
  if (final_copy)
    HIP_TRY(c, launch_copy_tick(X[1], X[0], (uint32_t)c->N, tick_by > 0 ? c->d_clock : nullptr, tick_by, strm));
  return EMRKC_OK;
}

// L split steps with s == 1 and m == 2: V^n alternates X[n % 2] (the inner
// kernel reads V^n with a halo while it writes V^{n+1}); an odd chunk ends
// with one copy back to X[0].
static int enqueue_chunk_split_s1m2(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int L,
                                    hipStream_t strm, KernelTimer *tm) {
  double *X[2] = {(double *)st->V, c->d_V1};
  for (int n = 0; n < L; ++n) {
    HeadArgs h = make_head(c, P, dt, 1, n);
    h.Vin = X[n % 2];
    h.zin = h.zout = zstate(c, st);
    h.uout = nullptr;
    TIMED(0, launch_head_pw(c->model, c->mixed, c->mesh, h, strm));
    Inner12Args a = make_inner12(c, P, dt, 1, X[n % 2], nullptr);
    a.out = X[(n + 1) % 2];
    a.tick = (n == L - 1 && L % 2 == 0) ? c->d_clock : nullptr;
    a.tick_by = L;
    TIMED(1, launch_inner12(c->mixed, c->mesh, a, strm));
  }
  if (L % 2) HIP_TRY(c, launch_copy_tick(X[1], X[0], (uint32_t)c->N, c->d_clock, L, strm));
  return EMRKC_OK;
}

// All inner stages of a stage in one launch (2-D grids, inner shape 2,
// 2 <= m <= kInnerAllMaxM): the head as usual (u_1 into U[0]), then
// k_inner_all2d, which reads V_{j-1} with a halo and so writes V_j to the
// other buffer: s == 1 alternates X[n % 2] over a chunk (an odd chunk ends
// with one copy), s >= 2 rotates as the generic step with the final copy
// of the m == 1 rule.
static bool inner_all_mode(const emrkc_ctx *c, const StepPlan &P) {
  return c->method == EMRKC_METHOD_EMRKC && !c->batch && inner_all_supported(c->mesh, P.m) &&
         c->mesh.grid.inner_variant >= 2 && c->mesh.grid.inner_variant <= 4;
}

// Inner shape 4 with s == 1: one kernel per step (the inner stages of step
// n and the head of step n + 1), after a head for the chunk's first step
// and before a last inner-stage kernel; u_1, S_V and V alternate buffers.
static bool step2d_mode(const emrkc_ctx *c, const StepPlan &P) {
  return inner_all_mode(c, P) && c->mesh.grid.inner_variant == 4 && P.s == 1;
}

static InnerAllArgs make_inner_all(emrkc_ctx *c, const StepPlan &P, double dt, int j) {
  InnerAllArgs a{};
  a.t = make_stage(P, dt, j, P.m);
  for (int k = 2; k <= P.m; ++k) {
    a.nu[k] = P.nui[k];
    a.kappa[k] = P.kai[k];
    a.mu_eta[k] = P.mui[k] * P.eta;
  }
  a.m = P.m;
  a.u1 = c->d_U[0];
  a.SV = c->d_SV;
  return a;
}

static int enqueue_chunk_inner_all(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int L,
                                   hipStream_t strm, KernelTimer *tm) {
  const int s = P.s;
  double *X[2] = {(double *)st->V, c->d_V1};
  void *Z[2] = {zstate(c, st), c->d_z1};
  if (step2d_mode(c, P)) {
    double *Ub[2] = {c->d_U[0], c->d_U[1]};
    void *S[2] = {c->d_SV, c->d_SV2};
    if (!Ub[0] || !Ub[1] || !S[0] || !S[1])
      return fail(c, EMRKC_EINVAL, "one-kernel 2-D step: a u_1 or S_V work buffer is missing");
    HeadArgs h = make_head(c, P, dt, 1, 0);
    h.Vin = X[0];
    h.zin = h.zout = zstate(c, st);
    h.SV = S[0];
    h.uout = Ub[0];
    TIMED(0, launch_head(c->model, c->mixed, c->mesh, h, strm));
    for (int n = 0; n + 1 < L; ++n) {
      InnerAllArgs a = make_inner_all(c, P, dt, 1);
      a.u1 = Ub[n % 2];
      a.V = X[n % 2];
      a.SV = S[n % 2];
      a.out = X[(n + 1) % 2];
      HeadArgs hn = make_head(c, P, dt, 1, n + 1);
      hn.zin = hn.zout = zstate(c, st);
      hn.SV = S[(n + 1) % 2];
      hn.uout = Ub[(n + 1) % 2];
      TIMED(2, launch_step2d(c->model, c->mixed, c->mesh, a, hn, strm));
    }
    InnerAllArgs a = make_inner_all(c, P, dt, 1);
    a.u1 = Ub[(L - 1) % 2];
    a.V = X[(L - 1) % 2];
    a.SV = S[(L - 1) % 2];
    a.out = X[L % 2];
    a.tick = L % 2 == 0 ? c->d_clock : nullptr;
    a.tick_by = L;
    TIMED(1, launch_inner_all(c->mixed, c->mesh, a, strm));
    if (L % 2) HIP_TRY(c, launch_copy_tick(X[1], X[0], (uint32_t)c->N, c->d_clock, L, strm));
    return EMRKC_OK;
  }
  if (s == 1) {
    for (int n = 0; n < L; ++n) {
      HeadArgs h = make_head(c, P, dt, 1, n);
      h.Vin = X[n % 2];
      h.zin = h.zout = zstate(c, st);
      h.uout = c->d_U[0];
      TIMED(0, launch_head(c->model, c->mixed, c->mesh, h, strm));
      InnerAllArgs a = make_inner_all(c, P, dt, 1);
      a.V = X[n % 2];
      a.out = X[(n + 1) % 2];
      a.tick = (n == L - 1 && L % 2 == 0) ? c->d_clock : nullptr;
      a.tick_by = L;
      TIMED(1, launch_inner_all(c->mixed, c->mesh, a, strm));
    }
    if (L % 2) HIP_TRY(c, launch_copy_tick(X[1], X[0], (uint32_t)c->N, c->d_clock, L, strm));
    return EMRKC_OK;
  }
  auto vidx = [&](int j) { return j == 0 ? 0 : (j < s ? j % 2 : 0); };
  const bool final_copy = vidx(s - 1) == 0;
  for (int n = 0; n < L; ++n) {
    for (int j = 1; j <= s; ++j) {
      const bool lastj = j == s;
      double *Vin = X[vidx(j - 1)];
      double *Vin2 = j >= 2 ? X[vidx(j - 2)] : nullptr;
      double *Vdst = (lastj && final_copy) ? X[1] : X[vidx(j)];
      HeadArgs h = make_head(c, P, dt, j, n);
      h.Vin = Vin;
      h.Vin2 = Vin2;
      h.zin = Z[vidx(j - 1)];
      h.zin2 = j >= 2 ? Z[vidx(j - 2)] : nullptr;
      h.zout = Z[vidx(j)];
      h.uout = c->d_U[0];
      TIMED(0, launch_head(c->model, c->mixed, c->mesh, h, strm));
      InnerAllArgs a = make_inner_all(c, P, dt, j);
      a.V = Vin;
      a.Vin2 = Vin2;
      a.out = Vdst;
      a.tick = (lastj && n == L - 1 && !final_copy) ? c->d_clock : nullptr;
      a.tick_by = L;
      TIMED(1, launch_inner_all(c->mixed, c->mesh, a, strm));
    }
    if (final_copy)
      HIP_TRY(c, launch_copy_tick(X[1], X[0], (uint32_t)c->N, n == L - 1 ? c->d_clock : nullptr, L, strm));
  }
  return EMRKC_OK;
}

// L steps with s == 1 and m >= 2 on a grid: head of step 0, then for each
// later step one fused kernel (last inner stage of the previous step + head
// of this step), and the last inner stage of step L-1 on its own.  Within
// the chunk V^n alternates X[n % 2] (the fused kernel reads V^{n-1} of
// neighbouring tiles while writing V^n), S_V alternates SV[n % 2], and
// u_k of step n lives in B[(b_n + k - 1) % 3] with b_{n+1} = b_n + m - 1, so
// the values the fused kernel reads (u_{m-1}, u_{m-2} of step n-1) never
// share a buffer with the u_1 it writes.  V^L ends in X[0].
static int enqueue_chunk_fused(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int L,
                               hipStream_t strm, KernelTimer *tm) {
  const int m = P.m;
  double *X[2] = {(double *)st->V, c->d_V1};
  double *B[3] = {c->d_U[0], c->d_U[1], c->d_U[2]};
  void *S[2] = {c->d_SV, c->d_SV2};
  if (!B[0] || !B[1] || !B[2] || !S[0] || !S[1])
    return fail(c, EMRKC_EINVAL, "fused chunk: an inner or S_V work buffer is missing");
  int base = 0;
  auto inner_range = [&](int n, int b) -> int {
    for (int k = 2; k <= m - 1; ++k) {
      InnerArgs a{};
      a.t = make_stage(P, dt, 1, k);
      a.t.uprev = B[(b + k - 2) % 3];
      a.t.uprev2 = k == 2 ? X[n % 2] : B[(b + k - 3) % 3];
      a.t.SV = S[n % 2];
      a.last = 0;
      a.out = B[(b + k - 1) % 3];
      TIMED(1, launch_inner(c->mixed, c->mesh, a, strm));
    }
    return EMRKC_OK;
  };
  auto tail_of = [&](int n, int b) {  // last inner stage of step n
    TailArgs t = make_stage(P, dt, 1, m);
    t.uprev = B[(b + m - 2) % 3];
    t.uprev2 = m == 2 ? X[n % 2] : B[(b + m - 3) % 3];
    t.SV = S[n % 2];
    t.Vin = X[n % 2];
    t.Vin2 = nullptr;
    return t;
  };
  HeadArgs h = make_head(c, P, dt, 1, 0);
  h.Vin = X[0];
  h.zin = h.zout = zstate(c, st);
  h.SV = S[0];
  h.uout = B[base];
  TIMED(0, launch_head(c->model, c->mixed, c->mesh, h, strm));
  int rc = inner_range(0, base);
  if (rc != EMRKC_OK) return rc;
  for (int n = 1; n < L; ++n) {
    FusedArgs f{};
    f.t = tail_of(n - 1, base);
    f.Vout = X[n % 2];
    base = (base + m - 1) % 3;
    f.h = make_head(c, P, dt, 1, n);
    f.h.zin = f.h.zout = zstate(c, st);
    f.h.SV = S[n % 2];
    f.h.uout = B[base];
    TIMED(2, launch_fused(c->model, c->mixed, c->mesh, f, strm));
    if ((rc = inner_range(n, base)) != EMRKC_OK) return rc;
  }
  InnerArgs a{};
  a.t = tail_of(L - 1, base);
  a.last = 1;
  a.out = X[0];
  a.tick = c->d_clock;
  a.tick_by = L;
  TIMED(1, launch_inner(c->mixed, c->mesh, a, strm));
  return EMRKC_OK;
}

// L steps with s == m == 1: the head kernel computes V^{n+1} directly from
// V^n read with neighbours, so V ping-pongs between X[0] and X[1] and only
// an odd chunk ends with one copy back to X[0].
static int enqueue_chunk_s1m1(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int L,
                              hipStream_t strm, KernelTimer *tm) {
  double *X[2] = {(double *)st->V, c->d_V1};
  for (int n = 0; n < L; ++n) {
    HeadArgs h = make_head(c, P, dt, 1, n);
    h.Vin = X[n % 2];
    h.zin = h.zout = zstate(c, st);
    h.uout = X[(n + 1) % 2];
    TIMED(0, launch_head(c->model, c->mixed, c->mesh, h, strm));
  }
  HIP_TRY(c, launch_copy_tick(L % 2 ? X[1] : nullptr, X[0], (uint32_t)c->N, c->d_clock, L, strm));
  return EMRKC_OK;
}

// One mRKC step, any (s, m): the buffer rotation of enqueue_step_generic,
// with gate 0 carried through the inner stages in d_W[] (its w_0 is plane 0
// of z_{j-1}, and its outer update lands in plane 0 of z_j at the last inner
// stage; the head leaves that plane alone when m >= 2).
static int enqueue_step_mrkc(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int step_off,
                             int64_t tick_by, hipStream_t strm, KernelTimer *tm) {
  const int s = P.s, m = P.m;
  double *X[2] = {(double *)st->V, c->d_V1};
  void *Z[2] = {st->z, c->d_z1};
  auto vidx = [&](int j) { return j == 0 ? 0 : (j < s ? j % 2 : 0); };
  const bool final_copy = (m == 1) && (vidx(s - 1) == 0);
  for (int j = 1; j <= s; ++j) {
    const bool lastj = j == s;
    double *Vin = X[vidx(j - 1)];
    double *Vin2 = j >= 2 ? X[vidx(j - 2)] : nullptr;
    double *Vdst = (lastj && final_copy) ? X[1] : X[vidx(j)];
    MrkcHeadArgs ha{};
    ha.h = make_head(c, P, dt, j, step_off);
    ha.h.Vin = Vin;
    ha.h.Vin2 = Vin2;
    ha.h.zin = Z[vidx(j - 1)];
    ha.h.zin2 = j >= 2 ? Z[vidx(j - 2)] : nullptr;
    ha.h.zout = Z[vidx(j)];
    ha.h.uout = m >= 2 ? c->d_U[0] : Vdst;
    ha.wout = c->d_W[0];
    TIMED(0, launch_mrkc_head(c->model, c->mesh, ha, strm));
    for (int k = 2; k <= m; ++k) {
      MrkcInnerArgs ia{};
      InnerArgs &a = ia.a;
      a.t = make_stage(P, dt, j, k);
      a.t.uprev = c->d_U[(k - 2) % 2];
      a.t.uprev2 = k == 2 ? Vin : c->d_U[(k - 3) % 2];
      a.t.SV = c->d_SV;
      a.t.Vin = Vin;
      a.t.Vin2 = Vin2;
      a.last = k == m;
      a.out = a.last ? Vdst : c->d_U[(k - 1) % 2];
      a.tick = (lastj && k == m && tick_by > 0) ? c->d_clock : nullptr;
      a.tick_by = tick_by;
      ia.wprev = c->d_W[(k - 2) % 2];
      ia.wprev2 = k == 2 ? (const double *)ha.h.zin : c->d_W[(k - 3) % 2];
      ia.wout = c->d_W[(k - 1) % 2];
      ia.zq_in = (const double *)ha.h.zin;
      ia.zq_in2 = (const double *)ha.h.zin2;
      ia.zq_out = (double *)ha.h.zout;
      ia.mp = c->mp;
      TIMED(1, launch_mrkc_inner(c->model, c->mesh, ia, strm));
    }
  }
  if (m == 1 && (final_copy || tick_by > 0)) {
    HIP_TRY(c, launch_copy_tick(final_copy ? X[1] : nullptr, X[0], (uint32_t)c->N, tick_by > 0 ? c->d_clock : nullptr,
                                tick_by, strm));
  }
  return EMRKC_OK;
}

static int enqueue_chunk_batch(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int L,
                               hipStream_t strm, KernelTimer *tm);

static int enqueue_chunk(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int L, hipStream_t strm,
                         KernelTimer *tm = nullptr) {
  if (c->batch) return enqueue_chunk_batch(c, st, P, dt, L, strm, tm);
  if (c->method == EMRKC_METHOD_MRKC) {
    for (int n = 0; n < L; ++n) {
      int rc = enqueue_step_mrkc(c, st, P, dt, n, n == L - 1 ? L : 0, strm, tm);
      if (rc != EMRKC_OK) return rc;
    }
    return EMRKC_OK;
  }
  if (inner_all_mode(c, P)) return enqueue_chunk_inner_all(c, st, P, dt, L, strm, tm);
  if (split_mode(c, P)) {
    if (P.s == 1 && P.m == 2) return enqueue_chunk_split_s1m2(c, st, P, dt, L, strm, tm);
    for (int n = 0; n < L; ++n) {
      int rc = enqueue_step_split(c, st, P, dt, n, n == L - 1 ? L : 0, strm, tm);
      if (rc != EMRKC_OK) return rc;
    }
    return EMRKC_OK;
  }
  if (c->use_fused && P.s == 1 && P.m >= 2 && fused_supported(c->mesh))
    return enqueue_chunk_fused(c, st, P, dt, L, strm, tm);
  if (P.s == 1 && P.m == 1) return enqueue_chunk_s1m1(c, st, P, dt, L, strm, tm);
  for (int n = 0; n < L; ++n) {
    int rc = enqueue_step_generic(c, st, P, dt, n, n == L - 1 ? L : 0, strm, tm);
    if (rc != EMRKC_OK) return rc;
  }
  return EMRKC_OK;
}

// z arrays of the library hold whole blocks of kZBlock nodes, so that they
// serve in either z layout
static size_t z_bytes(const emrkc_ctx *c) {
  const size_t nodes = (size_t)((c->N + kZBlock - 1) / kZBlock) * kZBlock;
  return (c->mixed ? sizeof(float) : sizeof(double)) * nodes * (size_t)(c->nv - 1);
}

static int ensure_z1(emrkc_ctx *c) {
  if (c->d_z1 != nullptr) return EMRKC_OK;
  return dalloc(c, &c->d_z1, z_bytes(c));
}

// emrkc_step keeps z in blocks of kZBlock nodes (all components of a block
// contiguous) while it steps: each wave of a head then reads and writes one
// contiguous run instead of 2 n_z component planes, which moved the
// pointwise head's bytes 14% faster on the 36.5M-node slab.  The caller's z
// is converted on entry and back on exit; EMRKC_Z_PLANES, rho_every (whose
// estimates read the caller's z between chunks), mRKC, the z-marching
// heads and a failed allocation of the block buffer keep the component
// planes.  So does a z array below kZBlocksMinBytes unless
// EMRKC_Z_BLOCKS asks for blocks: it is served from the 256 MB last-level
// cache in either layout (the 3-D grid of 442k nodes, 71 MB of z, steps at
// the same rate in both), so the two conversion launches per call would
// buy nothing.
constexpr size_t kZBlocksMinBytes = size_t(256) << 20;

static bool zblocks_mode(const emrkc_ctx *c, const StepPlan &P) {
  if (c->method != EMRKC_METHOD_EMRKC || (c->flags & EMRKC_Z_PLANES) || c->rho_every > 0) return false;
  if (!(c->flags & EMRKC_Z_BLOCKS) && z_bytes(c) < kZBlocksMinBytes) return false;
  // both batched heads read z through head_node (the tables are built
  // after the layout is chosen, with the buffer it uses)
  if (c->batch) return true;
  if (split_mode(c, P) || u1_split_mode(c, P)) return true;
  // every other emRKC head reads and writes z through head_node, which
  // takes either layout, except the z-marching heads (3-D shapes 1 and 2),
  // which stage component planes themselves
  const Grid &g = c->mesh.grid;
  return !(c->mesh.kind == kGrid && !c->mesh.flat && g.dim == 3 && (g.head_variant == 1 || g.head_variant == 2));
}

// Converts the state's z into the block buffer and points the heads at it
// (*on = true), or leaves the planes (*on = false) when the mode does not
// apply or the buffer cannot be allocated.
static int zblocks_begin(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, bool *on) {
  *on = false;
  if (!zblocks_mode(c, P)) return EMRKC_OK;
  if (c->d_zb == nullptr && hipMalloc(&c->d_zb, z_bytes(c)) != hipSuccess) {
    c->d_zb = nullptr;
    (void)hipGetLastError();
    return EMRKC_OK;
  }
  HIP_TRY(c, launch_z_layout(c->mixed, st->z, c->d_zb, (uint32_t)c->N, (uint32_t)(c->nv - 1), true, c->stream));
  c->zb_run = *on = true;
  return EMRKC_OK;
}

static int zblocks_end(emrkc_ctx *c, const emrkc_state *st, bool on) {
  if (!on) return EMRKC_OK;
  c->zb_run = false;
  HIP_TRY(c, launch_z_layout(c->mixed, c->d_zb, st->z, (uint32_t)c->N, (uint32_t)(c->nv - 1), false, c->stream));
  return EMRKC_OK;
}

static int build_batch_tables(emrkc_ctx *c, const emrkc_state *st, double dt, const StepPlan &P);

// (s, m, eta) of a single context under its stability condition (B unless
// EMRKC_COND_A).
static int select_stages(const emrkc_ctx *c, double dt, double rho_F, double rho_S, int *s, int *m, double *eta) {
  return c->cond_a ? emrkc_stage_counts_a(dt, rho_F, rho_S, c->eps, s, m, eta)
                   : emrkc_stage_counts(dt, rho_F, rho_S, c->eps, s, m, eta);
}

// (s, m, eta) and the coefficient tables for dt; for a batch, s and eta are
// common (from the largest rho_S) and m is the largest per-instance m.
static int make_plan(emrkc_ctx *c, double dt, StepPlan &P) {
  int rc = select_stages(c, dt, c->rho_F, c->rho_S, &P.s, &P.m, &P.eta);
  if (rc != EMRKC_OK) return fail(c, rc, "stage selection failed (dt=%g rho_F=%g rho_S=%g)", dt, c->rho_F, c->rho_S);
  if (c->batch) {
    if (P.s != 1) return fail(c, EMRKC_EUNSUPPORTED, "batched ensembles need s = 1 (dt=%g gives s=%d)", dt, P.s);
    P.m = 1;
    for (auto &I : c->inst) {
      int si, mi;
      double ei;
      rc = emrkc_stage_counts(dt, I.rho_F, c->rho_S, c->eps, &si, &mi, &ei);
      if (rc != EMRKC_OK) return fail(c, rc, "stage selection failed for an instance");
      I.m = mi;
      P.m = std::max(P.m, mi);
    }
  }
  rkc_coeffs(P.s, c->eps, P.mu, P.nu, P.ka, P.cc);
  rkc_coeffs(P.m, c->eps, P.mui, P.nui, P.kai, P.cci);
  if (P.s >= 2 && (rc = ensure_z1(c)) != EMRKC_OK) return rc;
  if (c->method == EMRKC_METHOD_MRKC && c->d_W[0] == nullptr) {
    const size_t vb = sizeof(double) * (size_t)c->N;
    if ((rc = dalloc(c, (void **)&c->d_W[0], vb)) || (rc = dalloc(c, (void **)&c->d_W[1], vb))) return rc;
  }
  return EMRKC_OK;
}

static int step_core(emrkc_ctx *c, emrkc_state *st, double dt, int64_t nsteps);

extern "C" int emrkc_step(emrkc_ctx *c, emrkc_state *st, double dt, int64_t nsteps) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  if (!(dt > 0) || !isfinite(dt) || nsteps < 0) return fail(c, EMRKC_EINVAL, "invalid dt or nsteps");
  if (!c->have_rho) return fail(c, EMRKC_EINVAL, "spectral radii not set: call emrkc_estimate_rho or emrkc_set_rho");
  if (nsteps == 0) return EMRKC_OK;
  rebase_clock(st, dt);
  if (c->rho_every <= 0) return step_core(c, st, dt, nsteps);
  // re-estimate the radii (warm started) before every step whose index is a
  // positive multiple of rho_every; runs of steps in between as usual.  A
  // re-estimate that reaches the iteration limit keeps its best value.
  const int64_t K = c->rho_every;
  int64_t left = nsteps;
  while (left > 0) {
    if (st->step > 0 && st->step % K == 0 && c->last_est_step != st->step) {
      st->t = state_time(st->t0, st->step, dt);
      const int rc = emrkc_estimate_rho(c, st, nullptr, nullptr, nullptr, nullptr);
      if (rc != EMRKC_OK && rc != EMRKC_ENOCONV) return rc;
      c->last_est_step = st->step;
    }
    const int64_t next = (st->step / K + 1) * K;
    const int64_t len = std::min(left, next - st->step);
    const int rc = step_core(c, st, dt, len);
    if (rc != EMRKC_OK) return rc;
    left -= len;
  }
  return EMRKC_OK;
}

// Enqueues nsteps steps in chunks of up to 32 (enq(L, stream) enqueues L
// steps); with graphs every chunk length is captured once per key and
// replayed, the step time coming from the device clock.
static int run_chunks(emrkc_ctx *c, const emrkc_state *st, double dt, int64_t nsteps, int key_s, int key_m,
                      const std::function<int(int, hipStream_t)> &enq, bool *used_graph) {
  int rc;
  HIP_TRY(c, launch_clock_set(c->d_clock, st->step, st->t0, c->stream));
  const bool eager = (c->flags & EMRKC_EAGER_FLAG) != 0 || getenv("EMRKC_EAGER") != nullptr;
  const int chunk = (int)std::min<int64_t>(nsteps, 32);
  const int64_t full = nsteps / chunk;
  const int rem = (int)(nsteps - full * chunk);
  *used_graph = false;
  for (int pass = 0; pass < 2; ++pass) {
    const int len = pass == 0 ? chunk : rem;
    const int64_t reps = pass == 0 ? full : (rem > 0 ? 1 : 0);
    if (len <= 0 || reps <= 0) continue;
    if (eager) {
      for (int64_t r = 0; r < reps; ++r)
        if ((rc = enq(len, c->stream)) != EMRKC_OK) return rc;
      continue;
    }
    uint64_t dtb;
    memcpy(&dtb, &dt, sizeof dtb);
    // keyed by the z buffer the kernels use (the state's, or the block
    // buffer), so a layout change between calls cannot replay a graph
    // captured for the other one
    GraphKey key{key_s, key_m, len, dtb, st->V, zstate(c, st)};
    hipGraphExec_t exec = nullptr;
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
      exec = it->second;
    } else {
      hipGraph_t graph = nullptr;
      HIP_TRY(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
      const int erc = enq(len, c->capture);
      hipError_t ee = hipStreamEndCapture(c->capture, &graph);
      if (erc != EMRKC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return erc;
      }
      if (ee != hipSuccess) return fail(c, EMRKC_EHIP, "graph capture failed: %s", hipGetErrorString(ee));
      ee = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ee != hipSuccess) return fail(c, EMRKC_EHIP, "graph instantiation failed: %s", hipGetErrorString(ee));
      if (c->graphs.size() >= 64) {
        for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        c->graphs.clear();
      }
      c->graphs[key] = exec;
    }
    for (int64_t r = 0; r < reps; ++r) HIP_TRY(c, hipGraphLaunch(exec, c->stream));
    *used_graph = true;
  }
  return EMRKC_OK;
}

// EMRKC_CHECK_FINITE: synchronises and reports a non-finite V.
static int check_finite(emrkc_ctx *c, const emrkc_state *st) {
  if (!(c->flags & EMRKC_CHECK_FINITE)) return EMRKC_OK;
  HIP_TRY(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
  HIP_TRY(c, launch_finite_check((uint32_t)c->N, (const double *)st->V, c->d_flag, c->stream));
  int flag = 0;
  HIP_TRY(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (flag) return fail(c, EMRKC_ENONFINITE, "V holds a non-finite value after step %lld", (long long)st->step);
  return EMRKC_OK;
}

static void set_last_stats(emrkc_ctx *c, const StepPlan &P, bool used_graph, bool z_blocks = false) {
  c->last.s = P.s;
  c->last.m = P.m;
  c->last.eta = P.eta;
  // split steps: s (head + m - 1 inner kernels), plus the copy when m == 2
  // and V_{s-1} ends in the caller's buffer (s odd, s > 1; s == 1 alternates)
  const int64_t split = (int64_t)P.s * P.m + (P.m == 2 && P.s > 1 && P.s % 2 == 1 ? 1 : 0);
  c->last.kernels_per_step = c->batch ? (int64_t)P.m
                              : split_mode(c, P) ? split
                              : u1_split_mode(c, P) ? (int64_t)P.s * (P.m + 1)
                              : step2d_mode(c, P) ? 1
                              : inner_all_mode(c, P) ? (int64_t)2 * P.s + (P.s > 1 && P.s % 2 == 1 ? 1 : 0)
                              : (c->use_fused && P.s == 1 && P.m >= 2 && fused_supported(c->mesh))
                                 ? (int64_t)P.m - 1
                                 : (P.s == 1 && P.m == 1) ? 1 : (int64_t)P.s * P.m + (P.m == 1 ? 1 : 0);
  c->last.used_graph = used_graph ? 1 : 0;
  c->last.z_blocks = z_blocks ? 1 : 0;
}

static int step_core(emrkc_ctx *c, emrkc_state *st, double dt, int64_t nsteps) {
  StepPlan P;
  int rc = make_plan(c, dt, P);
  if (rc != EMRKC_OK) return rc;
  bool used_graph = false, zb = false;
  if ((rc = zblocks_begin(c, st, P, &zb)) != EMRKC_OK) return rc;
  // a batch's tables name the z buffer the layout uses: built after it
  if (c->batch && (rc = build_batch_tables(c, st, dt, P)) != EMRKC_OK) {
    (void)zblocks_end(c, st, zb);
    return rc;
  }
  rc = run_chunks(c, st, dt, nsteps, P.s, P.m,
                  [&](int L, hipStream_t strm) { return enqueue_chunk(c, st, P, dt, L, strm); }, &used_graph);
  const int rc_end = zblocks_end(c, st, zb);
  if (rc == EMRKC_OK) rc = rc_end;
  if (rc != EMRKC_OK) return rc;
  st->step += nsteps;
  st->t = state_time(st->t0, st->step, dt);
  set_last_stats(c, P, used_graph, zb);
  return check_finite(c, st);
}

// ---------------------------------------------------------------------------
// emrkc_step without allocation: the step's work buffers (the device clock,
// V_1, the inner values u_k, S_V and, for s >= 2, z_1) come from the
// device's static scratch array instead of the context, the coefficient
// tables go to arrays sized at creation, and the kernels are launched
// directly on the context stream (no graph is instantiated).  The kernels
// and their order are those of emrkc_step's eager path, so the results are
// the same bits.
// ---------------------------------------------------------------------------
static int make_plan_fixed(emrkc_ctx *c, double dt) {
  StepPlan &P = c->fixed_plan;
  int rc = select_stages(c, dt, c->rho_F, c->rho_S, &P.s, &P.m, &P.eta);
  if (rc != EMRKC_OK) return fail(c, rc, "stage selection failed (dt=%g rho_F=%g rho_S=%g)", dt, c->rho_F, c->rho_S);
  if (P.s > kNoAllocMaxStages || P.m > kNoAllocMaxStages)
    return fail(c, EMRKC_EUNSUPPORTED, "emrkc_step_noalloc: stage counts (s=%d, m=%d) above %d", P.s, P.m,
                kNoAllocMaxStages);
  double *w = c->fixed_work.data();
  const size_t K = kNoAllocMaxStages + 1;
  rkc_coeffs_into(P.s, c->eps, P.mu.data(), P.nu.data(), P.ka.data(), P.cc.data(), w, w + K, w + 2 * K);
  rkc_coeffs_into(P.m, c->eps, P.mui.data(), P.nui.data(), P.kai.data(), P.cci.data(), w, w + K, w + 2 * K);
  return EMRKC_OK;
}

// Byte offsets of the work buffers in the scratch array (256-byte aligned).
struct ScratchLayout {
  size_t clock, V1, U[3], SV, SV2, z1, total;
};

static ScratchLayout scratch_layout(const emrkc_ctx *c, int s, bool fused) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t N = (size_t)c->N;
  const size_t vb = up(sizeof(double) * N);
  const size_t svb = up((c->mixed ? sizeof(float) : sizeof(double)) * N);
  ScratchLayout L{};
  size_t o = 0;
  L.clock = o;
  o += up(sizeof(Clock));
  L.V1 = o;
  o += vb;
  L.U[0] = o;
  o += vb;
  L.U[1] = o;
  o += vb;
  L.SV = o;
  o += svb;
  if (fused) {  // the fused chunk rotates three inner buffers and two S_V
    L.U[2] = o;
    o += vb;
    L.SV2 = o;
    o += svb;
  }
  if (s >= 2) {  // z_j of the odd stages
    L.z1 = o;
    o += up((c->mixed ? sizeof(float) : sizeof(double)) * N * (size_t)(c->nv - 1));
  }
  L.total = o;
  return L;
}

// Points the context's step work buffers into the scratch array while it
// lives (the enqueue functions take them from the context) and gives the
// context its own buffers back when it goes out of scope, on every return.
struct ScratchWork {
  emrkc_ctx *c;
  double *V1, *U[3];
  void *SV, *SV2, *z1;
  Clock *clock;
  ScratchWork(emrkc_ctx *ctx, const ScratchLayout &L, bool fused, int s) : c(ctx) {
    V1 = c->d_V1;
    for (int k = 0; k < 3; ++k) U[k] = c->d_U[k];
    SV = c->d_SV;
    SV2 = c->d_SV2;
    z1 = c->d_z1;
    clock = c->d_clock;
    unsigned char *b = c->scratch;
    c->d_clock = (Clock *)(b + L.clock);
    c->d_V1 = (double *)(b + L.V1);
    c->d_U[0] = (double *)(b + L.U[0]);
    c->d_U[1] = (double *)(b + L.U[1]);
    c->d_U[2] = fused ? (double *)(b + L.U[2]) : nullptr;
    c->d_SV = b + L.SV;
    c->d_SV2 = fused ? (void *)(b + L.SV2) : nullptr;
    c->d_z1 = s >= 2 ? (void *)(b + L.z1) : nullptr;
  }
  ~ScratchWork() {
    c->d_V1 = V1;
    for (int k = 0; k < 3; ++k) c->d_U[k] = U[k];
    c->d_SV = SV;
    c->d_SV2 = SV2;
    c->d_z1 = z1;
    c->d_clock = clock;
  }
};

extern "C" int emrkc_step_noalloc(emrkc_ctx *c, emrkc_state *st, double dt, int64_t nsteps) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  if (!(dt > 0) || !isfinite(dt) || nsteps < 0) return fail(c, EMRKC_EINVAL, "invalid dt or nsteps");
  if (!c->have_rho) return fail(c, EMRKC_EINVAL, "spectral radii not set: call emrkc_estimate_rho or emrkc_set_rho");
  if (c->batch || c->method != EMRKC_METHOD_EMRKC || c->rho_every > 0 || (c->flags & EMRKC_CHECK_FINITE))
    return fail(c, EMRKC_EUNSUPPORTED,
                "emrkc_step_noalloc takes single emRKC contexts without rho_every or EMRKC_CHECK_FINITE");
  if (c->scratch == nullptr) return fail(c, EMRKC_EHIP, "static scratch unavailable: %s", c->scratch_err.c_str());
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, EMRKC_EINVAL, "context created on device %d, current device is %d", c->device, dev);
  if (nsteps == 0) return EMRKC_OK;
  int rc = make_plan_fixed(c, dt);
  if (rc != EMRKC_OK) return rc;
  const StepPlan &P = c->fixed_plan;
  // (the one-kernel 2-D step alternates S_V buffers as the fused chunk does)
  const bool fused = (c->use_fused && P.s == 1 && P.m >= 2 && fused_supported(c->mesh)) || step2d_mode(c, P);
  const ScratchLayout L = scratch_layout(c, P.s, fused);
  if (L.total > kScratchBytes)
    return fail(c, EMRKC_EINVAL,
                "emrkc_step_noalloc: %lld nodes with s=%d need %zu bytes of scratch, more than the %zu of the "
                "static array",
                (long long)c->N, P.s, L.total, kScratchBytes);
  rebase_clock(st, dt);
  {
    ScratchWork work(c, L, fused, P.s);
    // the same chunking as emrkc_step, so the clock advances identically
    HIP_TRY(c, launch_clock_set(c->d_clock, st->step, st->t0, c->stream));
    const int chunk = (int)std::min<int64_t>(nsteps, 32);
    const int64_t full = nsteps / chunk;
    const int rem = (int)(nsteps - full * chunk);
    for (int64_t r = 0; r < full; ++r)
      if ((rc = enqueue_chunk(c, st, P, dt, chunk, c->stream)) != EMRKC_OK) return rc;
    if (rem > 0 && (rc = enqueue_chunk(c, st, P, dt, rem, c->stream)) != EMRKC_OK) return rc;
  }
  st->step += nsteps;
  st->t = state_time(st->t0, st->step, dt);
  set_last_stats(c, P, false);
  return EMRKC_OK;
}

// ---------------------------------------------------------------------------
// EXEX-RL reference stepping
// ---------------------------------------------------------------------------
// L steps, one kernel each; V alternates the caller's buffer and d_V1 (the
// kernel reads V^n with neighbours while writing V^{n+1}), z is updated in
// place; the chunk ends with V in the caller's buffer and the clock ticked.
static int enqueue_chunk_exexrl(emrkc_ctx *c, const emrkc_state *st, double dt, int L, hipStream_t strm) {
  double *X[2] = {(double *)st->V, c->d_V1};
  for (int n = 0; n < L; ++n) {
    ExArgs a{};
    a.Vin = X[n % 2];
    a.Vout = X[(n + 1) % 2];
    a.z = st->z;
    a.clock = c->d_clock;
    a.step_off = n;
    a.stim = stim_args(c);
    a.mp = c->mp;
    a.dt = dt;
    a.Cm = c->Cm;
    HIP_TRY(c, launch_exexrl(c->model, c->mixed, c->mesh, a, strm));
  }
  HIP_TRY(c, launch_copy_tick(L % 2 ? X[1] : nullptr, X[0], (uint32_t)c->N, c->d_clock, L, strm));
  return EMRKC_OK;
}

// ---------------------------------------------------------------------------
// IMEX-RL stepping: the pointwise part as in EXEX-RL, then the implicit
// diffusion line (I - dt F) V^{n+1} = V^n + dt S by conjugate gradients in
// the lumped-mass inner product (I - dt F is self-adjoint there), Jacobi
// preconditioned, from V^n.
// ---------------------------------------------------------------------------
constexpr double kCgTol = 1e-13;
constexpr int kCgMaxIter = 2000;

static int ensure_imexrl_data(emrkc_ctx *c) {
  int rc;
  if (!c->d_cgq && (rc = dalloc(c, (void **)&c->d_cgq, sizeof(double) * (size_t)c->N))) return rc;
  if (!c->d_cgp2 && (rc = dalloc(c, (void **)&c->d_cgp2, sizeof(double) * (size_t)c->N))) return rc;
  if (!c->d_cgpart) {
    const size_t nparts = std::max<size_t>(2 * (size_t)reduce_blocks((uint32_t)c->N), cg_apply_blocks(c->mesh));
    if ((rc = dalloc(c, (void **)&c->d_cgpart, nparts * sizeof(double)))) return rc;
  }
  if (!c->h_cgs) {
    HIP_TRY(c, hipHostMalloc((void **)&c->h_cgs, sizeof(CgScalars), hipHostMallocDefault));
    if ((rc = dalloc(c, (void **)&c->d_cgs, sizeof(CgScalars)))) return rc;
  }
  if (c->mesh.kind == kEll) {
    if (!c->d_ML) return fail(c, EMRKC_EUNSUPPORTED, "lumped mass missing");
    if (!c->d_Dsum) {
      if ((rc = dalloc(c, (void **)&c->d_Dsum, sizeof(double) * (size_t)c->N))) return rc;
      HIP_TRY(c, launch_ell_rowsum(c->mesh.ell, c->d_Dsum, c->stream));
    }
    return EMRKC_OK;
  }
  const Grid &g = c->mesh.grid;
  // every node of the tensor grid has the full set of neighbour offsets
  // (boundary neighbours mirrored): 2 per axis, 4 per face diagonal, 8 corners
  c->grid_dsum = c->dim == 3 ? 2 * (g.w[0] + g.w[1] + g.w[2]) + 4 * (g.w[3] + g.w[4] + g.w[5]) + 8 * g.w[6]
                             : 2 * (g.w[0] + g.w[1]) + 4 * g.w[3];
  if (c->d_ML) return EMRKC_OK;
  // lumped mass of the tensor grid: product over the axes of h (interior
  // node) or h/2 (end node)
  std::vector<double> ML((size_t)c->N);
  const uint32_t n[3] = {g.n0, g.n1, g.n2};
  for (uint32_t k = 0; k < n[2]; ++k)
    for (uint32_t j = 0; j < n[1]; ++j)
      for (uint32_t i = 0; i < n[0]; ++i) {
        const uint32_t ix[3] = {i, j, k};
        double m = 1.0;
        for (int d = 0; d < c->dim; ++d) m *= c->h[d] * ((ix[d] == 0 || ix[d] == n[d] - 1) ? 0.5 : 1.0);
        ML[i + (size_t)n[0] * (j + (size_t)n[1] * k)] = m;
      }
  if ((rc = dalloc(c, (void **)&c->d_ML, ML.size() * sizeof(double)))) return rc;
  HIP_TRY(c, hipMemcpy(c->d_ML, ML.data(), ML.size() * sizeof(double), hipMemcpyHostToDevice));
  return EMRKC_OK;
}

extern "C" int emrkc_imexrl_step(emrkc_ctx *c, emrkc_state *st, double dt, int64_t nsteps) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  if (!(dt > 0) || !isfinite(dt) || nsteps < 0) return fail(c, EMRKC_EINVAL, "invalid dt or nsteps");
  if (c->batch) return fail(c, EMRKC_EUNSUPPORTED, "IMEX-RL stepping is for single contexts");
  int rc;
  if ((rc = ensure_imexrl_data(c)) != EMRKC_OK) return rc;
  rebase_clock(st, dt);
  const uint32_t N = (uint32_t)c->N;
  double *x = (double *)st->V, *b = c->d_U[0], *r = c->d_U[1], *zv = c->d_U[2], *q = c->d_cgq;
  double *const P[2] = {c->d_V1, c->d_cgp2};
  c->cg_iters = 0;
  for (int64_t n = 0; n < nsteps; ++n) {
    ImexArgs a{};
    a.V = x;
    a.rhs = b;
    a.z = st->z;
    a.t = state_time(st->t0, st->step, dt);
    a.stim = stim_args(c);
    a.mp = c->mp;
    a.dt = dt;
    a.Cm = c->Cm;
    HIP_TRY(c, launch_imexrl_pre(c->model, c->mixed, N, a, c->stream));
    HIP_TRY(c, launch_cg_init(c->mesh, c->d_ML, c->d_Dsum, c->grid_dsum, dt, kCgTol * kCgTol, x, b, r, zv,
                              c->d_cgpart, c->d_cgs, c->stream));
    // enqueue as many iterations as the last solve needed (plus one), then
    // look at the flag; continue in batches until the solve is done
    int enq = 0, batch = std::max(c->cg_guess + 1, 4);
    for (;;) {
      const int k = std::min(batch, kCgMaxIter - enq);
      if (k > 0) {
        HIP_TRY(c, launch_cg_iterations(c->mesh, c->d_ML, c->d_Dsum, c->grid_dsum, dt, enq, k, x, r, zv, P, q,
                                        c->d_cgpart, c->d_cgs, c->stream));
        enq += k;
      }
      HIP_TRY(c, hipMemcpyAsync(c->h_cgs, c->d_cgs, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      const CgScalars &cs = *c->h_cgs;
      if (cs.done == 2)
        return fail(c, EMRKC_ENONFINITE, "IMEX-RL solve at step %lld: non-finite residual", (long long)st->step);
      if (cs.done == 1) {
        c->cg_guess = cs.iters;
        c->cg_iters += cs.iters;
        break;
      }
      if (enq >= kCgMaxIter)
        return fail(c, EMRKC_ENOCONV, "IMEX-RL solve at step %lld: no convergence in %d iterations",
                    (long long)st->step, kCgMaxIter);
      batch = std::max(4, enq / 2);
    }
    st->step += 1;
    st->t = state_time(st->t0, st->step, dt);
  }
  return check_finite(c, st);
}

// IMEX-RL steps with HIP events on every pointwise and vector kernel: the
// class means over the launches that did work (a solve's kernels after its
// convergence return at once and are left out).
extern "C" int emrkc_profile_imexrl(emrkc_ctx *c, emrkc_state *st, double dt, int64_t nsteps, double *ms,
                                    int64_t *counts) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  if (!(dt > 0) || !isfinite(dt) || nsteps < 1 || nsteps > 10000) return fail(c, EMRKC_EINVAL, "invalid dt or nsteps");
  if (c->batch) return fail(c, EMRKC_EUNSUPPORTED, "IMEX-RL stepping is for single contexts");
  int rc;
  if ((rc = ensure_imexrl_data(c)) != EMRKC_OK) return rc;
  rebase_clock(st, dt);
  const uint32_t N = (uint32_t)c->N;
  double *x = (double *)st->V, *b = c->d_U[0], *r = c->d_U[1], *zv = c->d_U[2], *q = c->d_cgq;
  double *const P[2] = {c->d_V1, c->d_cgp2};
  // classes: 0 pointwise (k_imexrl_pre), 1 k_cg_init, 2 direction and
  // operator (k_cg_dir_apply_*), 3 k_cg_update
  KernelTimer tm;
  double sum[4] = {0, 0, 0, 0};
  int64_t cnt[4] = {0, 0, 0, 0};
  auto body = [&]() -> int {
    for (int64_t n = 0; n < nsteps; ++n) {
      ImexArgs a{};
      a.V = x;
      a.rhs = b;
      a.z = st->z;
      a.t = state_time(st->t0, st->step, dt);
      a.stim = stim_args(c);
      a.mp = c->mp;
      a.dt = dt;
      a.Cm = c->Cm;
      KernelTimer *T = &tm;
      {
        KernelTimer *tm = T;
        TIMED(0, launch_imexrl_pre(c->model, c->mixed, N, a, c->stream));
        TIMED(1, launch_cg_init(c->mesh, c->d_ML, c->d_Dsum, c->grid_dsum, dt, kCgTol * kCgTol, x, b, r, zv,
                                c->d_cgpart, c->d_cgs, c->stream));
      }
      // one iteration at a time, so that every timed launch did work
      for (int it = 0;; ++it) {
        HIP_TRY(c, hipMemcpyAsync(c->h_cgs, c->d_cgs, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (c->h_cgs->done == 2) return fail(c, EMRKC_ENONFINITE, "IMEX-RL solve: non-finite residual");
        if (c->h_cgs->done == 1) break;
        if (it >= kCgMaxIter) return fail(c, EMRKC_ENOCONV, "IMEX-RL solve: no convergence");
        for (int w = 0; w < kCgLaunches; ++w) {
          const int cls = w == kCgApply ? 2 : w == kCgUpdate ? 3 : -1;  // the one-block reductions untimed
          KernelTimer *tm = cls >= 0 ? T : nullptr;
          TIMED(cls, launch_cg_step(w, c->mesh, c->d_ML, c->d_Dsum, c->grid_dsum, dt, x, r, zv, P[it & 1],
                                    P[(it + 1) & 1], q, c->d_cgpart, c->d_cgs, c->stream));
        }
      }
      st->step += 1;
      st->t = state_time(st->t0, st->step, dt);
    }
    return EMRKC_OK;
  };
  rc = body();
  hipError_t e = hipStreamSynchronize(c->stream);
  if (rc == EMRKC_OK && e == hipSuccess) {
    for (size_t k = 0; k + 1 < tm.used; k += 2) {
      float t_ms = 0;
      if (hipEventElapsedTime(&t_ms, tm.ev[k], tm.ev[k + 1]) != hipSuccess) {
        rc = fail(c, EMRKC_EHIP, "hipEventElapsedTime failed");
        break;
      }
      const int cl = tm.cls[k / 2];
      sum[cl] += t_ms;
      cnt[cl] += 1;
    }
  }
  for (hipEvent_t ev : tm.ev) (void)hipEventDestroy(ev);
  if (e != hipSuccess) return fail(c, EMRKC_EHIP, "profiled steps failed: %s", hipGetErrorString(e));
  if (rc != EMRKC_OK) return rc;
  for (int k = 0; k < 4; ++k) {
    if (ms) ms[k] = cnt[k] ? sum[k] / (double)cnt[k] : 0.0;
    if (counts) counts[k] = cnt[k];
  }
  return check_finite(c, st);
}

extern "C" int64_t emrkc_imexrl_iterations(const emrkc_ctx *c) { return c ? c->cg_iters : -1; }

extern "C" int emrkc_exexrl_step(emrkc_ctx *c, emrkc_state *st, double dt, int64_t nsteps) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  if (!(dt > 0) || !isfinite(dt) || nsteps < 0) return fail(c, EMRKC_EINVAL, "invalid dt or nsteps");
  if (c->batch) return fail(c, EMRKC_EUNSUPPORTED, "EXEX-RL stepping is for single contexts");
  if (nsteps == 0) return EMRKC_OK;
  rebase_clock(st, dt);
  bool used_graph = false;
  const int rc = run_chunks(c, st, dt, nsteps, -1, 0,
                            [&](int L, hipStream_t strm) { return enqueue_chunk_exexrl(c, st, dt, L, strm); },
                            &used_graph);
  if (rc != EMRKC_OK) return rc;
  st->step += nsteps;
  st->t = state_time(st->t0, st->step, dt);
  return check_finite(c, st);
}

int KernelTimer::arm(emrkc_ctx *c, int k) {
  while (ev.size() < used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return fail(c, EMRKC_EHIP, "hipEventCreate failed");
    ev.push_back(e);
  }
  cls.push_back(k);
  set_launch_events(ev[used], ev[used + 1]);
  used += 2;
  return EMRKC_OK;
}

extern "C" int emrkc_profile_step(emrkc_ctx *c, emrkc_state *st, double dt, int64_t nsteps, double *ms,
                                  int64_t *counts) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  if (!(dt > 0) || !isfinite(dt) || nsteps < 1 || nsteps > 100000) return fail(c, EMRKC_EINVAL, "invalid dt or nsteps");
  if (!c->have_rho) return fail(c, EMRKC_EINVAL, "spectral radii not set");
  StepPlan P;
  int rc = make_plan(c, dt, P);
  if (rc != EMRKC_OK) return rc;
  rebase_clock(st, dt);
  HIP_TRY(c, launch_clock_set(c->d_clock, st->step, st->t0, c->stream));
  KernelTimer tm;
  bool zb = false;
  if ((rc = zblocks_begin(c, st, P, &zb)) != EMRKC_OK) return rc;
  if (c->batch && (rc = build_batch_tables(c, st, dt, P)) != EMRKC_OK) {
    (void)zblocks_end(c, st, zb);
    return rc;
  }
  rc = enqueue_chunk(c, st, P, dt, (int)nsteps, c->stream, &tm);
  const int rc_end = zblocks_end(c, st, zb);
  if (rc == EMRKC_OK) rc = rc_end;
  hipError_t e = hipStreamSynchronize(c->stream);
  double sum[3] = {0, 0, 0};
  int64_t cnt[3] = {0, 0, 0};
  if (rc == EMRKC_OK && e == hipSuccess) {
    for (size_t k = 0; k + 1 < tm.used; k += 2) {
      float t_ms = 0;
      if (hipEventElapsedTime(&t_ms, tm.ev[k], tm.ev[k + 1]) != hipSuccess) {
        rc = fail(c, EMRKC_EHIP, "hipEventElapsedTime failed");
        break;
      }
      const int cl = tm.cls[k / 2];
      sum[cl] += t_ms;
      cnt[cl] += 1;
    }
  }
  for (hipEvent_t ev : tm.ev) (void)hipEventDestroy(ev);
  if (e != hipSuccess) return fail(c, EMRKC_EHIP, "profiled steps failed: %s", hipGetErrorString(e));
  if (rc != EMRKC_OK) return rc;
  st->step += nsteps;
  st->t = state_time(st->t0, st->step, dt);
  for (int k = 0; k < 3; ++k) {
    if (ms) ms[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
    if (counts) counts[k] = cnt[k];
  }
  return EMRKC_OK;
}

// ---------------------------------------------------------------------------
// Timing on a private copy of a state
// ---------------------------------------------------------------------------
struct StateCopy {
  void *V = nullptr, *Z = nullptr;
  emrkc_state st{};
  ~StateCopy() {
    if (V) (void)hipFree(V);
    if (Z) (void)hipFree(Z);
  }
};

static int copy_state(emrkc_ctx *c, const emrkc_state *src, StateCopy &cp) {
  const size_t vb = (size_t)c->N * sizeof(double);
  const size_t zb = (size_t)(c->nv - 1) * (size_t)c->N * (c->mixed ? sizeof(float) : sizeof(double));
  if (hipMalloc(&cp.V, vb) != hipSuccess || hipMalloc(&cp.Z, zb) != hipSuccess)
    return fail(c, EMRKC_ENOMEM, "no memory for a copy of the state");
  if (hipMemcpyAsync(cp.V, src->V, vb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(cp.Z, src->z, zb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, EMRKC_EHIP, "state copy failed");
  cp.st = *src;
  cp.st.V = cp.V;
  cp.st.z = cp.Z;
  return EMRKC_OK;
}

// ---------------------------------------------------------------------------
// Kernel shapes of 3-D grids and their autotuning
// ---------------------------------------------------------------------------
// Kernel shapes: variants[5] = {head kernel, head planes per column, inner
// kernel, inner planes per column, fused tail+head}.
static bool tunable(const emrkc_ctx *c) {  // the 3-D shapes (emRKC)
  return !c->batch && c->mesh.kind == kGrid && c->dim == 3 && !c->flat && c->method == EMRKC_METHOD_EMRKC;
}
static bool planar(const emrkc_ctx *c) {  // 2-D grids: inner shape 0 (tiles) or 2 (all stages in one launch)
  return !c->batch && c->mesh.kind == kGrid && c->dim == 2 && !c->flat && c->method == EMRKC_METHOD_EMRKC;
}
static bool fusable(const emrkc_ctx *c) {  // the fused kernel (emRKC, used when s == 1 and m >= 2)
  return !c->batch && !c->flat && fused_supported(c->mesh) && c->method == EMRKC_METHOD_EMRKC;
}

static void get_variants(const emrkc_ctx *c, int *v) {
  if (c->batch) {
    v[0] = c->batch_shape;
    v[1] = c->batch_flat_head ? 1 : 0;
    v[2] = c->batch_march_zc > 0 ? 1 : c->batch_pairs ? 2 : 0;
    v[3] = c->batch_march_zc;
    v[4] = 0;
    return;
  }
  const Grid &g = c->mesh.grid;
  const bool t = tunable(c);
  v[0] = t ? g.head_variant : 0;
  v[1] = t && (g.head_variant == 1 || g.head_variant == 2 || g.head_variant == 7) ? (int)g.head_zc : 0;
  v[2] = t || planar(c) ? g.inner_variant : 0;
  v[3] = t && g.inner_variant ? (int)g.zc : 0;
  v[4] = c->use_fused ? 1 : 0;
}

static int check_variants(const emrkc_ctx *c, const int *v) {
  if (c->batch) {
    if (v[0] < 0 || v[0] > 2 || v[1] < 0 || v[1] > 1 || v[2] < 0 || v[2] > 2) return EMRKC_EINVAL;
    if (v[2] == 1 && (v[3] < 1 || v[3] > 64)) return EMRKC_EINVAL;  // planes per marching column
    if (v[2] != 1 && v[3] != 0) return EMRKC_EINVAL;
    return v[4] == 0 ? EMRKC_OK : EMRKC_EUNSUPPORTED;
  }
  if (v[4] < 0 || v[4] > 1 || (v[4] == 1 && !fusable(c))) return EMRKC_EUNSUPPORTED;
  if (planar(c)) {
    if ((v[0] | v[1] | v[3]) != 0 || (v[2] != 0 && (v[2] < 2 || v[2] > 4))) return EMRKC_EUNSUPPORTED;
    return v[2] != 0 && v[4] != 0 ? EMRKC_EINVAL : EMRKC_OK;  // one or the other
  }
  if (!tunable(c)) return (v[0] | v[1] | v[2] | v[3]) == 0 ? EMRKC_OK : EMRKC_EUNSUPPORTED;
  const int n2 = (int)c->mesh.grid.n2;
  if (v[0] < 0 || v[0] > 8 || v[2] < 0 || v[2] > 1) return EMRKC_EINVAL;
  if (v[0] == 6 && !c->mixed) return EMRKC_EUNSUPPORTED;       // a mixed-precision kernel
  if (v[0] >= 7 && v[4] != 0) return EMRKC_EINVAL;             // the split stage replaces the fused kernel
  // the LDS-staged head addresses a component plane with 32-bit byte offsets
  if (v[0] == 2 && (uint64_t)c->N * sizeof(double) >= (1ull << 32)) return EMRKC_EUNSUPPORTED;
  const bool head_cols = v[0] == 1 || v[0] == 2 || v[0] == 7;
  if (head_cols && (v[1] < 1 || v[1] > 64 || v[1] > n2)) return EMRKC_EINVAL;
  if (v[2] != 0 && (v[3] < 1 || v[3] > 64 || v[3] > n2)) return EMRKC_EINVAL;
  if (!head_cols && v[1] != 0) return EMRKC_EINVAL;
  if (v[2] == 0 && v[3] != 0) return EMRKC_EINVAL;
  return EMRKC_OK;
}

static void set_variants(emrkc_ctx *c, const int *v) {
  if (c->batch) {
    c->batch_shape = v[0];
    c->batch_flat_head = v[1] != 0;
    c->batch_march_zc = v[2] == 1 ? v[3] : 0;
    c->batch_pairs = v[2] == 2;
    clear_graphs(c);
    return;
  }
  if (planar(c)) c->mesh.grid.inner_variant = v[2];
  if (tunable(c)) {
    Grid &g = c->mesh.grid;
    g.head_variant = v[0];
    g.head_zc = (v[0] == 1 || v[0] == 2 || v[0] == 7) ? (uint32_t)v[1] : 1u;
    g.inner_variant = v[2];
    g.zc = v[2] ? (uint32_t)v[3] : 1u;
  }
  c->use_fused = v[4] != 0;
  clear_graphs(c);
}

extern "C" int emrkc_get_variants(const emrkc_ctx *c, int *variants) {
  if (c == nullptr || variants == nullptr) return EMRKC_EINVAL;
  get_variants(c, variants);
  return EMRKC_OK;
}

extern "C" int emrkc_set_variants(emrkc_ctx *c, const int *variants) {
  if (c == nullptr || variants == nullptr) return EMRKC_EINVAL;
  const int rc = check_variants(c, variants);
  if (rc != EMRKC_OK)
    return fail(c, rc, "kernel variants (%d,%d,%d,%d,%d) not valid for this context", variants[0], variants[1],
                variants[2], variants[3], variants[4]);
  set_variants(c, variants);
  return EMRKC_OK;
}

// Mean duration per launch of the head (0), inner (1) and fused (2) kernels
// over `reps` steps on state `st` (advanced).
static int time_classes(emrkc_ctx *c, emrkc_state *st, const StepPlan &P, double dt, int reps, double *ms) {
  HIP_TRY(c, launch_clock_set(c->d_clock, st->step, st->t0, c->stream));
  bool zb = false;
  int rc = zblocks_begin(c, st, P, &zb);  // the z layout emrkc_step would use
  if (rc != EMRKC_OK) return rc;
  if (c->batch) rc = build_batch_tables(c, st, dt, P);
  if (rc == EMRKC_OK) rc = enqueue_chunk(c, st, P, dt, 1, c->stream, nullptr);  // untimed: first launches
  KernelTimer tm;
  if (rc == EMRKC_OK) rc = enqueue_chunk(c, st, P, dt, reps, c->stream, &tm);
  const int rc_end = zblocks_end(c, st, zb);
  if (rc == EMRKC_OK) rc = rc_end;
  hipError_t e = hipStreamSynchronize(c->stream);
  double sum[3] = {0, 0, 0};
  int cnt[3] = {0, 0, 0};
  if (rc == EMRKC_OK && e == hipSuccess) {
    for (size_t k = 0; k + 1 < tm.used; k += 2) {
      float t_ms = 0;
      if (hipEventElapsedTime(&t_ms, tm.ev[k], tm.ev[k + 1]) != hipSuccess) {
        rc = fail(c, EMRKC_EHIP, "hipEventElapsedTime failed");
        break;
      }
      sum[tm.cls[k / 2]] += t_ms;
      cnt[tm.cls[k / 2]] += 1;
    }
  }
  for (hipEvent_t ev : tm.ev) (void)hipEventDestroy(ev);
  if (e != hipSuccess) return fail(c, EMRKC_EHIP, "autotuning steps failed: %s", hipGetErrorString(e));
  if (rc != EMRKC_OK) return rc;
  for (int k = 0; k < 3; ++k) ms[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
  return EMRKC_OK;
}

// time_classes over `rounds` repetitions, the fastest per class: a single
// slow repetition (a clock or memory transient) does not decide a choice.
static int time_classes_best(emrkc_ctx *c, emrkc_state *st, const StepPlan &P, double dt, int reps, double *ms,
                             int rounds = 2) {
  double best[3] = {0, 0, 0};
  for (int r = 0; r < rounds; ++r) {
    double t[3];
    const int rc = time_classes(c, st, P, dt, reps, t);
    if (rc != EMRKC_OK) return rc;
    for (int k = 0; k < 3; ++k) best[k] = r == 0 ? t[k] : std::min(best[k], t[k]);
  }
  for (int k = 0; k < 3; ++k) ms[k] = best[k];
  return EMRKC_OK;
}

// Batched ensembles: the three tile shapes, compared by the time per step
// (one head launch and m_max - 1 inner launches).
static int autotune_batch(emrkc_ctx *c, const emrkc_state *st, double dt, int reps, const StepPlan &P,
                          int *variants) {
  int orig[5];
  get_variants(c, orig);
  StateCopy cp;
  int rc = copy_state(c, st, cp);
  if (rc != EMRKC_OK) return rc;
  const bool verbose = getenv("EMRKC_VERBOSE") != nullptr;
  // each choice compares the kernels it changes: the tile shape (tiled
  // head and inner tiles) by the time per step, the flat head by the head's
  // time, and marching columns for the 3-D instances by the inner stage's
  double best = 1e300, head_t = 0, inner_t = 0;
  int choice = orig[0];
  for (int shape = 0; shape < 3 && rc == EMRKC_OK; ++shape) {
    const int v[5] = {shape, 0, 0, 0, 0};
    set_variants(c, v);
    double ms[3];
    if ((rc = time_classes_best(c, &cp.st, P, dt, reps, ms)) != EMRKC_OK) break;
    const double step = ms[0] + (P.m - 1) * ms[1];
    if (verbose)
      fprintf(stderr, "emrkc_autotune: batch tiles %d: head %.5f ms, inner %.5f ms, step %.5f ms\n", shape, ms[0],
              ms[1], step);
    if (step < 0.97 * best) {
      best = step;
      choice = shape;
      head_t = ms[0];
      inner_t = ms[1];
    }
  }
  // the flat head with the chosen tiles for the inner stages
  int flat = 0;
  if (rc == EMRKC_OK) {
    const int v[5] = {choice, 1, 0, 0, 0};
    set_variants(c, v);
    double ms[3];
    if ((rc = time_classes_best(c, &cp.st, P, dt, reps, ms)) == EMRKC_OK) {
      if (verbose) fprintf(stderr, "emrkc_autotune: batch flat head: head %.5f ms (tiled %.5f ms)\n", ms[0], head_t);
      if (ms[0] < 0.97 * head_t) flat = 1;
    }
  }
  // inner stages with two tiles per block
  double best_in = inner_t;
  int pairs = 0;
  if (rc == EMRKC_OK && P.m >= 2) {
    const int v[5] = {choice, flat, 2, 0, 0};
    set_variants(c, v);
    double ms[3];
    if ((rc = time_classes_best(c, &cp.st, P, dt, reps, ms)) == EMRKC_OK) {
      if (verbose) fprintf(stderr, "emrkc_autotune: batch two tiles per block: inner %.5f ms (tiles %.5f ms)\n", ms[1],
                           inner_t);
      if (ms[1] < 0.97 * best_in) {
        best_in = ms[1];
        pairs = 1;
      }
    }
  }
  // inner stages of 3-D instances by z-marching columns (zc planes; 64 =
  // whole columns)
  int zc_choice = 0;
  bool any3d = false;
  for (auto &I : c->inst) any3d = any3d || I.mesh.grid.dim == 3;
  for (int zc : {4, 8, 64}) {
    if (rc != EMRKC_OK || !any3d || P.m < 2) break;
    const int v[5] = {choice, flat, 1, zc, 0};
    set_variants(c, v);
    double ms[3];
    if ((rc = time_classes_best(c, &cp.st, P, dt, reps, ms)) != EMRKC_OK) break;
    if (verbose)
      fprintf(stderr, "emrkc_autotune: batch marching columns of %d planes: inner %.5f ms (tiles %.5f ms)\n", zc,
              ms[1], inner_t);
    if (ms[1] < 0.97 * best_in) {
      best_in = ms[1];
      zc_choice = zc;
    }
  }
  (void)hipStreamSynchronize(c->stream);
  const int mode = zc_choice ? 1 : pairs ? 2 : 0;
  const int v[5] = {rc == EMRKC_OK ? choice : orig[0], rc == EMRKC_OK ? flat : orig[1], rc == EMRKC_OK ? mode : orig[2],
                    rc == EMRKC_OK ? zc_choice : orig[3], 0};
  set_variants(c, v);
  c->bdev.valid = false;  // the tables point into the state copy
  if (rc == EMRKC_OK && variants) get_variants(c, variants);
  return rc;
}

// Wall time per step of `reps` eagerly launched steps on state st
// (advanced), launch gaps included: what decides on small, launch-bound
// grids.
static int time_steps(emrkc_ctx *c, emrkc_state *st, const StepPlan &P, double dt, int reps, double *ms) {
  HIP_TRY(c, launch_clock_set(c->d_clock, st->step, st->t0, c->stream));
  bool zb = false;
  int rc = zblocks_begin(c, st, P, &zb);  // the z layout emrkc_step would use
  if (rc != EMRKC_OK) return rc;
  if (c->batch) rc = build_batch_tables(c, st, dt, P);
  if (rc == EMRKC_OK) rc = enqueue_chunk(c, st, P, dt, 2, c->stream, nullptr);  // untimed: first launches
  if (rc != EMRKC_OK) {
    (void)zblocks_end(c, st, zb);
    return rc;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) {
    (void)zblocks_end(c, st, zb);
    return fail(c, EMRKC_EHIP, "hipEventCreate failed");
  }
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    (void)zblocks_end(c, st, zb);
    return fail(c, EMRKC_EHIP, "hipEventCreate failed");
  }
  hipError_t e = hipEventRecord(e0, c->stream);
  if (e == hipSuccess) {
    rc = enqueue_chunk(c, st, P, dt, reps, c->stream, nullptr);
    e = hipEventRecord(e1, c->stream);
  }
  const int rc_end = zblocks_end(c, st, zb);
  if (rc == EMRKC_OK) rc = rc_end;
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0;
  if (e == hipSuccess && rc == EMRKC_OK) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(c, EMRKC_EHIP, "autotuning steps failed: %s", hipGetErrorString(e));
  if (rc != EMRKC_OK) return rc;
  *ms = t / reps;
  return EMRKC_OK;
}

// 2-D grids: separate inner-stage launches (the default), the fused kernel
// (s == 1) and all inner stages in one launch, compared by the wall time of
// a run of steps; a later candidate must be 3% faster to replace the choice.
static int autotune_planar(emrkc_ctx *c, const emrkc_state *st, double dt, int reps, const StepPlan &P,
                           int *variants) {
  int orig[5];
  get_variants(c, orig);
  StateCopy cp;
  int rc = copy_state(c, st, cp);
  if (rc != EMRKC_OK) return rc;
  const bool verbose = getenv("EMRKC_VERBOSE") != nullptr;
  std::vector<std::array<int, 5>> cands{{0, 0, 0, 0, 0}, {0, 0, 2, 0, 0}, {0, 0, 3, 0, 0}};
  if (P.s == 1) cands.push_back({0, 0, 4, 0, 0});
  if (fusable(c) && P.s == 1) cands.push_back({0, 0, 0, 0, 1});
  double best = 1e300;
  std::array<int, 5> choice = cands[0];
  for (const auto &v : cands) {
    set_variants(c, v.data());
    double ms = 0;
    if ((rc = time_steps(c, &cp.st, P, dt, reps, &ms)) != EMRKC_OK) break;
    if (verbose)
      fprintf(stderr, "emrkc_autotune: 2-D shapes (%d,%d,%d,%d,%d): %.5f ms per step\n", v[0], v[1], v[2], v[3], v[4],
              ms);
    if (ms < 0.97 * best) {
      best = ms;
      choice = v;
    }
  }
  (void)hipStreamSynchronize(c->stream);
  set_variants(c, rc == EMRKC_OK ? choice.data() : orig);
  if (rc == EMRKC_OK && variants) get_variants(c, variants);
  return rc;
}

extern "C" int emrkc_autotune(emrkc_ctx *c, const emrkc_state *st, double dt, int reps, int *variants) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  if (!(dt > 0) || !isfinite(dt) || reps < 1 || reps > 1000) return fail(c, EMRKC_EINVAL, "invalid dt or reps");
  if (!c->have_rho) return fail(c, EMRKC_EINVAL, "spectral radii not set");
  StepPlan P;
  int rc = make_plan(c, dt, P);
  if (rc != EMRKC_OK) return rc;
  if (c->batch) return autotune_batch(c, st, dt, reps, P, variants);
  if (planar(c) && inner_all_supported(c->mesh, P.m)) return autotune_planar(c, st, dt, reps, P, variants);
  const bool fuse_ok = fusable(c) && P.s == 1 && P.m >= 2;
  if (!tunable(c) && !fuse_ok) return emrkc_get_variants(c, variants);
  // shape candidates (3-D grids): 3-D tiles, and z-marching columns of zc
  // planes for every zc in {2, 3, 4, 8, 16, 32} that leaves at least one
  // block per compute unit
  // the flat head (the default) is the first head candidate: another shape
  // must beat it by the margin below
  std::vector<std::pair<int, int>> heads{{5, 0}}, inners{{0, 0}};
  if (tunable(c)) {
    if (c->mixed) heads.push_back({6, 0});  // the flat head for 7 waves per SIMD
    heads.push_back({0, 0});  // tiles; and tiles for 6 and 8 waves per SIMD
    heads.push_back({3, 0});
    heads.push_back({4, 0});
    const Grid &g = c->mesh.grid;
    const uint32_t cols = ((g.n0 + MX - 1) / MX) * ((g.n1 + MY - 1) / MY);
    const bool lds_ok = (uint64_t)c->N * sizeof(double) < (1ull << 32);
    for (int zc : {2, 3, 4, 8, 16, 32}) {
      if (zc > (int)g.n2 || cols * ((g.n2 + zc - 1) / zc) < 256) continue;
      heads.push_back({1, zc});
      if (lds_ok) heads.push_back({2, zc});
      inners.push_back({1, zc});
    }
  }
  int orig[5];
  get_variants(c, orig);
  // timing runs on a copy of the state
  StateCopy cp;
  if ((rc = copy_state(c, st, cp)) != EMRKC_OK) return rc;
  const bool verbose = getenv("EMRKC_VERBOSE") != nullptr;
  double best_h = 1e300, best_i = 1e300;
  int choice[5] = {orig[0], orig[1], orig[2], orig[3], 0};
  const size_t ncand = std::max(heads.size(), inners.size());
  for (size_t k = 0; k < ncand && rc == EMRKC_OK && tunable(c); ++k) {
    const auto hv = heads[k % heads.size()], iv = inners[k % inners.size()];
    const int v[5] = {hv.first, hv.second, iv.first, iv.second, 0};
    set_variants(c, v);
    double ms[3];
    rc = time_classes_best(c, &cp.st, P, dt, reps, ms);
    if (rc != EMRKC_OK) break;
    if (verbose)
      fprintf(stderr, "emrkc_autotune: head %d/%d %.5f ms, inner %d/%d %.5f ms\n", v[0], v[1], ms[0], v[2], v[3],
              ms[1]);
    // a later candidate must be faster by 3% to replace the current choice
    // (the first candidates are the flat head and the tiled inner stage), so
    // that timing noise does not pick among near-equals
    if (ms[0] > 0 && ms[0] < 0.97 * best_h) {
      best_h = ms[0];
      choice[0] = v[0];
      choice[1] = v[1];
    }
    if (ms[1] > 0 && ms[1] < 0.97 * best_i) {
      best_i = ms[1];
      choice[2] = v[2];
      choice[3] = v[3];
    }
  }
  // the split stage (m >= 2): the pointwise head and the two-stage inner
  // kernel with columns of zc planes, compared by the time per step
  bool split_chosen = false;
  if (rc == EMRKC_OK && tunable(c) && P.m >= 2) {
    const double plain = best_h + (P.m - 1) * best_i;
    double best_split = 1e300;
    int best_zc = 0;
    const Grid &g = c->mesh.grid;
    const uint32_t cols = ((g.n0 + MX - 1) / MX) * ((g.n1 + MY - 1) / MY);
    for (int zc : {4, 8, 16, 32, 64}) {
      if (zc > (int)g.n2 || cols * ((g.n2 + zc - 1) / zc) < 256) continue;
      const int vs[5] = {7, zc, choice[2], choice[3], 0};
      set_variants(c, vs);
      double ms[3];
      rc = time_classes_best(c, &cp.st, P, dt, reps, ms);
      if (rc != EMRKC_OK) break;
      const double step = ms[0] + (P.m - 1) * ms[1];
      if (verbose)
        fprintf(stderr, "emrkc_autotune: split %d planes: head %.5f ms, inner %.5f ms, step %.5f ms (separate %.5f)\n",
                zc, ms[0], ms[1], step, plain);
      if (step < best_split) {
        best_split = step;
        best_zc = zc;
      }
    }
    // shape 8: the pointwise head and u_1 as a launch of the inner kernel,
    // whose shape is chosen here by the mean of the u_1 and tail launches
    // (the first pass chose it by the tail alone); the head is the same
    // kernel for every candidate, so its fastest time enters the step
    double head8 = 1e300, inner8 = 1e300;
    int in8[2] = {choice[2], choice[3]};
    for (size_t k = 0; k < inners.size() && rc == EMRKC_OK; ++k) {
      const int v8[5] = {8, 0, inners[k].first, inners[k].second, 0};
      set_variants(c, v8);
      double ms[3];
      rc = time_classes_best(c, &cp.st, P, dt, reps, ms);
      if (rc != EMRKC_OK) break;
      if (verbose)
        fprintf(stderr, "emrkc_autotune: split with u_1 launch, inner %d/%d: head %.5f ms, inner %.5f ms\n", v8[2],
                v8[3], ms[0], ms[1]);
      head8 = std::min(head8, ms[0]);
      if (ms[1] < inner8) {
        inner8 = ms[1];
        in8[0] = v8[2];
        in8[1] = v8[3];
      }
    }
    const double step8 = head8 + P.m * inner8;
    if (verbose && rc == EMRKC_OK)
      fprintf(stderr, "emrkc_autotune: split with u_1 launch: step %.5f ms (separate %.5f)\n", step8, plain);
    // The sums above are of per-kernel minima over many candidates, each
    // biased low by its own selection; where the best split is within 3%
    // of the separate stages the two are timed head to head instead, as
    // whole steps (alternating, the fastest of three runs each), and the
    // faster is kept.
    if (rc == EMRKC_OK && std::min(best_split, step8) < 1.03 * plain) {
      int vs[5] = {8, 0, in8[0], in8[1], 0};
      if (step8 > best_split) {
        vs[0] = 7;
        vs[1] = best_zc;
        vs[2] = choice[2];
        vs[3] = choice[3];
      }
      const int vp[5] = {choice[0], choice[1], choice[2], choice[3], 0};
      double tp = 1e300, ts = 1e300;
      for (int r = 0; r < 3 && rc == EMRKC_OK; ++r) {
        double t;
        set_variants(c, vp);
        if ((rc = time_steps(c, &cp.st, P, dt, reps, &t)) != EMRKC_OK) break;
        tp = std::min(tp, t);
        set_variants(c, vs);
        if ((rc = time_steps(c, &cp.st, P, dt, reps, &t)) != EMRKC_OK) break;
        ts = std::min(ts, t);
      }
      if (verbose && rc == EMRKC_OK)
        fprintf(stderr, "emrkc_autotune: whole steps: split %d/%d %.5f ms, separate %.5f ms\n", vs[0], vs[1], ts,
                tp);
      if (rc == EMRKC_OK && ts < tp) {
        for (int k = 0; k < 5; ++k) choice[k] = vs[k];
        split_chosen = true;
      }
    }
  }
  // fused tail+head (s == 1, m >= 2): one kernel per step in place of the
  // head and the last inner stage; compared by the time per step
  if (rc == EMRKC_OK && fuse_ok && !split_chosen) {
    double ms[3];
    choice[4] = 0;
    set_variants(c, choice);
    if (!tunable(c)) {
      rc = time_classes_best(c, &cp.st, P, dt, reps, ms);
      best_h = ms[0];
      best_i = ms[1];
    }
    if (rc == EMRKC_OK) {
      const int vf[5] = {choice[0], choice[1], choice[2], choice[3], 1};
      set_variants(c, vf);
      rc = time_classes_best(c, &cp.st, P, dt, reps, ms);
      if (rc == EMRKC_OK) {
        const double plain = best_h + (P.m - 1) * best_i, fused = ms[2] + (P.m - 2) * ms[1];
        if (verbose)
          fprintf(stderr, "emrkc_autotune: step %.5f ms separate, %.5f ms fused (fused kernel %.5f ms)\n", plain,
                  fused, ms[2]);
        choice[4] = fused < 0.97 * plain ? 1 : 0;
      }
    }
  }
  (void)hipStreamSynchronize(c->stream);
  set_variants(c, rc == EMRKC_OK ? choice : orig);
  if (rc == EMRKC_OK && variants) get_variants(c, variants);
  return rc;
}

// ---------------------------------------------------------------------------
// Nonlinear power iteration (appendix, Compute_Rho)
// ---------------------------------------------------------------------------
static int fetch(emrkc_ctx *c, double *out) {
  HIP_TRY(c, hipMemcpyAsync(out, c->d_result, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return EMRKC_OK;
}

// One instance seen by the power iteration: its operator, its node range
// (component planes `stride` apart) and its warm-start data.  The warm
// vectors live in two buffers; sel says which one holds the current v.
struct RhoView {
  Mesh mesh;
  uint32_t N;
  size_t stride;
  const double *V;
  const void *z;
  StimArgs stim;
  double Cm;
  double *vF[2], *vS[2], *zV;
  int *selF, *selS;
  bool *warm_F, *warm_S;
  double *raw_F, *raw_S, *nv_F, *nv_S;
};

// Compute_Rho of the appendix for f_F and f_S of one instance.
static int estimate_view(emrkc_ctx *c, const RhoView &v, double t, int *iters_F, int *iters_S, bool *noconv) {
  int rc;
  double ny2 = 0;
  HIP_TRY(c, launch_norm2_state(c->mixed, v.N, v.stride, c->nv - 1, v.V, v.z, c->d_partials, c->d_result, c->stream));
  if ((rc = fetch(c, &ny2))) return rc;
  const double ny = sqrt(ny2);
  const double delta = ny > 0 ? ny * c->pi_eps : c->pi_eps;
  for (int which = 0; which < 2; ++which) {
    bool &warm = which == 0 ? *v.warm_F : *v.warm_S;
    int &sel = which == 0 ? *v.selF : *v.selS;
    double *const *buf = which == 0 ? v.vF : v.vS;
    double &raw = which == 0 ? *v.raw_F : *v.raw_S;
    double &nvs = which == 0 ? *v.nv_F : *v.nv_S;
    double nv;
    if (warm) {
      nv = nvs;
    } else {
      double s2;
      HIP_TRY(c, launch_norm2_random(c->pi_seed, (uint64_t)v.N * c->nv, c->d_partials, c->d_result, c->stream));
      if ((rc = fetch(c, &s2))) return rc;
      nv = sqrt(s2);
    }
    double q = delta / nv, rho = warm ? raw : 0.0, rho_old = 0.0;
    int it = 0;
    while (fabs(rho - rho_old) >= c->pi_tol * rho) {
      if (it >= c->pi_max_iter) {
        *noconv = true;
        break;
      }
      rho_old = rho;
      const double *vin = warm ? buf[sel] : nullptr;
      double *vout = buf[1 - sel];
      if (which == 0) {
        // only the V component of v enters f_F(y + q v) - f_F(y)
        HIP_TRY(c, launch_powF_shift(v.N, v.V, vin, c->pi_seed, q, v.zV, c->stream));
        HIP_TRY(c, launch_powF_diff(c->mixed, v.mesh, v.zV, v.V, vout, c->d_partials, c->d_result, c->stream));
      } else {
        // f_S on (V, z_E, z_S); the gate components of f_S vanish
        HIP_TRY(c, launch_powS_iter(c->model, c->mixed, v.N, v.stride, v.V, v.z, vin, c->pi_seed, q, t, v.stim, v.Cm,
                                    c->mp, vout, c->d_partials, c->d_result, c->stream));
      }
      double s2;
      if ((rc = fetch(c, &s2))) return rc;
      sel = 1 - sel;
      warm = true;
      nv = sqrt(s2);
      ++it;
      if (nv == 0.0) {
        rho = 0.0;
        break;
      }
      q = delta / nv;
      rho = nv / delta;
    }
    raw = rho;
    nvs = nv;
    if (which == 0 && iters_F) *iters_F = it;
    if (which == 1 && iters_S) *iters_S = it;
  }
  return EMRKC_OK;
}

static int alloc_rho_buffers(emrkc_ctx *c) {
  if (c->d_vF[0]) return EMRKC_OK;
  const size_t vb = sizeof(double) * (size_t)c->N;
  int rc;
  if ((rc = dalloc(c, (void **)&c->d_vF[0], vb)) || (rc = dalloc(c, (void **)&c->d_vF[1], vb)) ||
      (rc = dalloc(c, (void **)&c->d_zV, vb)) || (rc = dalloc(c, (void **)&c->d_vS[0], vb * (1 + c->ns))) ||
      (rc = dalloc(c, (void **)&c->d_vS[1], vb * (1 + c->ns))))
    return rc;
  return EMRKC_OK;
}

// ---- mRKC: the power iteration on full-state vectors ----------------------
// Compute_Rho of the appendix applied to f~_F and f~_S as whole right-hand
// sides: vectors of all n_v N components (zero where a term has no
// component), the same splitmix64 start over all of them, and the warm
// start kept per term.
static int mrkc_buffers(emrkc_ctx *c) {
  if (c->d_Y) return EMRKC_OK;
  const uint64_t n = (uint64_t)c->nv * (uint64_t)c->N;
  if (n >= (1ull << 32)) return fail(c, EMRKC_EUNSUPPORTED, "mRKC state vectors need n_v N < 2^32");
  const size_t vb = sizeof(double) * n;
  int rc;
  if ((rc = dalloc(c, (void **)&c->d_Y, vb)) || (rc = dalloc(c, (void **)&c->d_FY, vb)) ||
      (rc = dalloc(c, (void **)&c->d_Wv, vb)) || (rc = dalloc(c, (void **)&c->d_FW, vb)) ||
      (rc = dalloc(c, (void **)&c->d_mpart, sizeof(double) * (n / 256 + 1))))
    return rc;
  return EMRKC_OK;
}

static int copy_to_full(emrkc_ctx *c, const emrkc_state *st) {
  const size_t N = (size_t)c->N;
  HIP_TRY(c, hipMemcpyAsync(c->d_Y, st->V, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_Y + N, st->z, sizeof(double) * N * (size_t)(c->nv - 1), hipMemcpyDeviceToDevice,
                            c->stream));
  return EMRKC_OK;
}

static int estimate_mrkc(emrkc_ctx *c, const emrkc_state *st, int *iters_F, int *iters_S, bool *noconv) {
  int rc;
  if ((rc = mrkc_buffers(c)) != EMRKC_OK) return rc;
  const uint64_t n = (uint64_t)c->nv * (uint64_t)c->N;
  for (int w = 0; w < 2; ++w)
    for (int b = 0; b < 2; ++b)
      if (!c->d_mv[w][b] && (rc = dalloc(c, (void **)&c->d_mv[w][b], sizeof(double) * n))) return rc;
  if ((rc = copy_to_full(c, st)) != EMRKC_OK) return rc;
  const StimArgs stim = stim_args(c);
  double ny2 = 0;
  HIP_TRY(c, launch_vec_diff_norm(n, c->d_Y, nullptr, nullptr, c->d_mpart, c->d_result, c->stream));
  if ((rc = fetch(c, &ny2))) return rc;
  const double ny = sqrt(ny2);
  const double delta = ny > 0 ? ny * c->pi_eps : c->pi_eps;
  for (int which = 0; which < 2; ++which) {
    bool &warm = c->m_warm[which];
    int &sel = c->m_sel[which];
    double nv;
    if (warm) {
      nv = c->m_nv[which];
    } else {
      double s2;
      HIP_TRY(c, launch_norm2_random(c->pi_seed, n, c->d_mpart, c->d_result, c->stream));
      if ((rc = fetch(c, &s2))) return rc;
      nv = sqrt(s2);
    }
    HIP_TRY(c, launch_mrkc_rhs(c->model, which, c->mesh, (uint32_t)c->N, st->t, c->d_Y, c->d_FY, stim, c->Cm, c->mp,
                               c->stream));
    double q = delta / nv, rho = warm ? c->m_raw[which] : 0.0, rho_old = 0.0;
    int it = 0;
    while (fabs(rho - rho_old) >= c->pi_tol * rho) {
      if (it >= c->pi_max_iter) {
        *noconv = true;
        break;
      }
      rho_old = rho;
      const double *vin = warm ? c->d_mv[which][sel] : nullptr;
      double *vout = c->d_mv[which][1 - sel];
      HIP_TRY(c, launch_powF_shift((uint32_t)n, c->d_Y, vin, c->pi_seed, q, c->d_Wv, c->stream));
      HIP_TRY(c, launch_mrkc_rhs(c->model, which, c->mesh, (uint32_t)c->N, st->t, c->d_Wv, c->d_FW, stim, c->Cm,
                                 c->mp, c->stream));
      HIP_TRY(c, launch_vec_diff_norm(n, c->d_FW, c->d_FY, vout, c->d_mpart, c->d_result, c->stream));
      double s2;
      if ((rc = fetch(c, &s2))) return rc;
      sel = 1 - sel;
      warm = true;
      nv = sqrt(s2);
      ++it;
      if (nv == 0.0) {
        rho = 0.0;
        break;
      }
      q = delta / nv;
      rho = nv / delta;
    }
    c->m_raw[which] = rho;
    c->m_nv[which] = nv;
    if (which == 0 && iters_F) *iters_F = it;
    if (which == 1 && iters_S) *iters_S = it;
  }
  return EMRKC_OK;
}

extern "C" int emrkc_eval_mrkc_terms(emrkc_ctx *c, const emrkc_state *st, double t, int which, double *out) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st) || out == nullptr || (which != 0 && which != 1))
    return fail(c, EMRKC_EINVAL, "invalid state, output or term");
  if (c->batch || c->mixed) return fail(c, EMRKC_EUNSUPPORTED, "mRKC terms need a double precision single context");
  int rc;
  if ((rc = mrkc_buffers(c)) != EMRKC_OK) return rc;
  if ((rc = copy_to_full(c, st)) != EMRKC_OK) return rc;
  HIP_TRY(c, launch_mrkc_rhs(c->model, which, c->mesh, (uint32_t)c->N, t, c->d_Y, out, stim_args(c), c->Cm, c->mp,
                             c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return EMRKC_OK;
}

static int estimate_batch(emrkc_ctx *c, const emrkc_state *st, double *rho_F, double *rho_S, int *iters_F,
                          int *iters_S);

extern "C" int emrkc_estimate_rho(emrkc_ctx *c, const emrkc_state *st, double *rho_F, double *rho_S, int *iters_F,
                                  int *iters_S) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (!state_ok(c, st)) return fail(c, EMRKC_EINVAL, "state buffers missing");
  int rc = alloc_rho_buffers(c);
  if (rc != EMRKC_OK) return rc;
  if (c->batch) return estimate_batch(c, st, rho_F, rho_S, iters_F, iters_S);
  if (c->method == EMRKC_METHOD_MRKC) {
    bool noconv = false;
    if ((rc = estimate_mrkc(c, st, iters_F, iters_S, &noconv)) != EMRKC_OK) return rc;
    c->rho_F = c->safety * c->m_raw[0];
    c->rho_S = c->safety * c->m_raw[1];
    c->have_rho = true;
    if (rho_F) *rho_F = c->rho_F;
    if (rho_S) *rho_S = c->rho_S;
    if (noconv) return fail(c, EMRKC_ENOCONV, "power iteration reached %d iterations", c->pi_max_iter);
    return EMRKC_OK;
  }
  RhoView v{};
  v.mesh = c->mesh;
  v.N = (uint32_t)c->N;
  v.stride = (size_t)c->N;
  v.V = (const double *)st->V;
  v.z = st->z;
  v.stim = stim_args(c);
  v.Cm = c->Cm;
  v.vF[0] = c->d_vF[0];
  v.vF[1] = c->d_vF[1];
  v.vS[0] = c->d_vS[0];
  v.vS[1] = c->d_vS[1];
  v.zV = c->d_zV;
  v.selF = &c->sel_F;
  v.selS = &c->sel_S;
  v.warm_F = &c->warm_F;
  v.warm_S = &c->warm_S;
  v.raw_F = &c->raw_F;
  v.raw_S = &c->raw_S;
  v.nv_F = &c->nv_F;
  v.nv_S = &c->nv_S;
  bool noconv = false;
  if ((rc = estimate_view(c, v, st->t, iters_F, iters_S, &noconv)) != EMRKC_OK) return rc;
  c->rho_F = c->safety * c->raw_F;
  c->rho_S = c->safety * c->raw_S;
  c->have_rho = true;
  if (rho_F) *rho_F = c->rho_F;
  if (rho_S) *rho_S = c->rho_S;
  if (noconv) return fail(c, EMRKC_ENOCONV, "power iteration reached %d iterations", c->pi_max_iter);
  return EMRKC_OK;
}

// ---------------------------------------------------------------------------
// Single-term evaluations
// ---------------------------------------------------------------------------
extern "C" int emrkc_apply_diffusion(emrkc_ctx *c, const double *V, double *out) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (c->batch) {
    if (V == nullptr || out == nullptr || (const void *)V == (const void *)out)
      return fail(c, EMRKC_EINVAL, "invalid buffers");
    for (auto &I : c->inst) HIP_TRY(c, launch_apply_diffusion(c->mixed, I.mesh, V + I.off, out + I.off, c->stream));
    return EMRKC_OK;
  }
  if (V == nullptr || out == nullptr || (const void *)V == (const void *)out)
    return fail(c, EMRKC_EINVAL, "invalid buffers");
  HIP_TRY(c, launch_apply_diffusion(c->mixed, c->mesh, V, out, c->stream));
  return EMRKC_OK;
}

extern "C" int emrkc_eval_rhs_slow(emrkc_ctx *c, const emrkc_state *st, double t, double *out) {
  if (c == nullptr) return EMRKC_EINVAL;
  if (c->batch) return fail(c, EMRKC_EUNSUPPORTED, "emrkc_eval_rhs_slow takes single-instance contexts");
  if (!state_ok(c, st) || out == nullptr) return fail(c, EMRKC_EINVAL, "invalid buffers");
  HIP_TRY(c, launch_eval_rhs_slow(c->model, c->mixed, (uint32_t)c->N, (const double *)st->V, st->z, t, stim_args(c),
                                  c->Cm, c->mp, out, c->stream));
  return EMRKC_OK;
}

// ---------------------------------------------------------------------------
// P1 tetrahedral meshes: assembled on the host at creation (element
// stiffness |T| G D G^T, row-sum lumped mass |T|/4 per vertex) into an ELL
// operator on neighbour differences: w_ij = -K_ij / (chi Cm M_L,i) for the
// off-diagonal entries of each row, so that (chi Cm M_L)^{-1} A V =
// sum_j w_ij (V_j - V_i) (rows of K sum to zero).  Columns are ordered by
// first appearance in the element list; unused slots repeat the row index
// with weight 0.
// ---------------------------------------------------------------------------
static int upload_ell(emrkc_ctx *c, int64_t N, int maxdeg, const std::vector<uint32_t> &ncol,
                      const std::vector<double> &aval, const std::vector<uint8_t> &deg, const std::vector<double> &ML);

static int build_p1(emrkc_ctx *c, const emrkc_mesh *mesh, const emrkc_conductivity *cond) {
  const int64_t N = mesh->n_nodes, E = mesh->n_elems;
  const double *X = mesh->coords;
  const int64_t *T = mesh->tets;
  constexpr int kMaxDeg = 32;
  std::vector<uint32_t> ncol((size_t)N * kMaxDeg);
  std::vector<double> nval((size_t)N * kMaxDeg, 0.0);
  std::vector<uint8_t> deg((size_t)N, 0);
  std::vector<double> ML((size_t)N, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    int64_t v[4];
    for (int a = 0; a < 4; ++a) {
      v[a] = T[4 * e + a];
      if (v[a] < 0 || v[a] >= N) return fail(c, EMRKC_EINVAL, "element %lld has node index %lld out of range",
                                              (long long)e, (long long)v[a]);
    }
    double B[3][3];  // columns x_a - x_0
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) B[d][a] = X[3 * v[a + 1] + d] - X[3 * v[0] + d];
    const double det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                       B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                       B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    if (!(fabs(det) > 0) || !isfinite(det))
      return fail(c, EMRKC_EINVAL, "element %lld is degenerate", (long long)e);
    // inverse by cofactors: rows of B^{-1} are the gradients of lambda_1..3
    double Bi[3][3];
    Bi[0][0] = (B[1][1] * B[2][2] - B[1][2] * B[2][1]) / det;
    Bi[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) / det;
    Bi[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) / det;
    Bi[1][0] = (B[1][2] * B[2][0] - B[1][0] * B[2][2]) / det;
    Bi[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) / det;
    Bi[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) / det;
    Bi[2][0] = (B[1][0] * B[2][1] - B[1][1] * B[2][0]) / det;
    Bi[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) / det;
    Bi[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) / det;
    double G[4][3];
    for (int d = 0; d < 3; ++d) {
      G[1][d] = Bi[0][d];
      G[2][d] = Bi[1][d];
      G[3][d] = Bi[2][d];
      G[0][d] = -(Bi[0][d] + Bi[1][d] + Bi[2][d]);
    }
    const double *f = mesh->fibres + 3 * e;
    const double fn = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fn > 0) || !isfinite(fn)) return fail(c, EMRKC_EINVAL, "element %lld has no fibre direction", (long long)e);
    const double a3[3] = {f[0] / fn, f[1] / fn, f[2] / fn};
    double D[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        D[i][j] = cond->sigma_l * a3[i] * a3[j] + cond->sigma_t * ((i == j ? 1.0 : 0.0) - a3[i] * a3[j]);
    const double vol = fabs(det) / 6.0;
    for (int a = 0; a < 4; ++a) {
      ML[v[a]] += vol / 4.0;
      double DGa[3];
      for (int i = 0; i < 3; ++i) DGa[i] = D[i][0] * G[a][0] + D[i][1] * G[a][1] + D[i][2] * G[a][2];
      for (int b = 0; b < 4; ++b) {
        if (b == a) continue;
        const double kab = vol * (G[b][0] * DGa[0] + G[b][1] * DGa[1] + G[b][2] * DGa[2]);
        const size_t row = (size_t)v[a] * kMaxDeg;
        int k = 0;
        while (k < deg[v[a]] && ncol[row + k] != (uint32_t)v[b]) ++k;
        if (k == deg[v[a]]) {
          if (k == kMaxDeg) return fail(c, EMRKC_EUNSUPPORTED, "node %lld has more than %d neighbours",
                                        (long long)v[a], kMaxDeg);
          ncol[row + k] = (uint32_t)v[b];
          deg[v[a]] = (uint8_t)(k + 1);
        }
        nval[row + k] += kab;
      }
    }
  }
  for (int64_t i = 0; i < N; ++i)
    if (!(ML[i] > 0)) return fail(c, EMRKC_EINVAL, "node %lld belongs to no element", (long long)i);
  // the off-diagonal entries of A = -K
  for (double &v : nval) v = -v;
  return upload_ell(c, N, kMaxDeg, ncol, nval, deg, ML);
}

// The ELL operator (chi Cm M_L)^{-1} A in difference form from the
// off-diagonal entries of A: row i has deg[i] neighbours ncol[i maxdeg + k]
// with values aval[i maxdeg + k]; also keeps M_L on the device.
static int upload_ell(emrkc_ctx *c, int64_t N, int maxdeg, const std::vector<uint32_t> &ncol,
                      const std::vector<double> &aval, const std::vector<uint8_t> &deg, const std::vector<double> &ML) {
  uint32_t width = 1;
  for (int64_t i = 0; i < N; ++i) width = std::max<uint32_t>(width, deg[i]);
  const double chiCm = c->chi * c->Cm;
  std::vector<uint32_t> col((size_t)width * N);
  std::vector<double> w64((size_t)width * N);
  std::vector<float> w32((size_t)width * N);
  for (int64_t i = 0; i < N; ++i) {
    for (uint32_t k = 0; k < width; ++k) {
      const bool used = k < deg[i];
      const size_t o = (size_t)k * N + i;
      col[o] = used ? ncol[(size_t)i * maxdeg + k] : (uint32_t)i;
      w64[o] = used ? aval[(size_t)i * maxdeg + k] / (chiCm * ML[i]) : 0.0;
      w32[o] = (float)w64[o];
    }
  }
  int rc;
  if ((rc = dalloc(c, (void **)&c->d_ell_col, col.size() * sizeof(uint32_t))) ||
      (rc = dalloc(c, (void **)&c->d_ell_w64, w64.size() * sizeof(double))) ||
      (rc = dalloc(c, (void **)&c->d_ell_w32, w32.size() * sizeof(float))))
    return rc;
  HIP_TRY(c, hipMemcpy(c->d_ell_col, col.data(), col.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->d_ell_w64, w64.data(), w64.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->d_ell_w32, w32.data(), w32.size() * sizeof(float), hipMemcpyHostToDevice));
  c->mesh.kind = kEll;
  c->mesh.ell.N = (uint32_t)N;
  c->mesh.ell.width = width;
  c->mesh.ell.col = c->d_ell_col;
  c->mesh.ell.w64 = c->d_ell_w64;
  c->mesh.ell.w32 = c->d_ell_w32;
  c->dim = 3;
  // lumped mass, for the implicit diffusion solve of IMEX-RL
  if ((rc = dalloc(c, (void **)&c->d_ML, ML.size() * sizeof(double)))) return rc;
  HIP_TRY(c, hipMemcpy(c->d_ML, ML.data(), ML.size() * sizeof(double), hipMemcpyHostToDevice));
  return EMRKC_OK;
}

// Assembled operator A = -K (CSR) and lumped mass given by the caller:
// off-diagonal entries (duplicates summed) become the ELL difference form;
// rows must sum to zero, which makes the diagonal implied.
static int build_csr(emrkc_ctx *c, const emrkc_mesh *mesh) {
  const int64_t N = mesh->n_nodes;
  const int64_t *rp = mesh->row_ptr;
  constexpr int kMaxDeg = 64;
  if (rp[0] != 0) return fail(c, EMRKC_EINVAL, "CSR row_ptr[0] must be 0");
  std::vector<uint32_t> ncol((size_t)N * kMaxDeg);
  std::vector<double> aval((size_t)N * kMaxDeg, 0.0);
  std::vector<uint8_t> deg((size_t)N, 0);
  std::vector<double> ML((size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    if (rp[i + 1] < rp[i]) return fail(c, EMRKC_EINVAL, "CSR row_ptr decreases at row %lld", (long long)i);
    const double m = mesh->lumped_mass[i];
    if (!(m > 0) || !isfinite(m)) return fail(c, EMRKC_EINVAL, "lumped mass of node %lld is not positive", (long long)i);
    ML[i] = m;
    double sum = 0.0, mag = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int64_t j = mesh->col_idx[e];
      const double v = mesh->values[e];
      if (j < 0 || j >= N) return fail(c, EMRKC_EINVAL, "CSR column %lld out of range in row %lld", (long long)j,
                                       (long long)i);
      if (!isfinite(v)) return fail(c, EMRKC_EINVAL, "CSR value not finite in row %lld", (long long)i);
      sum += v;
      mag += fabs(v);
      if (j == i) continue;
      const size_t row = (size_t)i * kMaxDeg;
      int k = 0;
      while (k < deg[i] && ncol[row + k] != (uint32_t)j) ++k;
      if (k == deg[i]) {
        if (k == kMaxDeg)
          return fail(c, EMRKC_EUNSUPPORTED, "row %lld has more than %d off-diagonal entries", (long long)i, kMaxDeg);
        ncol[row + k] = (uint32_t)j;
        deg[i] = (uint8_t)(k + 1);
      }
      aval[row + k] += v;
    }
    if (fabs(sum) > 1e-10 * mag)
      return fail(c, EMRKC_EINVAL, "CSR row %lld does not sum to zero (%g of %g): A 1 = 0 is required", (long long)i,
                  sum, mag);
  }
  return upload_ell(c, N, kMaxDeg, ncol, aval, deg, ML);
}

// ---------------------------------------------------------------------------
// Batched ensembles
// ---------------------------------------------------------------------------
extern "C" int emrkc_create_batch(int n_inst, const emrkc_mesh *meshes, const emrkc_conductivity *conds,
                                  int ionic_model, const emrkc_params *params, emrkc_ctx **out) {
  if (out == nullptr) return EMRKC_EINVAL;
  *out = nullptr;
  if (n_inst < 1 || n_inst > 65535 || meshes == nullptr || conds == nullptr || params == nullptr)
    return EMRKC_EINVAL;
  if (model_gates(ionic_model) < 0) return EMRKC_EINVAL;
  const emrkc_params &p0 = params[0];
  if (p0.precision != EMRKC_FP64 && p0.precision != EMRKC_MIXED32) return EMRKC_EINVAL;
  if (!(p0.eps > 0) || !(p0.eps < 1) || !(p0.rho_safety >= 1.0)) return EMRKC_EINVAL;
  if (!(p0.powiter_tol > 0) || !(p0.powiter_eps > 0) || p0.powiter_max_iter < 1) return EMRKC_EINVAL;
  if (p0.rho_every != 0) return EMRKC_EUNSUPPORTED;        // ensembles keep the radii they are given
  if (p0.method != EMRKC_METHOD_EMRKC) return EMRKC_EUNSUPPORTED;
  if (p0.flags & EMRKC_COND_A) return EMRKC_EUNSUPPORTED;  // one eta per outer stage for all instances
  int64_t Ntot = 0;
  for (int k = 0; k < n_inst; ++k) {
    const emrkc_mesh &m = meshes[k];
    const emrkc_params &p = params[k];
    if (m.kind != EMRKC_MESH_Q1_GRID) return EMRKC_EUNSUPPORTED;
    if (m.dim != 2 && m.dim != 3) return EMRKC_EINVAL;
    int64_t N = 1;
    for (int d = 0; d < m.dim; ++d) {
      if (m.n[d] < 2 || m.n[d] > (1 << 30) || !(m.h[d] > 0) || !isfinite(m.h[d])) return EMRKC_EINVAL;
      if (m.n[d] > kMaxNodes / N) return EMRKC_EUNSUPPORTED;  // before the product: no overflow
      N *= m.n[d];
    }
    if (!(p.chi > 0) || !(p.Cm > 0) || !isfinite(p.chi) || !isfinite(p.Cm)) return EMRKC_EINVAL;
    if (!isfinite(p.stim_amp) || !isfinite(p.stim_t_on) || !isfinite(p.stim_t_off)) return EMRKC_EINVAL;
    const double sg[3] = {conds[k].sigma_l, conds[k].sigma_t, conds[k].sigma_n};
    for (int d = 0; d < m.dim; ++d)
      if (!(sg[d] >= 0) || !isfinite(sg[d])) return EMRKC_EINVAL;
    if (N > kMaxNodes - Ntot) return EMRKC_EUNSUPPORTED;
    Ntot += N;
  }

  emrkc_ctx *c = new (std::nothrow) emrkc_ctx();
  if (c == nullptr) return EMRKC_ENOMEM;
  c->batch = true;
  c->mesh_kind = EMRKC_MESH_Q1_GRID;
  c->N = Ntot;
  c->model = ionic_model;
  c->ng = model_gates(ionic_model);
  c->ns = model_slow(ionic_model);
  c->nv = 1 + c->ng + c->ns;
  c->mixed = p0.precision == EMRKC_MIXED32;
  c->flags = p0.flags;
  c->progressive = (p0.flags & EMRKC_PROGRESSIVE) != 0;
  c->chi = p0.chi;
  c->Cm = p0.Cm;
  c->eps = p0.eps;
  c->safety = p0.rho_safety;
  c->mp.lin_a = p0.linear_a;
  c->mp.lin_lamE = p0.linear_lambda_E;
  c->pi_tol = p0.powiter_tol;
  c->pi_eps = p0.powiter_eps;
  c->pi_max_iter = p0.powiter_max_iter;
  c->pi_seed = p0.powiter_seed;
  c->mesh.kind = kGrid;
  c->inst.resize(n_inst);
  std::vector<uint8_t> mask((size_t)Ntot, 0);
  bool any_mask = false, all_rho = true;
  uint32_t off = 0;
  for (int k = 0; k < n_inst; ++k) {
    const emrkc_mesh &m = meshes[k];
    const emrkc_params &p = params[k];
    Inst &I = c->inst[k];
    Grid &g = I.mesh.grid;
    I.mesh.kind = kGrid;
    g.dim = m.dim;
    g.n0 = (uint32_t)m.n[0];
    g.n1 = (uint32_t)m.n[1];
    g.n2 = m.dim == 3 ? (uint32_t)m.n[2] : 1u;
    g.N = g.n0 * g.n1 * g.n2;
    g.div0 = make_fastdiv(g.n0);
    g.div1 = make_fastdiv(g.n1);
    g.inner_variant = g.head_variant = 0;
    g.zc = g.head_zc = 1;
    const double h[3] = {m.h[0], m.h[1], m.dim == 3 ? m.h[2] : 1.0};
    const double sg[3] = {conds[k].sigma_l, conds[k].sigma_t, conds[k].sigma_n};
    grid_weights(m.dim, h, sg, p.chi * p.Cm, g.w);
    I.off = off;
    I.N = g.N;
    I.chi = p.chi;
    I.Cm = p.Cm;
    I.amp = p.stim_amp;
    I.t_on = p.stim_t_on;
    I.t_off = p.stim_t_off;
    if (p.stim_mask != nullptr) {
      memcpy(mask.data() + off, p.stim_mask, g.N);
      any_mask = true;
    }
    if (p.rho_F > 0 && p.rho_S > 0) {
      I.rho_F = p.rho_F;
      I.rho_S = p.rho_S;
      I.have_rho = true;
    } else {
      all_rho = false;
    }
    off += g.N;
  }
  if (all_rho) {
    c->have_rho = true;
    for (auto &I : c->inst) {
      c->rho_F = std::max(c->rho_F, I.rho_F);
      c->rho_S = std::max(c->rho_S, I.rho_S);
    }
  }
  int rc = EMRKC_OK;
  {
    const size_t vb = sizeof(double) * (size_t)Ntot;
    const size_t svb = (c->mixed ? sizeof(float) : sizeof(double)) * (size_t)Ntot;
    if ((rc = dalloc(c, (void **)&c->d_V1, vb)) || (rc = dalloc(c, (void **)&c->d_U[0], vb)) ||
        (rc = dalloc(c, (void **)&c->d_U[1], vb)) || (rc = dalloc(c, (void **)&c->d_U[2], vb)) ||
        (rc = dalloc(c, &c->d_SV, svb)) || (rc = dalloc(c, &c->d_SV2, svb)) ||
        (rc = dalloc(c, (void **)&c->d_clock, sizeof(Clock))) ||
        (rc = dalloc(c, (void **)&c->d_result, 2 * sizeof(double))) ||
        (rc = dalloc(c, (void **)&c->d_flag, sizeof(int))))
      goto error;
    const size_t nparts = std::max<size_t>(reduce_blocks((uint32_t)Ntot), 65536);
    if ((rc = dalloc(c, (void **)&c->d_partials, nparts * sizeof(double)))) goto error;
    if (any_mask) {
      if ((rc = dalloc(c, (void **)&c->d_mask, (size_t)Ntot))) goto error;
      hipError_t e = hipMemcpy(c->d_mask, mask.data(), (size_t)Ntot, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        rc = fail(c, EMRKC_EHIP, "mask upload failed: %s", hipGetErrorString(e));
        goto error;
      }
    }
    hipError_t e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemset(c->d_clock, 0, sizeof(Clock));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      rc = fail(c, EMRKC_EHIP, "initialisation failed: %s", hipGetErrorString(e));
      goto error;
    }
  }
  *out = c;
  return EMRKC_OK;
error:
  free_ctx(c);
  delete c;
  return rc;
}

static int estimate_batch(emrkc_ctx *c, const emrkc_state *st, double *rho_F, double *rho_S, int *iters_F,
                          int *iters_S) {
  const size_t Ntot = (size_t)c->N;
  const size_t zw = c->mixed ? sizeof(float) : sizeof(double);
  bool noconv = false;
  int maxF = 0, maxS = 0;
  c->rho_F = c->rho_S = 0.0;
  for (auto &I : c->inst) {
    RhoView v{};
    v.mesh = I.mesh;
    v.N = I.N;
    v.stride = Ntot;
    v.V = (const double *)st->V + I.off;
    v.z = (const char *)st->z + zw * I.off;
    v.stim.mask = c->d_mask ? c->d_mask + I.off : nullptr;
    v.stim.amp = I.amp;
    v.stim.t_on = I.t_on;
    v.stim.t_off = I.t_off;
    v.Cm = I.Cm;
    for (int b = 0; b < 2; ++b) {
      v.vF[b] = c->d_vF[b] + I.off;
      v.vS[b] = c->d_vS[b] + I.off;
    }
    v.zV = c->d_zV + I.off;
    v.selF = &I.sel_F;
    v.selS = &I.sel_S;
    v.warm_F = &I.warm_F;
    v.warm_S = &I.warm_S;
    v.raw_F = &I.raw_F;
    v.raw_S = &I.raw_S;
    v.nv_F = &I.nv_F;
    v.nv_S = &I.nv_S;
    int itF = 0, itS = 0;
    int rc = estimate_view(c, v, st->t, &itF, &itS, &noconv);
    if (rc != EMRKC_OK) return rc;
    maxF = std::max(maxF, itF);
    maxS = std::max(maxS, itS);
    I.rho_F = c->safety * I.raw_F;
    I.rho_S = c->safety * I.raw_S;
    I.have_rho = true;
    c->rho_F = std::max(c->rho_F, I.rho_F);
    c->rho_S = std::max(c->rho_S, I.rho_S);
  }
  c->have_rho = true;
  clear_graphs(c);
  c->bdev.valid = false;
  if (rho_F) *rho_F = c->rho_F;
  if (rho_S) *rho_S = c->rho_S;
  if (iters_F) *iters_F = maxF;
  if (iters_S) *iters_S = maxS;
  if (noconv) return fail(c, EMRKC_ENOCONV, "power iteration reached %d iterations", c->pi_max_iter);
  return EMRKC_OK;
}

// Tables of the batched step (see BatchDev): instance coefficients from the
// instance's own m_i, pointers into the concatenated buffers.
static int build_batch_tables(emrkc_ctx *c, const emrkc_state *st, double dt, const StepPlan &P) {
  uint64_t dtb;
  memcpy(&dtb, &dt, sizeof dtb);
  const int shape_key =
      c->batch_shape + (c->batch_flat_head ? 3 : 0) + 8 * c->batch_march_zc + (c->batch_pairs ? 1024 : 0);
  void *const zbuf = zstate(c, st);  // the state's z, or the block buffer while a call steps on it
  if (c->bdev.valid && c->bdev.dt_bits == dtb && c->bdev.V == st->V && c->bdev.z == zbuf &&
      c->bdev.shape == shape_key)
    return EMRKC_OK;
  (void)hipStreamSynchronize(c->stream);
  clear_graphs(c);
  free_batch_tables(c);
  double *X[2] = {(double *)st->V, c->d_V1};
  // the kernels read the map as 32-bit words: an even number of entries
  auto upload = [&](BatchLaunch &L, const std::vector<BatchInst> &tab, std::vector<uint16_t> map) -> int {
    L.nblocks = (uint32_t)map.size();
    map.resize(std::max<size_t>(2, (map.size() + 1) & ~(size_t)1), 0);
    int rc;
    if ((rc = dalloc(c, (void **)&L.tab, std::max<size_t>(1, tab.size()) * sizeof(BatchInst))) ||
        (rc = dalloc(c, (void **)&L.map, map.size() * sizeof(uint16_t))))
      return rc;
    if (!tab.empty()) HIP_TRY(c, hipMemcpy(L.tab, tab.data(), tab.size() * sizeof(BatchInst), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(L.map, map.data(), map.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    return EMRKC_OK;
  };
  for (int par = 0; par < 2; ++par) {
    for (int k = 1; k <= P.m; ++k) {  // k == 1: the head launch
      std::vector<BatchInst> tab;
      std::vector<uint16_t> map;
      for (auto &I : c->inst) {
        if (I.m < k) continue;
        std::vector<double> mu, nu, ka, cc;
        rkc_coeffs(I.m, c->eps, mu, nu, ka, cc);
        BatchInst b{};
        b.g = I.mesh.grid;
        b.off = I.off;
        b.tile0 = (uint32_t)map.size();
        // head launch with the flat kernel: blocks of 256 consecutive nodes;
        // inner stages of 3-D instances with marching columns: columns of
        // MX x MY nodes and batch_march_zc planes (x fastest, then y, then z)
        const bool march = k >= 2 && c->batch_march_zc > 0 && b.g.dim == 3;
        uint32_t nt;
        if (k == 1 && c->batch_flat_head) {
          nt = (b.g.N + 255u) / 256u;
        } else if (march) {
          b.g.inner_variant = 1;
          b.g.zc = std::min<uint32_t>((uint32_t)c->batch_march_zc, b.g.n2);
          b.ntx = (b.g.n0 + MX - 1) / MX;
          b.nty = (b.g.n1 + MY - 1) / MY;
          nt = b.ntx * b.nty * ((b.g.n2 + b.g.zc - 1) / b.g.zc);
        } else if (k >= 2 && c->batch_pairs) {  // two tiles per block
          b.g.inner_variant = 2;
          nt = (grid_tiles(b.g, b.ntx, b.nty, c->batch_shape) + 1) / 2;
        } else {
          nt = grid_tiles(b.g, b.ntx, b.nty, c->batch_shape);
        }
        if (k == 1) {
          HeadArgs &h = b.h;
          h.Vin = X[par];
          h.zin = h.zout = zbuf;
          h.z_aos = c->zb_run ? 1 : 0;
          h.SV = c->d_SV;
          h.uout = I.m == 1 ? X[1 - par] : c->d_U[0];
          h.clock = c->d_clock;
          h.stim.mask = c->d_mask;
          h.stim.amp = I.amp;
          h.stim.t_on = I.t_on;
          h.stim.t_off = I.t_off;
          h.mp = c->mp;
          h.dt = dt;
          h.eta = P.eta;
          h.inv_eta = 1.0 / P.eta;
          h.Cm = I.Cm;
          h.c_prev = 0.0;
          h.mu_dt = P.mu[1] * dt;
          h.mu1_eta = mu[1] * P.eta;
          h.cm_eta = cc[I.m] * P.eta;
          h.j1 = 1;
          h.m_is_one = I.m == 1;
          h.progressive = c->progressive ? 1 : 0;
          h.cm = cc[I.m];
        } else {
          InnerArgs &a = b.in;
          a.t.nu = nu[k];
          a.t.kappa = ka[k];
          a.t.mu_eta = mu[k] * P.eta;
          a.t.inv_eta = 1.0 / P.eta;
          a.t.mu_dt = P.mu[1] * dt;
          a.t.j1 = 1;
          a.t.uprev = c->d_U[(k - 2) % 2];
          a.t.uprev2 = k == 2 ? X[par] : c->d_U[(k - 3) % 2];
          a.t.SV = c->d_SV;
          a.t.Vin = X[par];
          a.last = k == I.m;
          a.out = a.last ? X[1 - par] : c->d_U[(k - 1) % 2];
        }
        const uint16_t slot = (uint16_t)tab.size();
        tab.push_back(b);
        map.insert(map.end(), nt, slot);
      }
      BatchLaunch L;
      int rc = upload(L, tab, map);
      if (rc != EMRKC_OK) return rc;
      if (k == 1)
        c->bdev.head[par] = L;
      else
        c->bdev.inner[par].push_back(L);
    }
  }
  c->bdev.valid = true;
  c->bdev.dt_bits = dtb;
  c->bdev.shape = shape_key;
  c->bdev.V = st->V;
  c->bdev.z = zbuf;
  c->bdev.s = P.s;
  c->bdev.m_max = P.m;
  c->bdev.eta = P.eta;
  return EMRKC_OK;
}

// L batched steps: V^n ping-pongs between X[0] and X[1]; an odd chunk ends
// with one copy back to X[0].
static int enqueue_chunk_batch(emrkc_ctx *c, const emrkc_state *st, const StepPlan &P, double dt, int L,
                               hipStream_t strm, KernelTimer *tm) {
  (void)dt;
  (void)P;
  const uint32_t Ntot = (uint32_t)c->N;
  for (int n = 0; n < L; ++n) {
    const int par = n % 2;
    const BatchLaunch &H = c->bdev.head[par];
    TIMED(0, launch_head_batch(c->model, c->mixed, c->batch_flat_head ? kBatchFlatHead : c->batch_shape, H.tab, H.map,
                               H.nblocks, Ntot, n, strm));
    for (const BatchLaunch &B : c->bdev.inner[par])
      if (B.nblocks)
        TIMED(1, launch_inner_batch(c->mixed, c->batch_shape, c->batch_march_zc > 0 ? 1 : c->batch_pairs ? 2 : 0,
                                    B.tab, B.map, B.nblocks, Ntot, strm));
  }
  double *X1 = c->d_V1;
  HIP_TRY(c, launch_copy_tick(L % 2 ? X1 : nullptr, (double *)st->V, Ntot, c->d_clock, L, strm));
  return EMRKC_OK;
}

extern "C" int emrkc_batch_size(const emrkc_ctx *c) { return c == nullptr ? -1 : (c->batch ? (int)c->inst.size() : 1); }

extern "C" int emrkc_batch_info(const emrkc_ctx *c, double dt, int64_t *offsets, int *m, double *rho_F, double *rho_S) {
  if (c == nullptr) return EMRKC_EINVAL;
  const int n = c->batch ? (int)c->inst.size() : 1;
  for (int k = 0; k < n; ++k) {
    if (offsets) offsets[k] = c->batch ? c->inst[k].off : 0;
    const double rF = c->batch ? c->inst[k].rho_F : c->rho_F;
    const double rS = c->batch ? c->inst[k].rho_S : c->rho_S;
    if (rho_F) rho_F[k] = rF;
    if (rho_S) rho_S[k] = rS;
    if (m) {
      int si = 0, mi = 0;
      double ei;
      m[k] = (c->have_rho && emrkc_stage_counts(dt, rF, c->rho_S, c->eps, &si, &mi, &ei) == EMRKC_OK) ? mi : 0;
    }
  }
  if (offsets) offsets[n] = c->N;
  return EMRKC_OK;
}

extern "C" int emrkc_batch_set_rho(emrkc_ctx *c, const double *rho_F, const double *rho_S) {
  if (c == nullptr || rho_F == nullptr || rho_S == nullptr) return EMRKC_EINVAL;
  if (!c->batch) return emrkc_set_rho(c, rho_F[0], rho_S[0]);
  for (size_t k = 0; k < c->inst.size(); ++k)
    if (!(rho_F[k] >= 0) || !(rho_S[k] >= 0) || !isfinite(rho_F[k]) || !isfinite(rho_S[k]))
      return fail(c, EMRKC_EINVAL, "invalid spectral radii for instance %zu", k);
  c->rho_F = c->rho_S = 0.0;
  for (size_t k = 0; k < c->inst.size(); ++k) {
    c->inst[k].rho_F = rho_F[k];
    c->inst[k].rho_S = rho_S[k];
    c->inst[k].have_rho = true;
    c->rho_F = std::max(c->rho_F, rho_F[k]);
    c->rho_S = std::max(c->rho_S, rho_S[k]);
  }
  c->have_rho = true;
  clear_graphs(c);
  c->bdev.valid = false;
  return EMRKC_OK;
}
