// Kernels of the emRKC library (gfx950).  One thread per mesh node, state
// in structure-of-arrays layout; no floating-point atomics, reductions are
// two-pass with a fixed order (bit-reproducible).
#include <hip/hip_ext.h>
#include <type_traits>

#include "emrkc_internal.h"

namespace emrkc {

// Events that the next launches record around the kernel itself (from the
// dispatch's own timestamps); set by the host's profiling pass, null
// otherwise.
static thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}

#define EMRKC_LAUNCH(kern, grid, block, shm, st, ...)                                               \
  do {                                                                                              \
    if (g_ev_start != nullptr)                                                                      \
      hipExtLaunchKernelGGL(kern, grid, block, shm, st, g_ev_start, g_ev_stop, 0u, __VA_ARGS__);    \
    else                                                                                            \
      hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);                                  \
  } while (0)

constexpr int kBlock = 256;

template <bool MIXED>
using MathOf = typename std::conditional<MIXED, MathF32, MathF64>::type;

// Stage time t_n + c_{j-1} dt with t_n = t0 + n dt, n = chunk base + offset,
// without contraction so that host and device obtain the same double.
// Every array the kernels touch is in global memory.  A pointer that a
// kernel reads from a table in memory (the batched kernels' instance
// records) is generic, and the compiler issues flat instructions through
// it, which also count against the LDS counter so that every LDS access
// waits for them; the global-pointer form below gives global instructions.
// (Pointers in kernel arguments are global to the compiler already.)
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p) {
  return (__attribute__((address_space(1))) T *)(uintptr_t)p;
}

__device__ __forceinline__ double stage_time(const Clock *c, int step_off, double dt, double c_prev) {
#pragma clang fp contract(off)
  const auto g = gptr(c);
  const double tn = g->t0 + (double)(g->step + step_off) * dt;
  return tn + c_prev * dt;
}

__device__ __forceinline__ double stimulus(const StimArgs &s, uint32_t i, double t) {
  return (s.mask != nullptr && gptr(s.mask)[i] != 0 && s.t_on <= t && t <= s.t_off) ? s.amp : 0.0;
}

__device__ __forceinline__ uint32_t node_index() {
  return xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ void grid_coords(const Grid &g, uint32_t i, uint32_t &ix, uint32_t &iy,
                                            uint32_t &iz) {
  const uint32_t q0 = fdiv(i, g.div0);
  ix = i - q0 * g.n0;
  iz = fdiv(q0, g.div1);
  iy = q0 - iz * g.n1;
}

template <bool MIXED>
__device__ __forceinline__ double ell_apply(const Ell &e, const double *__restrict__ u, uint32_t i) {
  const double uc = u[i];
  if (MIXED) {
    float acc = 0.0f;
    for (uint32_t k = 0; k < e.width; ++k) {
      const uint32_t c = e.col[(size_t)k * e.N + i];
      acc = __builtin_fmaf(e.w32[(size_t)k * e.N + i], (float)(u[c] - uc), acc);
    }
    return (double)acc;
  }
  double acc = 0.0;
  for (uint32_t k = 0; k < e.width; ++k) {
    const uint32_t c = e.col[(size_t)k * e.N + i];
    acc = __builtin_fma(e.w64[(size_t)k * e.N + i], u[c] - uc, acc);
  }
  return acc;
}

template <bool MIXED>
__device__ __forceinline__ double apply_op(const Mesh &mesh, const double *__restrict__ u, uint32_t i) {
  if (mesh.kind == kGrid) {
    uint32_t ix, iy, iz;
    grid_coords(mesh.grid, i, ix, iy, iz);
    return mesh.grid.dim == 3 ? grid_apply<3>(u, mesh.grid, ix, iy, iz)
                              : grid_apply<2>(u, mesh.grid, ix, iy, iz);
  }
  return ell_apply<MIXED>(mesh.ell, u, i);
}

// ---------------------------------------------------------------------------
// Resting state
// ---------------------------------------------------------------------------
template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_init_state(uint32_t N, double *V, void *zv, ModelParams mp) {
  using M = MathOf<MIXED>;
  using R = typename M::R;
  using Mod = Model<M>;
  constexpr int NG = Mod::NG, NS = Mod::NS;
  const uint32_t i = node_index();
  if (i >= N) return;
  R lam[NG], zinf[NG];
  Mod::gates(R(Mod::V_REST), mp, lam, zinf);
  V[i] = Mod::V_REST;
  R *z = (R *)zv;
#pragma unroll
  for (int g = 0; g < NG; ++g) z[(size_t)g * N + i] = zinf[g];
#pragma unroll
  for (int s = 0; s < NS; ++s) z[(size_t)(NG + s) * N + i] = R(Mod::slow_rest(s));
}

// First inner stage u_1 = u_0 + mu'_1 eta (f_F(u_0) + S_V) with one fused
// multiply-add, the same in every kernel that forms it (the head, or the
// two-stage inner kernel of the split stage), so that they round alike.
__device__ __forceinline__ double first_inner(double mu1_eta, double u0, double Fu0, double sv) {
#pragma clang fp contract(off)
  return __builtin_fma(mu1_eta, Fu0 + sv, u0);
}

// ---------------------------------------------------------------------------
// Outer-stage head at one node, given V_{j-1} and f_F(V_{j-1}) there
// ---------------------------------------------------------------------------
// FVf() evaluates f_F(V_{j-1}) at the node; it is called after the z update
// so that the stencil operands are not live across the ionic model.
// Where node i's components sit in a z array: component k at
// base + k * stride; component planes of N (base i, stride N) or, with
// `blocks`, blocks of kZBlock nodes x nz components.
struct ZAt {
  size_t base, stride;
};
__device__ __forceinline__ ZAt z_at(bool blocks, uint32_t N, uint32_t i, int nz) {
  if (blocks) return ZAt{(size_t)(i / kZBlock) * kZBlock * (size_t)nz + i % kZBlock, kZBlock};
  return ZAt{i, N};
}

// z_{j-1} of node i (all ionic components).  NT: non-temporal loads, used
// by the pointwise head of the split stage when z is held in blocks (which
// the host does only for arrays of 256 MiB and more): each value is read
// once per step and does not stay in the caches anyway, and bypassing them
// keeps the inner kernel's operands there (on the 36.5M-node slab the
// pointwise head took 2.31 instead of 2.37 ms, 1.07 instead of 1.16 ms in
// the mixed form, and the following inner kernel 0.310 instead of
// 0.321 ms).  Heads that read the V stencil through the caches lose by it
// (the flat batched head of the 64-instance ensemble: 0.455 against
// 0.431 ms), and so does a cache-resident z (a 442k-node grid's head took
// 64 instead of 38 us).  NT is a template parameter: with a run-time
// choice the compiler merged the two paths' accesses into ordinary ones.
template <template <class> class Model, bool MIXED>
struct HeadZ {
  using R = typename MathOf<MIXED>::R;
  static constexpr int NZ = Model<MathOf<MIXED>>::NG + Model<MathOf<MIXED>>::NS;
  R z[NZ];
  template <bool NT>
  __device__ __forceinline__ void load(const void *zin, ZAt at) {
    const auto p = gptr((const R *)zin);
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
      if (NT)
        z[k] = __builtin_nontemporal_load(&p[at.base + k * at.stride]);
      else
        z[k] = p[at.base + k * at.stride];
    }
  }
  __device__ __forceinline__ void load(const void *zin, uint32_t N, uint32_t i) {
    load<false>(zin, z_at(false, N, i, NZ));
  }
};

// A store of z: non-temporal for z held in blocks (see HeadZ).
template <bool NT, class P, class R>
__device__ __forceinline__ void z_store(P zout, size_t idx, R v) {
  if (NT)
    __builtin_nontemporal_store(v, &zout[idx]);
  else
    zout[idx] = v;
}

// NT: non-temporal z accesses (the kernel is launched so only with z in
// blocks; see HeadZ)
template <template <class> class Model, bool MIXED, bool SV_ONLY = false, bool NT = false, class FVf>
__device__ __forceinline__ void head_node_z(const HeadArgs &a, uint32_t N, uint32_t i, double V,
                                            const typename MathOf<MIXED>::R *z, double Is, FVf FVfun);

template <template <class> class Model, bool MIXED, bool SV_ONLY = false, bool NT = false, class FVf>
__device__ __forceinline__ void head_node(const HeadArgs &a, uint32_t N, uint32_t i, double V, FVf FVfun) {
  HeadZ<Model, MIXED> hz;
  hz.template load<NT>(a.zin, z_at(a.z_aos != 0, N, i, HeadZ<Model, MIXED>::NZ));
  const double tj = stage_time(a.clock, a.step_off, a.dt, a.c_prev);
  head_node_z<Model, MIXED, SV_ONLY, NT>(a, N, i, V, hz.z, stimulus(a.stim, i, tj), FVfun);
}

// The head at node i with z_{j-1} and the stimulus current I_stim(t_j) at
// the node given.  SV_ONLY: the pointwise head of the split stage (m >= 2),
// which stores S_V and leaves the first inner stage to k_inner12_march.
template <template <class> class Model, bool MIXED, bool SV_ONLY, bool NT, class FVf>
__device__ __forceinline__ void head_node_z(const HeadArgs &a, uint32_t N, uint32_t i, double V,
                                            const typename MathOf<MIXED>::R *z, double Is, FVf FVfun) {
  using M = MathOf<MIXED>;
  using R = typename M::R;
  using Mod = Model<M>;
  constexpr int NG = Mod::NG, NS = Mod::NS, NZ = NG + NS;

  // exponential Euler for the gates: z_E + (e^{eta Lambda} - 1)(z_E - z_inf)
  R lam[NG], zinf[NG], zE[NG];
  Mod::gates(R(V), a.mp, lam, zinf);
  const R eta = R(a.eta);
#pragma unroll
  for (int g = 0; g < NG; ++g) zE[g] = z[g] + M::expm1(eta * lam[g]) * (z[g] - zinf[g]);

  // slow right-hand side at y_E, frozen over the inner iteration
  R dS[NS > 0 ? NS : 1];
  const R iion = Mod::eval(R(V), zE, z + NG, dS, a.mp);
  double SV;
  if (MIXED)
    SV = (double)((R(Is) - R(a.Cm) * iion) * R(1.0 / a.Cm));
  else
    SV = (Is - a.Cm * (double)iion) / a.Cm;

  // outer recurrence of z with the averaged force (u_eta - y)/eta; the
  // inner iteration leaves gates at z_E and moves the slow variables by
  // c'_m eta g_S (f_F has no z component).  Mixed form, first outer stage:
  // the gate update z + (mu dt / eta)(z_E - z) is one float FMA on the float
  // gate (its rounding stays at the level of the float storage it is written
  // to); later stages, whose coefficients nu and kappa can exceed 1, and the
  // slow variables recur in double.
  const auto zout = gptr((R *)a.zout);
  const auto zin2 = gptr((const R *)a.zin2);
  const ZAt za = z_at(a.z_aos != 0, N, i, NZ);
  const float gate_c = (float)(a.mu_dt * a.inv_eta * (a.progressive ? a.cm : 1.0));
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    if (MIXED && k < NG && a.j1) {
      z_store<NT>(zout, za.base + k * za.stride, R(__builtin_fmaf(gate_c, (float)(zE[k] - z[k]), (float)z[k])));
      continue;
    }
    double fbar;
    if (k < NG) {
      fbar = (double)(zE[k] - z[k]) * a.inv_eta;
      if (a.progressive) fbar *= a.cm;
    } else {
      const double zs = (double)z[k];
      const double um = zs + a.cm_eta * (double)dS[k - NG];
      fbar = (um - zs) * a.inv_eta;
    }
    double zj;
    if (a.j1)
      zj = (double)z[k] + a.mu_dt * fbar;
    else
      zj = a.nu * (double)z[k] + a.kappa * (double)zin2[za.base + k * za.stride] + a.mu_dt * fbar;
    z_store<NT>(zout, za.base + k * za.stride, R(zj));
  }

  if (SV_ONLY) {
    if (MIXED)
      gptr((float *)a.SV)[i] = (float)SV;
    else
      gptr((double *)a.SV)[i] = SV;
    return;
  }
  // first inner stage u_1 = u_0 + mu'_1 eta (f_F(u_0) + S_V), u_0 = V (in
  // the mixed precision S_V is a float value, so it equals what is stored)
  const double FV = FVfun();
  const double u1 = first_inner(a.mu1_eta, V, FV, SV);
  if (a.m_is_one) {
    const double fbarV = (u1 - V) * a.inv_eta;
    gptr(a.uout)[i] = a.j1 ? V + a.mu_dt * fbarV : a.nu * V + a.kappa * gptr(a.Vin2)[i] + a.mu_dt * fbarV;
  } else {
    gptr(a.uout)[i] = u1;
    if (MIXED)
      gptr((float *)a.SV)[i] = (float)SV;
    else
      gptr((double *)a.SV)[i] = SV;
  }
}

template <template <class> class Model, bool MIXED>
__device__ __forceinline__ void head_flat(const HeadArgs &a, const Mesh &mesh) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t i = node_index();
  if (i >= N) return;
  const double V = a.Vin[i];
  head_node<Model, MIXED>(a, N, i, V, [&]() { return apply_op<MIXED>(mesh, a.Vin, i); });
}

template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_head(HeadArgs a, Mesh mesh) {
  head_flat<Model, MIXED>(a, mesh);
}

// The mixed-precision flat head compiled for at least 7 resident waves per
// SIMD (at most 72 registers): on grids of about one round of waves the
// extra wave removes the tail round.  (The FP64 head would spill at the
// corresponding budget, and gains nothing.)
template <template <class> class Model>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_head_occ(HeadArgs a,
                                                                                               Mesh mesh) {
  head_flat<Model, true>(a, mesh);
}

// Pointwise head of the split stage (m >= 2): exponential Euler, ionic
// model, outer z recurrence and S_V at each node, in index order with no
// stencil (the first inner stage moves to k_inner12_march).  On the large
// slab this keeps the head a pure stream of the ionic state: the 27 V
// operands of the flat head cost it about a tenth of its time.
template <template <class> class Model, bool MIXED, bool NT>
__global__ __launch_bounds__(kBlock) void k_head_pw(HeadArgs a, uint32_t N) {
  const uint32_t i = node_index();
  if (i >= N) return;
  head_node<Model, MIXED, true, NT>(a, N, i, a.Vin[i], []() { return 0.0; });
}

// ---------------------------------------------------------------------------
// EXEX-RL reference step (the IMEX-RL algorithm of the numerical experiments
// with its diffusion line taken explicitly): Rush-Larsen for the gates at
// V^n, explicit Euler for the other ionic variables with the new gates,
// explicit Euler for V with the ionic current at (V^n, z_E^{n+1}, z_S^{n+1}).
// ---------------------------------------------------------------------------
template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_exexrl(ExArgs a, Mesh mesh) {
  using M = MathOf<MIXED>;
  using R = typename M::R;
  using Mod = Model<M>;
  constexpr int NG = Mod::NG, NS = Mod::NS, NZ = NG + NS;
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t i = node_index();
  if (i >= N) return;
  const double V = a.Vin[i];
  const double tn = stage_time(a.clock, a.step_off, a.dt, 0.0);
  const double Is = stimulus(a.stim, i, tn);
  R *zp = (R *)a.z;
  R z[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) z[k] = zp[(size_t)k * N + i];
  R lam[NG], zinf[NG];
  Mod::gates(R(V), a.mp, lam, zinf);
  const R dt = R(a.dt);
#pragma unroll
  for (int g = 0; g < NG; ++g) z[g] = z[g] + M::expm1(dt * lam[g]) * (z[g] - zinf[g]);
  R dS[NS > 0 ? NS : 1];
  R iion = Mod::eval(R(V), z, z + NG, dS, a.mp);
  if (NS > 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) z[NG + k] = z[NG + k] + dt * dS[k];
    iion = Mod::eval(R(V), z, z + NG, dS, a.mp);
  }
#pragma unroll
  for (int k = 0; k < NZ; ++k) zp[(size_t)k * N + i] = z[k];
  double SV;
  if (MIXED)
    SV = (double)((R(Is) - R(a.Cm) * iion) * R(1.0 / a.Cm));
  else
    SV = (Is - a.Cm * (double)iion) / a.Cm;
  const double FV = apply_op<MIXED>(mesh, a.Vin, i);
  a.Vout[i] = V + a.dt * (FV + SV);
}

// IMEX-RL pointwise part: the gate and slow-variable updates of k_exexrl,
// then the right-hand side of the implicit diffusion line instead of the
// explicit V update.
template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_imexrl_pre(ImexArgs a, uint32_t N) {
  using M = MathOf<MIXED>;
  using R = typename M::R;
  using Mod = Model<M>;
  constexpr int NG = Mod::NG, NS = Mod::NS, NZ = NG + NS;
  const uint32_t i = node_index();
  if (i >= N) return;
  const double V = a.V[i];
  const double Is = stimulus(a.stim, i, a.t);
  R *zp = (R *)a.z;
  R z[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) z[k] = zp[(size_t)k * N + i];
  R lam[NG], zinf[NG];
  Mod::gates(R(V), a.mp, lam, zinf);
  const R dt = R(a.dt);
#pragma unroll
  for (int g = 0; g < NG; ++g) z[g] = z[g] + M::expm1(dt * lam[g]) * (z[g] - zinf[g]);
  R dS[NS > 0 ? NS : 1];
  R iion = Mod::eval(R(V), z, z + NG, dS, a.mp);
  if (NS > 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) z[NG + k] = z[NG + k] + dt * dS[k];
    iion = Mod::eval(R(V), z, z + NG, dS, a.mp);
  }
#pragma unroll
  for (int k = 0; k < NZ; ++k) zp[(size_t)k * N + i] = z[k];
  double SV;
  if (MIXED)
    SV = (double)((R(Is) - R(a.Cm) * iion) * R(1.0 / a.Cm));
  else
    SV = (Is - a.Cm * (double)iion) / a.Cm;
  a.rhs[i] = V + a.dt * SV;
}

// ---------------------------------------------------------------------------
// Inner stages
// ---------------------------------------------------------------------------
__device__ __forceinline__ double load_sv(const void *SV, bool mixed, uint32_t i) {
  return mixed ? (double)gptr((const float *)SV)[i] : gptr((const double *)SV)[i];
}

// u_k = nu u_{k-1} + kappa u_{k-2} + mu eta (f_F(u_{k-1}) + S_V)
// The combinations are written with explicit fused multiply-adds and no
// further contraction, so that every kernel that evaluates them (flat,
// tiled, z-marching, fused, batched) rounds identically.
__device__ __forceinline__ double inner_combine(const TailArgs &t, double uc, double u2, double Fu, double sv) {
#pragma clang fp contract(off)
  return __builtin_fma(t.nu, uc, __builtin_fma(t.kappa, u2, t.mu_eta * (Fu + sv)));
}

__device__ __forceinline__ double tail_combine(const TailArgs &t, double um, double vp, double vp2) {
#pragma clang fp contract(off)
  const double fbar = (um - vp) * t.inv_eta;
  return t.j1 ? __builtin_fma(t.mu_dt, fbar, vp)
              : __builtin_fma(t.nu_o, vp, __builtin_fma(t.kappa_o, vp2, t.mu_dt * fbar));
}

__device__ __forceinline__ double inner_value(const TailArgs &t, double Fu, double sv, uint32_t i) {
  return inner_combine(t, t.uprev[i], t.uprev2[i], Fu, sv);
}

// outer V update from the last inner value: V_j = nu V_{j-1} + kappa V_{j-2}
// + mu dt (u_m - V_{j-1})/eta
__device__ __forceinline__ double tail_from_um(const TailArgs &t, double um, uint32_t i) {
  return tail_combine(t, um, t.Vin[i], t.j1 ? 0.0 : t.Vin2[i]);
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_inner(InnerArgs a, Mesh mesh) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t i = node_index();
  if (a.tick != nullptr && blockIdx.x == 0 && threadIdx.x == 0) a.tick->step += a.tick_by;
  if (i >= N) return;
  const double Fu = apply_op<MIXED>(mesh, a.t.uprev, i);
  const double sv = load_sv(a.t.SV, MIXED, i);
  if (a.first) {
    a.out[i] = first_inner(a.t.mu_eta, a.t.uprev[i], Fu, sv);
    return;
  }
  const double uk = inner_value(a.t, Fu, sv, i);
  a.out[i] = a.last ? tail_from_um(a.t, uk, i) : uk;
}

// ---------------------------------------------------------------------------
// mRKC (double precision, flat kernels).  The fast term is f_F plus the rate
// of gate 0 (the stiffest gate), the slow term f_S plus the rates of the
// other gates; there is no exponential stage.  The head of outer stage j
// evaluates the slow term at y_{j-1}, finishes the outer recurrence of every
// component except V and gate 0 (their inner problems have constant
// forcing, so they end at z + c'_m eta S), and takes the first inner stage
// of V and gate 0; the inner stages advance both, with the gate-0 rate at
// the current inner V.
// ---------------------------------------------------------------------------
template <template <class> class Model>
__global__ __launch_bounds__(kBlock) void k_mrkc_head(MrkcHeadArgs ma, Mesh mesh) {
  using M = MathF64;
  using Mod = Model<M>;
  constexpr int NG = Mod::NG, NS = Mod::NS, NZ = NG + NS;
  const HeadArgs &a = ma.h;
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t i = node_index();
  if (i >= N) return;
  const double V = a.Vin[i];
  const double tj = stage_time(a.clock, a.step_off, a.dt, a.c_prev);
  const double Is = stimulus(a.stim, i, tj);
  const double *zin = (const double *)a.zin;
  const double *zin2 = (const double *)a.zin2;
  double *zout = (double *)a.zout;
  double z[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) z[k] = zin[(size_t)k * N + i];
  double lam[NG], zinf[NG];
  Mod::gates(V, a.mp, lam, zinf);
  double dS[NS > 0 ? NS : 1];
  const double iion = Mod::eval(V, z, z + NG, dS, a.mp);
  const double SV = (Is - a.Cm * iion) / a.Cm;
#pragma unroll
  for (int k = 1; k < NZ; ++k) {
    const double S = k < NG ? lam[k] * (z[k] - zinf[k]) : dS[k - NG];
    const double um = z[k] + a.cm_eta * S;
    const double fbar = (um - z[k]) * a.inv_eta;
    zout[(size_t)k * N + i] =
        a.j1 ? z[k] + a.mu_dt * fbar : a.nu * z[k] + a.kappa * zin2[(size_t)k * N + i] + a.mu_dt * fbar;
  }
  const double g0 = lam[0] * (z[0] - zinf[0]);
  const double FV = apply_op<false>(mesh, a.Vin, i);
  const double u1 = V + a.mu1_eta * (FV + SV);
  const double w1 = z[0] + a.mu1_eta * g0;
  if (a.m_is_one) {
    const double fbarV = (u1 - V) * a.inv_eta;
    const double fbarW = (w1 - z[0]) * a.inv_eta;
    a.uout[i] = a.j1 ? V + a.mu_dt * fbarV : a.nu * V + a.kappa * a.Vin2[i] + a.mu_dt * fbarV;
    zout[i] = a.j1 ? z[0] + a.mu_dt * fbarW : a.nu * z[0] + a.kappa * zin2[i] + a.mu_dt * fbarW;
  } else {
    a.uout[i] = u1;
    ma.wout[i] = w1;
    ((double *)a.SV)[i] = SV;
  }
}

template <template <class> class Model>
__global__ __launch_bounds__(kBlock) void k_mrkc_inner(MrkcInnerArgs ma, Mesh mesh) {
  using M = MathF64;
  using Mod = Model<M>;
  const InnerArgs &a = ma.a;
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t i = node_index();
  if (a.tick != nullptr && blockIdx.x == 0 && threadIdx.x == 0) a.tick->step += a.tick_by;
  if (i >= N) return;
  const double u = a.t.uprev[i];
  const double w = ma.wprev[i];
  double lam0, zinf0;
  Mod::gate0(u, ma.mp, lam0, zinf0);
  const double g = lam0 * (w - zinf0);
  const double Fu = apply_op<false>(mesh, a.t.uprev, i);
  const double uk = inner_combine(a.t, u, a.t.uprev2[i], Fu, load_sv(a.t.SV, false, i));
  const double wk = inner_combine(a.t, w, ma.wprev2[i], g, 0.0);
  if (a.last) {
    a.out[i] = tail_combine(a.t, uk, a.t.Vin[i], a.t.j1 ? 0.0 : a.t.Vin2[i]);
    ma.zq_out[i] = tail_combine(a.t, wk, ma.zq_in[i], a.t.j1 ? 0.0 : ma.zq_in2[i]);
  } else {
    a.out[i] = uk;
    ma.wout[i] = wk;
  }
}

template <template <class> class Model>
__global__ __launch_bounds__(kBlock) void k_mrkc_rhs(int which, Mesh mesh, uint32_t N, double t, const double *y,
                                                     double *out, StimArgs stim, double Cm, ModelParams mp) {
  using M = MathF64;
  using Mod = Model<M>;
  constexpr int NG = Mod::NG, NS = Mod::NS, NZ = NG + NS;
  const uint32_t i = node_index();
  if (i >= N) return;
  const double V = y[i];
  double z[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) z[k] = y[(size_t)(k + 1) * N + i];
  double lam[NG], zinf[NG];
  Mod::gates(V, mp, lam, zinf);
  if (which == 0) {
    out[i] = apply_op<false>(mesh, y, i);
    out[(size_t)N + i] = lam[0] * (z[0] - zinf[0]);
#pragma unroll
    for (int k = 1; k < NZ; ++k) out[(size_t)(k + 1) * N + i] = 0.0;
    return;
  }
  double dS[NS > 0 ? NS : 1];
  const double iion = Mod::eval(V, z, z + NG, dS, mp);
  out[i] = (stimulus(stim, i, t) - Cm * iion) / Cm;
  out[(size_t)N + i] = 0.0;
#pragma unroll
  for (int k = 1; k < NZ; ++k)
    out[(size_t)(k + 1) * N + i] = k < NG ? lam[k] * (z[k] - zinf[k]) : dS[k - NG];
}

// ---------------------------------------------------------------------------
// Fused tail + head on a structured grid.  Each block owns a TX x TY x TZ
// tile; phase 1 computes V^n on the tile plus a one-node halo (mirrored at
// the domain boundary) into LDS, phase 2 runs the head of the next step on
// the tile's own nodes with f_F(V^n) taken from LDS.  The arithmetic is the
// same as k_inner (last) followed by k_head.
// ---------------------------------------------------------------------------
// Tile shapes of 256 nodes: SH = 0 (the default) 16x4x4 / 64x4, SH = 1
// 32x4x2 / 32x8, SH = 2 8x8x4 / 128x2 (3-D / 2-D).
template <int DIM, int SH = 0>
struct Tile {
  static constexpr int TX = DIM == 3 ? (SH == 0 ? 16 : SH == 1 ? 32 : 8) : (SH == 0 ? 64 : SH == 1 ? 32 : 128);
  static constexpr int TY = DIM == 3 ? (SH == 2 ? 8 : 4) : (SH == 0 ? 4 : SH == 1 ? 8 : 2);
  static constexpr int TZ = DIM == 3 ? (SH == 1 ? 2 : 4) : 1;
  static constexpr int SX = TX + 2, SY = TY + 2, SZ = DIM == 3 ? TZ + 2 : 1;
  static constexpr int NS = SX * SY * SZ;
  static_assert(TX * TY * TZ == kBlock, "one node per thread");
};

__device__ __forceinline__ uint32_t mirror_any(int c, uint32_t n) {
  int r = c < 0 ? -c : (c >= (int)n ? 2 * ((int)n - 1) - c : c);
  r = r < 0 ? 0 : (r > (int)n - 1 ? (int)n - 1 : r);
  return (uint32_t)r;
}

template <template <class> class Model, bool MIXED, int DIM>
__global__ __launch_bounds__(kBlock) void k_fused(FusedArgs a, Grid g, uint32_t ntx, uint32_t nty) {
  using T = Tile<DIM>;
  __shared__ double sV[T::NS];
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bx = b % ntx, byz = b / ntx;
  const uint32_t by = byz % nty, bz = byz / nty;
  const int x0 = (int)(bx * T::TX), y0 = (int)(by * T::TY), z0 = (int)(bz * T::TZ);

  for (int r = threadIdx.x; r < T::NS; r += kBlock) {
    const int hx = r % T::SX, hy = (r / T::SX) % T::SY, hz = r / (T::SX * T::SY);
    const uint32_t gx = mirror_any(x0 + hx - 1, g.n0);
    const uint32_t gy = mirror_any(y0 + hy - 1, g.n1);
    const uint32_t gz = DIM == 3 ? mirror_any(z0 + hz - 1, g.n2) : 0u;
    const uint32_t i = gx + g.n0 * (gy + g.n1 * gz);
    const double Fu = grid_apply<DIM>(a.t.uprev, g, gx, gy, gz);
    const double um = inner_value(a.t, Fu, load_sv(a.t.SV, MIXED, i), i);
    sV[r] = tail_from_um(a.t, um, i);
  }
  __syncthreads();

  const int lx = threadIdx.x % T::TX, ly = (threadIdx.x / T::TX) % T::TY, lz = threadIdx.x / (T::TX * T::TY);
  const uint32_t gx = (uint32_t)(x0 + lx), gy = (uint32_t)(y0 + ly), gz = (uint32_t)(z0 + lz);
  if (gx >= g.n0 || gy >= g.n1 || (DIM == 3 && gz >= g.n2)) return;
  const uint32_t i = gx + g.n0 * (gy + g.n1 * (DIM == 3 ? gz : 0u));
  const int c = ((DIM == 3 ? lz + 1 : 0) * T::SY + (ly + 1)) * T::SX + (lx + 1);
  const double V = sV[c];
  a.Vout[i] = V;
  head_node<Model, MIXED>(a.h, g.N, i, V, [&]() {
    return grid_stencil<DIM>(g.w, [&](int dx, int dy, int dz) {
      return sV[c + (DIM == 3 ? dz * T::SX * T::SY : 0) + dy * T::SX + dx];
    });
  });
}

// ---------------------------------------------------------------------------
// LDS-tiled head and inner kernels for structured grids.  Each block owns a
// tile, stages the operand of the stencil on the tile plus a one-node halo
// (mirrored at the domain boundary) in LDS with coalesced loads, and
// evaluates the stencil from LDS; the arithmetic is the same as the flat
// kernels'.
// ---------------------------------------------------------------------------
template <int DIM, int SH = 0>
__device__ __forceinline__ void tile_origin(uint32_t ntx, uint32_t nty, int &x0, int &y0, int &z0) {
  using T = Tile<DIM, SH>;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bx = b % ntx, byz = b / ntx;
  const uint32_t by = byz % nty, bz = byz / nty;
  x0 = (int)(bx * T::TX);
  y0 = (int)(by * T::TY);
  z0 = (int)(bz * T::TZ);
}

// All of a thread's halo loads are issued before the first is stored (one
// memory latency instead of one per load); slots beyond the halo load its
// last position again and store nothing.
template <int DIM, int SH = 0>
struct Halo {
  using T = Tile<DIM, SH>;
  static constexpr int NSL = (T::NS + kBlock - 1) / kBlock;
  double v[NSL];
  __device__ __forceinline__ void load(const double *__restrict__ u, const Grid &g, int x0, int y0, int z0) {
#pragma unroll
    for (int k = 0; k < NSL; ++k) {
      const int r = min((int)threadIdx.x + k * kBlock, T::NS - 1);
      const int hx = r % T::SX, hy = (r / T::SX) % T::SY, hz = r / (T::SX * T::SY);
      const uint32_t gx = mirror_any(x0 + hx - 1, g.n0);
      const uint32_t gy = mirror_any(y0 + hy - 1, g.n1);
      const uint32_t gz = DIM == 3 ? mirror_any(z0 + hz - 1, g.n2) : 0u;
      v[k] = gptr(u)[gx + g.n0 * (gy + g.n1 * gz)];
    }
  }
  __device__ __forceinline__ void store(double *sU) const {
#pragma unroll
    for (int k = 0; k < NSL; ++k) {
      const int r = (int)threadIdx.x + k * kBlock;
      if (r < T::NS) sU[r] = v[k];
    }
  }
};

template <int DIM, int SH = 0>
__device__ __forceinline__ void stage_halo(double *sU, const double *__restrict__ u, const Grid &g, int x0, int y0,
                                           int z0) {
  Halo<DIM, SH> h;
  h.load(u, g, x0, y0, z0);
  h.store(sU);
}

// Own node of this thread in the tile: global index (or false when outside
// the grid) and the LDS index of the node's centre.
template <int DIM, int SH = 0>
__device__ __forceinline__ bool tile_node(const Grid &g, int x0, int y0, int z0, uint32_t &i, int &c) {
  using T = Tile<DIM, SH>;
  const int lx = threadIdx.x % T::TX, ly = (threadIdx.x / T::TX) % T::TY, lz = threadIdx.x / (T::TX * T::TY);
  const uint32_t gx = (uint32_t)(x0 + lx), gy = (uint32_t)(y0 + ly), gz = (uint32_t)(z0 + lz);
  if (gx >= g.n0 || gy >= g.n1 || (DIM == 3 && gz >= g.n2)) return false;
  i = gx + g.n0 * (gy + g.n1 * (DIM == 3 ? gz : 0u));
  c = ((DIM == 3 ? lz + 1 : 0) * T::SY + (ly + 1)) * T::SX + (lx + 1);
  return true;
}

template <int DIM, int SH = 0>
__device__ __forceinline__ double lds_stencil(const double *sU, const Grid &g, int c) {
  using T = Tile<DIM, SH>;
  return grid_stencil<DIM>(g.w, [&](int dx, int dy, int dz) {
    return sU[c + (DIM == 3 ? dz * T::SX * T::SY : 0) + dy * T::SX + dx];
  });
}

// Tiled head at this thread's node of the tile at (x0, y0, z0): V with its
// halo staged in LDS, then the node's head.  z planes are Nplane apart; the
// node's index is off + its index in the grid g; Vg is V of that grid.
// (Loading the node's ionic state before the barrier, as the inner stage
// does with its operands, measured slower here: the state's registers are
// held across the staging.)
template <template <class> class Model, bool MIXED, int DIM, int SH>
__device__ __forceinline__ void head_tiled_node(const HeadArgs &a, const Grid &g, uint32_t Nplane, uint32_t off,
                                                const double *Vg, int x0, int y0, int z0, double *sV) {
  stage_halo<DIM, SH>(sV, Vg, g, x0, y0, z0);
  __syncthreads();
  uint32_t il;
  int c;
  if (!tile_node<DIM, SH>(g, x0, y0, z0, il, c)) return;
  head_node<Model, MIXED>(a, Nplane, off + il, sV[c], [&]() { return lds_stencil<DIM, SH>(sV, g, c); });
}

template <template <class> class Model, bool MIXED, int DIM>
__global__ __launch_bounds__(kBlock) void k_head_tiled(HeadArgs a, Grid g, uint32_t ntx, uint32_t nty) {
  __shared__ double sV[Tile<DIM>::NS];
  int x0, y0, z0;
  tile_origin<DIM>(ntx, nty, x0, y0, z0);
  head_tiled_node<Model, MIXED, DIM, 0>(a, g, g.N, 0u, a.Vin, x0, y0, z0, sV);
}

// The tiled head compiled for at least WPE resident waves per SIMD (fewer
// registers, possibly spilled): one round of blocks on small grids.
template <template <class> class Model, bool MIXED, int DIM, int WPE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void k_head_tiled_occ(
    HeadArgs a, Grid g, uint32_t ntx, uint32_t nty) {
  __shared__ double sV[Tile<DIM>::NS];
  int x0, y0, z0;
  tile_origin<DIM>(ntx, nty, x0, y0, z0);
  head_tiled_node<Model, MIXED, DIM, 0>(a, g, g.N, 0u, a.Vin, x0, y0, z0, sV);
}

// Pointwise operands of an inner stage at one node, loaded a plane ahead.
// S_V stays in its storage type (float in the mixed form) until it is used:
// converting it where it is loaded would wait for the load there, which
// undoes the prefetch of the next plane's operands
template <bool MIXED>
struct InnerPoint {
  double u2;
  typename std::conditional<MIXED, float, double>::type sv;
  double vp, vp2;
};

template <bool MIXED>
__device__ __forceinline__ InnerPoint<MIXED> load_point(const InnerArgs &a, uint32_t i) {
  InnerPoint<MIXED> p;
  p.u2 = a.first ? 0.0 : gptr(a.t.uprev2)[i];
  p.sv = gptr((const decltype(p.sv) *)a.t.SV)[i];
  p.vp = 0.0;
  p.vp2 = 0.0;
  if (a.last) {
    // m == 2: u_0 is V_{j-1}, taken from u2 where it is used (a copy here
    // would wait for that load before the next ones are issued)
    if (a.t.uprev2 != a.t.Vin) p.vp = gptr(a.t.Vin)[i];
    if (!a.t.j1) p.vp2 = gptr(a.t.Vin2)[i];
  }
  return p;
}

// inner_value / tail_from_um with the operands given (same expressions);
// the first inner stage (a.first) is u_1 = u_0 + mu'_1 eta (f_F(u_0) + S_V)
template <bool MIXED>
__device__ __forceinline__ double inner_point(const InnerArgs &a, double uc, double Fu, const InnerPoint<MIXED> &p) {
  const double sv = (double)p.sv;
  if (a.first) return first_inner(a.t.mu_eta, uc, Fu, sv);
  const double uk = inner_combine(a.t, uc, p.u2, Fu, sv);
  return a.last ? tail_combine(a.t, uk, a.t.uprev2 == a.t.Vin ? p.u2 : p.vp, p.vp2) : uk;
}

// The node's pointwise operands are loaded before the halo is staged (both
// in flight together; global loads cannot move across the barrier).
template <bool MIXED, int DIM>
__global__ __launch_bounds__(kBlock) void k_inner_tiled(InnerArgs a, Grid g, uint32_t ntx, uint32_t nty) {
  __shared__ double sU[Tile<DIM>::NS];
  if (a.tick != nullptr && blockIdx.x == 0 && threadIdx.x == 0) a.tick->step += a.tick_by;
  int x0, y0, z0;
  tile_origin<DIM>(ntx, nty, x0, y0, z0);
  uint32_t i;
  int c;
  const bool own = tile_node<DIM>(g, x0, y0, z0, i, c);
  InnerPoint<MIXED> pt{};
  if (own) pt = load_point<MIXED>(a, i);
  stage_halo<DIM>(sU, a.t.uprev, g, x0, y0, z0);
  __syncthreads();
  if (!own) return;
  const double Fu = lds_stencil<DIM>(sU, g, c);
  a.out[i] = inner_point(a, sU[c], Fu, pt);
}

// ---------------------------------------------------------------------------
// Inner stage on 3-D grids by z-marching columns (2.5-D): a block owns an
// MX x MY column of zc planes and keeps the planes z-1, z, z+1 of u_{k-1}
// (with a one-node mirrored halo in x and y) in an LDS ring; plane z+2 is
// loaded into registers while plane z is computed.  Each plane is read
// from memory once per column instead of once per neighbouring tile.
// ---------------------------------------------------------------------------
constexpr int MSX = MX + 2, MSY = MY + 2, MPL = MSX * MSY;
constexpr int MSLOT = (MPL + kBlock - 1) / kBlock;

// One column (block b of the grid's columns, x fastest) of the z-marching
// inner stage; the grid's nodes start at index `base` of every array (a
// batched instance), and ring is the block's LDS.
template <bool MIXED>
__device__ __forceinline__ void inner_march_col(const InnerArgs &a, const Grid &g, uint32_t base, uint32_t b,
                                                uint32_t ncx, uint32_t ncy, double (*ring)[MPL]) {
  const uint32_t bx = b % ncx, byz = b / ncx;
  const uint32_t by = byz % ncy, bz = byz / ncy;
  const int x0 = (int)(bx * MX), y0 = (int)(by * MY);
  const int zb = (int)(bz * g.zc);
  const int ze = min(zb + (int)g.zc, (int)g.n2);
  const uint32_t plane = g.n0 * g.n1;
  // this thread's staging slots of a plane (xy offsets with mirrored halo)
  uint32_t off[MSLOT];
  bool act[MSLOT];
#pragma unroll
  for (int k = 0; k < MSLOT; ++k) {
    const int r = threadIdx.x + k * kBlock;
    act[k] = r < MPL;
    const int hx = r % MSX, hy = r / MSX;
    off[k] = act[k] ? mirror_any(x0 + hx - 1, g.n0) + g.n0 * mirror_any(y0 + hy - 1, g.n1) : 0u;
  }
  const auto u = gptr(a.t.uprev + base);
  const auto out = gptr(a.out + base);
  auto gplane = [&](int z) { return (size_t)mirror_any(z, g.n2) * plane; };
  // Every load is unconditional (inactive slots read offset 0 of the plane,
  // nodes outside the grid the nearest node, values never used), so that
  // the loads of the first three planes and of the first node's operands
  // are all in flight together, and the compiler can count the loads it
  // waits for.
  double pre[MSLOT], s0[MSLOT], s1[MSLOT];
  {
    const size_t pa = gplane(zb - 1), pb = gplane(zb), pc = gplane(zb + 1);
#pragma unroll
    for (int k = 0; k < MSLOT; ++k) {
      s0[k] = u[pa + off[k]];
      s1[k] = u[pb + off[k]];
      pre[k] = u[pc + off[k]];
    }
  }
  const int lx = threadIdx.x % MX, ly = threadIdx.x / MX;
  const uint32_t gx = (uint32_t)(x0 + lx), gy = (uint32_t)(y0 + ly);
  const bool own = gx < g.n0 && gy < g.n1;
  const int c = (ly + 1) * MSX + (lx + 1);
  // the node whose operands are loaded: this thread's own node, or the
  // nearest node of the grid for threads beyond its edge
  uint32_t i = min(gx, g.n0 - 1) + g.n0 * min(gy, g.n1 - 1) + plane * (uint32_t)zb;
  InnerPoint<MIXED> pt = load_point<MIXED>(a, base + i);
  // slot of plane p is p mod 3 (p >= -1)
#pragma unroll
  for (int k = 0; k < MSLOT; ++k)
    if (act[k]) {
      ring[(zb + 2) % 3][threadIdx.x + k * kBlock] = s0[k];
      ring[zb % 3][threadIdx.x + k * kBlock] = s1[k];
    }
  for (int z = zb; z < ze; ++z, i += plane) {
    double *nxt = ring[(z + 1) % 3];
#pragma unroll
    for (int k = 0; k < MSLOT; ++k)
      if (act[k]) nxt[threadIdx.x + k * kBlock] = pre[k];
    __syncthreads();
    const InnerPoint<MIXED> cur = pt;
    if (z + 1 < ze) {
      const size_t pz = gplane(z + 2);
#pragma unroll
      for (int k = 0; k < MSLOT; ++k) pre[k] = u[pz + off[k]];
      pt = load_point<MIXED>(a, base + i + plane);
    }
    if (own) {
      const double *pm = ring[(z + 2) % 3], *pc = ring[z % 3], *pp = ring[(z + 1) % 3];
      const double Fu = grid_stencil<3>(g.w, [&](int dx, int dy, int dz) {
        const double *pl = dz < 0 ? pm : (dz > 0 ? pp : pc);
        return pl[c + dy * MSX + dx];
      });
      out[i] = inner_point(a, pc[c], Fu, cur);
    }
    __syncthreads();
  }
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_inner_march(InnerArgs a, Grid g, uint32_t ncx, uint32_t ncy) {
  __shared__ double ring[3][MPL];
  if (a.tick != nullptr && blockIdx.x == 0 && threadIdx.x == 0) a.tick->step += a.tick_by;
  inner_march_col<MIXED>(a, g, 0u, xcd_block(blockIdx.x, gridDim.x), ncx, ncy, ring);
}

// ---------------------------------------------------------------------------
// First two inner stages of the split stage on 3-D grids, by z-marching
// columns: u_1 = u_0 + mu'_1 eta (f_F(u_0) + S_V) with u_0 = V_{j-1}, then
// u_2 = nu'_2 u_1 + kappa'_2 u_0 + mu'_2 eta (f_F(u_1) + S_V), and, when
// m == 2, the outer V update.  A block owns an MX x MY column of zc planes.
// V_{j-1} is staged in LDS with a two-node halo in x and y (a ring of four
// planes), and u_1 is formed on a one-node halo from the stencil's plane
// terms of V (grid_stencil), each plane's terms formed once per halo
// position and kept: in registers for the first kBlock positions, in a
// thread-private LDS ring for the remaining ones.  The newest u_1 plane
// goes to LDS, and the node's own u_1 plane terms stay in registers, so
// each plane costs 9 LDS reads per halo position and per node instead of
// 27.  V plane z+3 and the halo's S_V of plane z+2 are loaded into
// registers while plane z is computed.  Positions beyond the grid are
// reflected at both ends (mirror2; at most twice, for two-node axes), so
// that u_1 on the halo equals u_1 at the reflected node: the plane terms
// pair opposite neighbours, and exchanging the two members of every pair
// (or the planes above and below) leaves each sum's bits unchanged.
// ---------------------------------------------------------------------------
constexpr int VSX = MX + 4, VSY = MY + 4, VPL = VSX * VSY;
constexpr int VSLOT = (VPL + kBlock - 1) / kBlock;
constexpr int UXTRA = MPL - kBlock;  // halo positions beyond one per thread
static_assert(UXTRA > 0 && UXTRA <= kBlock, "one or two u_1 halo positions per thread");

__device__ __forceinline__ uint32_t mirror2(int c, uint32_t n) {
  int r = c < 0 ? -c : c;
  r = r > (int)n - 1 ? 2 * ((int)n - 1) - r : r;
  r = r < 0 ? -r : r;
  return (uint32_t)(r > (int)n - 1 ? (int)n - 1 : r);
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_inner12_march(
    Inner12Args a, Grid g, uint32_t ncx, uint32_t ncy) {
  // ring slots are numbered from the column's first plane zb: plane zb + c
  // sits in slot c mod 4 (c >= -2), so that with the loop unrolled by four
  // every slot index is a constant
  __shared__ double vring[4][VPL];       // V planes
  __shared__ double uring[MPL];          // the newest u_1 plane
  __shared__ double xring[4][3][UXTRA];  // V plane terms (c, o, t) at the extra positions
  if (a.tick != nullptr && blockIdx.x == 0 && threadIdx.x == 0) a.tick->step += a.tick_by;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bx = b % ncx, byz = b / ncx;
  const uint32_t by = byz % ncy, bz = byz / ncy;
  const int x0 = (int)(bx * MX), y0 = (int)(by * MY);
  const int zb = (int)(bz * g.zc);
  const int ze = min(zb + (int)g.zc, (int)g.n2);
  const uint32_t plane = g.n0 * g.n1;
  // V staging slots (two-node halo)
  uint32_t voff[VSLOT];
  bool vact[VSLOT];
#pragma unroll
  for (int k = 0; k < VSLOT; ++k) {
    const int r = threadIdx.x + k * kBlock;
    vact[k] = r < VPL;
    const int hx = r % VSX, hy = r / VSX;
    voff[k] = vact[k] ? mirror2(x0 + hx - 2, g.n0) + g.n0 * mirror2(y0 + hy - 2, g.n1) : 0u;
  }
  // u_1 halo positions: threadIdx.x, and kBlock + threadIdx.x for the
  // first UXTRA threads (global in-plane offset for S_V, V-ring index)
  const bool xact = threadIdx.x < UXTRA;
  uint32_t uoff[2];
  int ucv[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = k == 0 ? (int)threadIdx.x : (xact ? kBlock + (int)threadIdx.x : 0);
    const int hx = r % MSX, hy = r / MSX;
    uoff[k] = mirror2(x0 + hx - 1, g.n0) + g.n0 * mirror2(y0 + hy - 1, g.n1);
    ucv[k] = (hy + 1) * VSX + (hx + 1);
  }
  const auto V = gptr(a.V);
  auto vplane = [&](int z) { return (size_t)mirror2(z, g.n2) * plane; };
  // Every load is unconditional (inactive slots read offset 0 of the plane,
  // threads beyond the grid the nearest node, planes beyond the column
  // reflected; nothing they load is used), so that the prologue's loads are
  // all in flight together and the compiler can count the loads it waits
  // for.
  auto load_v = [&](int z, double *v) {
    const size_t pz = vplane(z);
#pragma unroll
    for (int k = 0; k < VSLOT; ++k) v[k] = V[pz + voff[k]];
  };
  auto put_v = [&](int s, const double *v) {
    double *dst = vring[s];
#pragma unroll
    for (int k = 0; k < VSLOT; ++k)
      if (vact[k]) dst[threadIdx.x + k * kBlock] = v[k];
  };
  // S_V is kept in its storage type (float in the mixed form) until it is
  // used: a conversion at the load would wait for the load there
  using SR = typename std::conditional<MIXED, float, double>::type;
  const auto SVg = gptr((const SR *)a.SV);
  auto load_svh = [&](int z, SR *sv) {
    const size_t pz = vplane(z);
#pragma unroll
    for (int k = 0; k < 2; ++k) sv[k] = SVg[pz + uoff[k]];
  };
  // V plane terms of the plane in slot s at halo position k
  auto vterms = [&](int s, int k) {
    const double *src = vring[s];
    const int cc = ucv[k];
    return plane_terms(g.w, [&](int dx, int dy) { return src[cc + dy * VSX + dx]; });
  };
  auto xput = [&](int s, const PlaneTerms &v) {
    xring[s][0][threadIdx.x] = v.c;
    xring[s][1][threadIdx.x] = v.o;
    xring[s][2][threadIdx.x] = v.t;
  };
  auto xget = [&](int s) {
    return PlaneTerms{xring[s][0][threadIdx.x], xring[s][1][threadIdx.x], xring[s][2][threadIdx.x]};
  };
  // u_1 at halo position k of the plane whose V terms are o (m below, p above)
  auto put_u = [&](int k, const PlaneTerms &m, const PlaneTerms &o, const PlaneTerms &p, double sv) {
    uring[threadIdx.x + k * kBlock] = first_inner(a.mu1_eta, o.c, plane_combine(g.w, m, o, p), sv);
  };
  const int lx = threadIdx.x % MX, ly = threadIdx.x / MX;
  const uint32_t gx = (uint32_t)(x0 + lx), gy = (uint32_t)(y0 + ly);
  const bool own = gx < g.n0 && gy < g.n1;
  const int cu = (ly + 1) * MSX + (lx + 1);
  const int cv = (ly + 2) * VSX + (lx + 2);
  auto uterms = [&]() { return plane_terms(g.w, [&](int dx, int dy) { return uring[cu + dy * MSX + dx]; }); };
  // the node whose operands are loaded: this thread's own node, or the
  // nearest node of the grid for threads beyond its edge
  uint32_t i = min(gx, g.n0 - 1) + g.n0 * min(gy, g.n1 - 1) + plane * (uint32_t)zb;
  const bool need_v2 = a.last && !a.t.j1;
  // the prologue: V planes zb - 2 .. zb + 2, the halo's S_V of planes
  // zb - 1 .. zb + 1 and the first node's operands, all loaded at once
  double v0[VSLOT], v1[VSLOT], v2[VSLOT], v3[VSLOT], vpre[VSLOT];
  SR svm[2], sv0[2], svpre[2];
  load_v(zb - 2, v0);
  load_v(zb - 1, v1);
  load_v(zb, v2);
  load_v(zb + 1, v3);
  load_v(zb + 2, vpre);
  load_svh(zb - 1, svm);
  load_svh(zb, sv0);
  load_svh(zb + 1, svpre);
  const auto Vin2 = gptr(a.Vin2);
  const auto out = gptr(a.out);
  SR sv_own = SVg[i];
  double v2_own = need_v2 ? Vin2[i] : 0.0;
  put_v(2, v0);  // planes zb - 2 .. zb + 1
  put_v(3, v1);
  put_v(0, v2);
  put_v(1, v3);
  __syncthreads();
  // u_1 planes zb - 1 and zb; kept: V terms of planes zb and zb + 1 (C, D)
  PlaneTerms C, D;
  {
    const PlaneTerms A = vterms(2, 0), B = vterms(3, 0);
    C = vterms(0, 0);
    D = vterms(1, 0);
    put_u(0, A, B, C, svm[0]);
    if (xact) {
      const PlaneTerms xa = vterms(2, 1), xb = vterms(3, 1), xc = vterms(0, 1), xd = vterms(1, 1);
      put_u(1, xa, xb, xc, svm[1]);
      xput(0, xc);
      xput(1, xd);
    }
  }
  __syncthreads();
  PlaneTerms um = uterms();  // u_1 terms of plane z - 1
  __syncthreads();
  put_u(0, vterms(3, 0), C, D, sv0[0]);
  if (xact) put_u(1, vterms(3, 1), xget(0), xget(1), sv0[1]);
  __syncthreads();
  PlaneTerms uo = uterms();  // u_1 terms of plane z
  // plane z = zb + 4q + r; R is r as a constant
  auto body = [&](int z, auto R) {
    constexpr int r = decltype(R)::value;
    // V plane z + 2 into the slot of plane z - 2, whose last readers
    // finished before the barriers of the previous plane
    put_v((r + 2) & 3, vpre);
    __syncthreads();
    const SR svh0 = svpre[0], svh1 = svpre[1];
    const SR sv_cur = sv_own;
    const double v2_cur = v2_own;
    // the column needs V up to plane ze + 1 and S_V up to ze: the last
    // plane's loads repeat the previous plane's (served by L2) instead of
    // fetching planes nothing uses
    load_v(min(z + 3, ze + 1), vpre);
    load_svh(min(z + 2, ze), svpre);
    if (z + 1 < ze) {
      sv_own = SVg[i + plane];
      if (need_v2) v2_own = Vin2[i + plane];
    }
    // u_1 plane z + 1 (the ring's only plane: its readers finished before
    // this plane's first barrier)
    const PlaneTerms E = vterms((r + 2) & 3, 0);
    put_u(0, C, D, E, svh0);
    if (xact) {
      const PlaneTerms xe = vterms((r + 2) & 3, 1);
      put_u(1, xget(r & 3), xget((r + 1) & 3), xe, svh1);
      xput((r + 2) & 3, xe);
    }
    __syncthreads();
    const PlaneTerms up = uterms();
    if (own) {
      const double Fu = plane_combine(g.w, um, uo, up);
      const double u0 = vring[r & 3][cv];
      const double u2 = inner_combine(a.t, uo.c, u0, Fu, (double)sv_cur);
      if (a.last) {
        out[i] = tail_combine(a.t, u2, u0, v2_cur);
      } else {
        gptr(a.u1out)[i] = uo.c;
        out[i] = u2;
      }
    }
    C = D;
    D = E;
    um = uo;
    uo = up;
    i += plane;
  };
  for (int z = zb; z < ze; z += 4) {
    body(z, std::integral_constant<int, 0>());
    if (z + 1 < ze) body(z + 1, std::integral_constant<int, 1>());
    if (z + 2 < ze) body(z + 2, std::integral_constant<int, 2>());
    if (z + 3 < ze) body(z + 3, std::integral_constant<int, 3>());
  }
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// `lds` is an LDS byte address (an offset into the workgroup's LDS, which
// may be 0); it is converted to an LDS pointer directly, never through a
// generic pointer, whose null value would map to the LDS null (-1).
__device__ __forceinline__ void lds_dma_dword(const void *src, uint32_t lds) {
  __builtin_amdgcn_global_load_lds((glb_void_t *)src, (lds_void_t *)(uintptr_t)lds, 4, 0, 0);
}

// ---------------------------------------------------------------------------
// All inner stages of an outer stage in one launch on 2-D grids (the small,
// launch-bound unit-square case): a block owns a 16 x 16 (inner shape 2) or
// 8 x 8 (inner shape 3, four times the blocks) tile and holds u_1
// on the tile plus a halo of m - 1 nodes, and V_{j-1} and S_V on a halo of
// m - 2, in LDS; stage k forms u_k on a halo of m - k from u_{k-1} and
// u_{k-2}, and the last one the outer V update on the tile.  The halo work
// is repeated by neighbouring blocks instead of exchanged, so one launch and
// m - 1 block barriers replace m - 1 launches.  Positions beyond the grid
// are reflected at its edges (repeatedly for narrow grids); a value there
// equals the value at the reflected node, since the stencil's sums pair
// opposite neighbours.  V_j goes to another buffer than V_{j-1}, which
// neighbouring blocks still read.
// ---------------------------------------------------------------------------
constexpr int kAllR = 16 + 2 * (kInnerAllMaxM - 1);       // LDS frame edge (32) for tiles up to 16 x 16

__device__ __forceinline__ uint32_t reflect(int c, uint32_t n) {
  const int p = 2 * ((int)n - 1);  // period of the reflected sequence (n >= 2)
  int r = c % p;
  r = r < 0 ? r + p : r;
  return (uint32_t)(r > (int)n - 1 ? p - r : r);
}

// The inner stages k = 2..m of one tile: u_1 is read on a halo of
// m - 1 + e nodes, V_{j-1} and S_V on m - 2 + e, and the last stage gives
// V_j on a halo of e (0, or 1 when the next step's head follows in the same
// kernel): the tile's nodes to a.out and, when vn is given, every position
// of the halo to vn (frame layout).  U holds three frames.
template <bool MIXED, int kAllT>
__device__ __forceinline__ void inner_all_tile(const InnerAllArgs &a, const Grid &g, int x0, int y0, int e,
                                               double (*U)[kAllR * kAllR], double *sV, double *sS, double *vn) {
  const int m = a.m, rmax = m - 1 + e;
  const int F = kAllT + 2 * rmax;  // frame edge used; frame (0, 0) is node (x0 - rmax, y0 - rmax)
  // u_1 on the whole frame, V and S_V on the frame less one ring; all of a
  // thread's loads are issued before the first is stored (one latency)
  constexpr int kPass = (kAllR * kAllR + kBlock - 1) / kBlock;
  // S_V in its storage type until it is stored (a conversion at the load
  // would wait for it before the next loads)
  using SR = typename std::conditional<MIXED, float, double>::type;
  double lu[kPass], lv[kPass];
  SR ls[kPass];
#pragma unroll
  for (int k = 0; k < kPass; ++k) {
    const int p = threadIdx.x + k * kBlock;
    lu[k] = lv[k] = 0.0;
    ls[k] = SR(0);
    if (p < F * F) {
      const int fx = p % F, fy = p / F;
      const uint32_t i = reflect(x0 + fx - rmax, g.n0) + g.n0 * reflect(y0 + fy - rmax, g.n1);
      lu[k] = a.u1[i];
      if (fx >= 1 && fx < F - 1 && fy >= 1 && fy < F - 1) {
        lv[k] = a.V[i];
        ls[k] = gptr((const SR *)a.SV)[i];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kPass; ++k) {
    const int p = threadIdx.x + k * kBlock;
    if (p < F * F) {
      const int q = (p / F) * kAllR + p % F;
      U[1][q] = lu[k];
      sV[q] = lv[k];
      sS[q] = (double)ls[k];
    }
  }
  __syncthreads();
  // u_{k-2} is V for k = 2; buffers rotate: prev2, prev, next
  const double *prev2 = sV, *prev = U[1];
  int nexti = 2;
  for (int k = 2; k <= m; ++k) {
    const int r = m - k + e;       // halo of u_k
    const int lo = rmax - r, w = kAllT + 2 * r;
    TailArgs t = a.t;
    t.nu = a.nu[k];
    t.kappa = a.kappa[k];
    t.mu_eta = a.mu_eta[k];
    double *next = U[nexti];
    for (int p = threadIdx.x; p < w * w; p += kBlock) {
      const int fx = lo + p % w, fy = lo + p / w;
      const int q = fy * kAllR + fx;
      const double Fu = grid_stencil<2>(g.w, [&](int dx, int dy, int) { return prev[q + dy * kAllR + dx]; });
      const double uk = inner_combine(t, prev[q], prev2[q], Fu, sS[q]);
      if (k < m) {
        next[q] = uk;
      } else {
        // outer V update on the halo of e (reflected positions as elsewhere)
        const int gxs = x0 + fx - rmax, gys = y0 + fy - rmax;
        const uint32_t i = reflect(gxs, g.n0) + g.n0 * reflect(gys, g.n1);
        const double Vj = tail_combine(t, uk, sV[q], t.j1 ? 0.0 : a.Vin2[i]);
        if (vn != nullptr) vn[q] = Vj;
        const bool tile = fx >= rmax && fx < rmax + kAllT && fy >= rmax && fy < rmax + kAllT;
        if (tile && gxs < (int)g.n0 && gys < (int)g.n1) a.out[i] = Vj;
      }
    }
    __syncthreads();
    prev2 = prev;
    prev = next;
    nexti = (nexti + 1) % 3;
  }
}

template <bool MIXED, int kAllT>
__global__ __launch_bounds__(kBlock) void k_inner_all2d(InnerAllArgs a, Grid g, uint32_t ntx) {
  static_assert(kAllT <= 16, "the LDS frame holds tiles up to 16 x 16");
  __shared__ double U[3][kAllR * kAllR];
  __shared__ double sV[kAllR * kAllR];
  __shared__ double sS[kAllR * kAllR];
  if (a.tick != nullptr && blockIdx.x == 0 && threadIdx.x == 0) a.tick->step += a.tick_by;
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  inner_all_tile<MIXED, kAllT>(a, g, (int)((b % ntx) * kAllT), (int)((b / ntx) * kAllT), 0, U, sV, sS, nullptr);
}

// One kernel per step on small 2-D grids (s == 1): the inner stages of step
// n on the tile (V^{n+1} on a one-node halo, in LDS) and then the head of
// step n + 1 at the tile's nodes, whose f_F(V^{n+1}) is the stencil on that
// halo.  u_1, S_V and V alternate between two buffers from step to step
// (read with halos while the next ones are written); z is updated in place.
template <template <class> class Model, bool MIXED, int kAllT>
__global__ __launch_bounds__(kBlock) void k_step2d(InnerAllArgs a, HeadArgs h, Grid g, uint32_t ntx) {
  __shared__ double U[3][kAllR * kAllR];
  __shared__ double sV[kAllR * kAllR];
  __shared__ double sS[kAllR * kAllR];
  __shared__ double sVn[kAllR * kAllR];
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)((b % ntx) * kAllT), y0 = (int)((b / ntx) * kAllT);
  inner_all_tile<MIXED, kAllT>(a, g, x0, y0, 1, U, sV, sS, sVn);
  if (threadIdx.x >= kAllT * kAllT) return;
  const int lx = threadIdx.x % kAllT, ly = threadIdx.x / kAllT;
  const uint32_t gx = (uint32_t)(x0 + lx), gy = (uint32_t)(y0 + ly);
  if (gx >= g.n0 || gy >= g.n1) return;
  const int rmax = a.m;  // the halo of u_1 in this kernel
  const int q = (ly + rmax) * kAllR + (lx + rmax);
  head_node<Model, MIXED>(h, g.N, gx + g.n0 * gy, sVn[q], [&]() {
    return grid_stencil<2>(g.w, [&](int dx, int dy, int) { return sVn[q + dy * kAllR + dx]; });
  });
}

// Head on 3-D grids by z-marching columns: the MX x MY column layout and
// LDS ring of V_{j-1} of k_inner_march, with the ionic state z_{j-1} of the
// next plane loaded into registers while the current plane is computed, so
// that every wave keeps loads in flight during its ionic arithmetic.
template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_head_march(HeadArgs a, Grid g, uint32_t ncx, uint32_t ncy) {
  __shared__ double ring[3][MPL];
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bx = b % ncx, byz = b / ncx;
  const uint32_t by = byz % ncy, bz = byz / ncy;
  const int x0 = (int)(bx * MX), y0 = (int)(by * MY);
  const int zb = (int)(bz * g.zc);
  const int ze = min(zb + (int)g.zc, (int)g.n2);
  const uint32_t plane = g.n0 * g.n1;
  uint32_t off[MSLOT];
  bool act[MSLOT];
#pragma unroll
  for (int k = 0; k < MSLOT; ++k) {
    const int r = threadIdx.x + k * kBlock;
    act[k] = r < MPL;
    const int hx = r % MSX, hy = r / MSX;
    off[k] = act[k] ? mirror_any(x0 + hx - 1, g.n0) + g.n0 * mirror_any(y0 + hy - 1, g.n1) : 0u;
  }
  const double *__restrict__ u = a.Vin;
  auto gplane = [&](int z) { return (size_t)mirror_any(z, g.n2) * plane; };
  auto stage = [&](double *dst, int z) {
    const size_t pz = gplane(z);
#pragma unroll
    for (int k = 0; k < MSLOT; ++k)
      if (act[k]) dst[threadIdx.x + k * kBlock] = u[pz + off[k]];
  };
  stage(ring[(zb + 2) % 3], zb - 1);
  stage(ring[zb % 3], zb);
  double pre[MSLOT];
  {
    const size_t pz = gplane(zb + 1);
#pragma unroll
    for (int k = 0; k < MSLOT; ++k) pre[k] = act[k] ? u[pz + off[k]] : 0.0;
  }
  const int lx = threadIdx.x % MX, ly = threadIdx.x / MX;
  const uint32_t gx = (uint32_t)(x0 + lx), gy = (uint32_t)(y0 + ly);
  const bool own = gx < g.n0 && gy < g.n1;
  const int c = (ly + 1) * MSX + (lx + 1);
  uint32_t i = gx + g.n0 * gy + plane * (uint32_t)zb;
  HeadZ<Model, MIXED> nz;
  if (own) nz.load(a.zin, g.N, i);
  const double tj = stage_time(a.clock, a.step_off, a.dt, a.c_prev);
  for (int z = zb; z < ze; ++z, i += plane) {
    double *nxt = ring[(z + 1) % 3];
#pragma unroll
    for (int k = 0; k < MSLOT; ++k)
      if (act[k]) nxt[threadIdx.x + k * kBlock] = pre[k];
    __syncthreads();
    const HeadZ<Model, MIXED> cz = nz;
    if (z + 1 < ze) {
      const size_t pz = gplane(z + 2);
#pragma unroll
      for (int k = 0; k < MSLOT; ++k) pre[k] = act[k] ? u[pz + off[k]] : 0.0;
      if (own) nz.load(a.zin, g.N, i + plane);
    }
    if (own) {
      const double *pm = ring[(z + 2) % 3], *pc = ring[z % 3], *pp = ring[(z + 1) % 3];
      head_node_z<Model, MIXED>(a, g.N, i, pc[c], cz.z, stimulus(a.stim, i, tj), [&]() {
        return grid_stencil<3>(g.w, [&](int dx, int dy, int dz) {
          const double *pl = dz < 0 ? pm : (dz > 0 ? pp : pc);
          return pl[c + dy * MSX + dx];
        });
      });
    }
    __syncthreads();
  }
}

// Head by z-marching columns with the ionic state staged through LDS: each
// wave copies z_{j-1} of its own 64 nodes of the next plane into its LDS
// slice with direct global-to-LDS loads (no registers held while in
// flight), and reads the current plane's slice into registers first.  Only
// the wave that loads a slice reads it, so the slices need no barrier; the
// V ring is shared as in k_inner_march.
// Waits (and orders the compiler's memory accesses) for this wave's
// outstanding vector-memory loads, including the LDS copies, or for its LDS
// reads.
__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_lgkm() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <template <class> class Model, bool MIXED>
struct ZSlice {
  using R = typename MathOf<MIXED>::R;
  static constexpr int NZ = HeadZ<Model, MIXED>::NZ;
  static constexpr int DW = sizeof(R) / 4;          // dwords per value
  static constexpr int SLICE = NZ * 64 * (int)sizeof(R);
  static constexpr int BYTES = (kBlock / 64) * SLICE;
  // Copies component k of the lane's nodes (byte offsets voff[h] within a
  // component plane) to bytes [k * 64 * sizeof(R), ...) of the wave's slice
  // at LDS address `slice`.  `zb` is the state base, made opaque per call so
  // that the per-component addresses are formed here and not kept live.
  static __device__ __forceinline__ void copy(uint32_t slice, const char *zb, uint64_t plane_bytes,
                                              const uint32_t voff[DW]) {
    asm volatile("" : "+s"(zb));
    asm volatile("" : "+s"(slice));
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
#pragma unroll
      for (int h = 0; h < DW; ++h)
        lds_dma_dword(zb + voff[h], slice + (uint32_t)((k * 64 + h * 32) * sizeof(R)));
      zb += plane_bytes;
    }
  }
  static __device__ __forceinline__ void read(const char *lds, R *z) {
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const R *src = (const R *)(lds + (size_t)w * SLICE);
#pragma unroll
    for (int k = 0; k < NZ; ++k) z[k] = src[k * 64 + lane];
  }
};

template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_head_march_lds(HeadArgs a, Grid g, uint32_t ncx, uint32_t ncy) {
  using ZS = ZSlice<Model, MIXED>;
  using R = typename ZS::R;
  __shared__ double ring[3][MPL];
  __shared__ __attribute__((aligned(16))) char zlds[ZS::BYTES];
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bx = b % ncx, byz = b / ncx;
  const uint32_t by = byz % ncy, bz = byz / ncy;
  const int x0 = (int)(bx * MX), y0 = (int)(by * MY);
  const int zb = (int)(bz * g.zc);
  const int ze = min(zb + (int)g.zc, (int)g.n2);
  const uint32_t plane = g.n0 * g.n1;
  uint32_t off[MSLOT];
  bool act[MSLOT];
#pragma unroll
  for (int k = 0; k < MSLOT; ++k) {
    const int r = threadIdx.x + k * kBlock;
    act[k] = r < MPL;
    const int hx = r % MSX, hy = r / MSX;
    off[k] = act[k] ? mirror_any(x0 + hx - 1, g.n0) + g.n0 * mirror_any(y0 + hy - 1, g.n1) : 0u;
  }
  const double *__restrict__ u = a.Vin;
  auto gplane = [&](int z) { return (size_t)mirror_any(z, g.n2) * plane; };
  auto stage = [&](double *dst, int z) {
    const size_t pz = gplane(z);
#pragma unroll
    for (int k = 0; k < MSLOT; ++k)
      if (act[k]) dst[threadIdx.x + k * kBlock] = u[pz + off[k]];
  };
  // byte offsets (within a component plane, at plane z = 0) of the dwords
  // this lane copies: nodes of this wave, those outside the grid clamped
  // onto it (their values are never used)
  const uint32_t lane = threadIdx.x & 63, wbase = threadIdx.x & ~63u;
  uint32_t voff0[ZS::DW];
#pragma unroll
  for (int h = 0; h < ZS::DW; ++h) {
    const uint32_t t = wbase + (ZS::DW == 2 ? h * 32 + (lane >> 1) : lane);
    const uint32_t cx = min((uint32_t)x0 + t % MX, g.n0 - 1), cy = min((uint32_t)y0 + t / MX, g.n1 - 1);
    voff0[h] = (cx + g.n0 * cy) * (uint32_t)sizeof(R) + (ZS::DW == 2 ? (lane & 1) * 4u : 0u);
  }
  const uint32_t slice = (uint32_t)(uintptr_t)(lds_void_t *)(zlds) +
                         (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * (uint32_t)ZS::SLICE;
  const uint64_t comp_bytes = (uint64_t)g.N * sizeof(R);
  auto copy_plane = [&](int z) {
    uint32_t voff[ZS::DW];
#pragma unroll
    for (int h = 0; h < ZS::DW; ++h) voff[h] = voff0[h] + (uint32_t)z * plane * (uint32_t)sizeof(R);
    ZS::copy(slice, (const char *)a.zin, comp_bytes, voff);
  };
  const int lx = threadIdx.x % MX, ly = threadIdx.x / MX;
  const uint32_t gx = (uint32_t)(x0 + lx), gy = (uint32_t)(y0 + ly);
  const bool own = gx < g.n0 && gy < g.n1;
  const int c = (ly + 1) * MSX + (lx + 1);
  uint32_t i = gx + g.n0 * gy + plane * (uint32_t)zb;
  // the stage time is uniform; the stimulus mask of the next plane is
  // loaded with its state copy, so no load is waited for during the ionic
  // arithmetic
  const double tj = stage_time(a.clock, a.step_off, a.dt, a.c_prev);
  const bool stim_on = a.stim.mask != nullptr && a.stim.t_on <= tj && tj <= a.stim.t_off;
  uint8_t mnext = (stim_on && own) ? a.stim.mask[i] : (uint8_t)0;
  stage(ring[(zb + 2) % 3], zb - 1);
  stage(ring[zb % 3], zb);
  double pre[MSLOT];
  {
    const size_t pz = gplane(zb + 1);
#pragma unroll
    for (int k = 0; k < MSLOT; ++k) pre[k] = act[k] ? u[pz + off[k]] : 0.0;
  }
  copy_plane(zb);
  for (int z = zb; z < ze; ++z, i += plane) {
    double *nxt = ring[(z + 1) % 3];
#pragma unroll
    for (int k = 0; k < MSLOT; ++k)
      if (act[k]) nxt[threadIdx.x + k * kBlock] = pre[k];
    const uint8_t mcur = mnext;
    wait_vm();  // this wave's slice of plane z, the mask byte
    __syncthreads();
    R zc[ZS::NZ];
    ZS::read(zlds, zc);
    wait_lgkm();  // slice read before it is overwritten
    if (z + 1 < ze) {
      mnext = (stim_on && own) ? a.stim.mask[i + plane] : (uint8_t)0;
      const size_t pz = gplane(z + 2);
#pragma unroll
      for (int k = 0; k < MSLOT; ++k) pre[k] = act[k] ? u[pz + off[k]] : 0.0;
      copy_plane(z + 1);
    }
    if (own) {
      const double *pm = ring[(z + 2) % 3], *pc = ring[z % 3], *pp = ring[(z + 1) % 3];
      head_node_z<Model, MIXED>(a, g.N, i, pc[c], zc, mcur != 0 ? a.stim.amp : 0.0, [&]() {
        return grid_stencil<3>(g.w, [&](int dx, int dy, int dz) {
          const double *pl = dz < 0 ? pm : (dz > 0 ? pp : pc);
          return pl[c + dy * MSX + dx];
        });
      });
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Batched ensembles: one launch covers the tiles of every participating
// instance; each block finds its instance through a block map and runs the
// LDS-tiled head or inner stage with that instance's grid and coefficients.
// ---------------------------------------------------------------------------
template <int DIM, int SH>
__device__ __forceinline__ void tile_xyz(const BatchInst &I, uint32_t tile, int &x0, int &y0, int &z0) {
  using T = Tile<DIM, SH>;
  const uint32_t bx = tile % I.ntx, byz = tile / I.ntx;
  const uint32_t by = byz % I.nty, bz = byz / I.nty;
  x0 = (int)(bx * T::TX);
  y0 = (int)(by * T::TY);
  z0 = (int)(bz * T::TZ);
}

// Table slot of logical block lb: the u16 map is read as 32-bit words, a
// scalar load (its allocation holds an even number of entries), and the
// instance record is then copied by value, so that its fields are loaded
// together rather than one dependent load at a time where they are used.
__device__ __forceinline__ uint32_t batch_slot(const uint16_t *__restrict__ map, uint32_t lb) {
  const uint32_t w = ((const uint32_t *)map)[lb >> 1];
  return (lb & 1u) ? (w >> 16) : (w & 0xffffu);
}

template <template <class> class Model, bool MIXED, int DIM, int SH>
__device__ __forceinline__ void head_tile(const BatchInst &I, const HeadArgs &h, uint32_t tile, double *sV,
                                          uint32_t Ntot) {
  int x0, y0, z0;
  tile_xyz<DIM, SH>(I, tile, x0, y0, z0);
  head_tiled_node<Model, MIXED, DIM, SH>(h, I.g, Ntot, I.off, h.Vin + I.off, x0, y0, z0, sV);
}

template <int SH>
struct BatchLds {
  static constexpr int NS = Tile<3, SH>::NS > Tile<2, SH>::NS ? Tile<3, SH>::NS : Tile<2, SH>::NS;
};

template <template <class> class Model, bool MIXED, int SH>
__global__ __launch_bounds__(kBlock) void k_head_batch(const BatchInst *__restrict__ tab,
                                                       const uint16_t *__restrict__ map, uint32_t Ntot, int step_off) {
  __shared__ double sV[BatchLds<SH>::NS];
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  BatchInst I = tab[batch_slot(map, lb)];
  HeadArgs h = I.h;
  h.step_off = step_off;
  if (I.g.dim == 3)
    head_tile<Model, MIXED, 3, SH>(I, h, lb - I.tile0, sV, Ntot);
  else
    head_tile<Model, MIXED, 2, SH>(I, h, lb - I.tile0, sV, Ntot);
}

// Flat batched head: block b covers nodes 256 (b - tile0) .. of its
// instance, one node per thread, stencil operands through the caches (no LDS
// staging, no barrier).
template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_head_batch_flat(const BatchInst *__restrict__ tab,
                                                            const uint16_t *__restrict__ map, uint32_t Ntot,
                                                            int step_off) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  BatchInst I = tab[batch_slot(map, lb)];
  const uint32_t il = (lb - I.tile0) * kBlock + threadIdx.x;
  if (il >= I.g.N) return;
  HeadArgs h = I.h;
  h.step_off = step_off;
  const auto Vg = gptr(h.Vin + I.off);
  head_node<Model, MIXED>(h, Ntot, I.off + il, Vg[il], [&]() {
    uint32_t ix, iy, iz;
    grid_coords(I.g, il, ix, iy, iz);
    return I.g.dim == 3 ? grid_apply<3>(Vg, I.g, ix, iy, iz) : grid_apply<2>(Vg, I.g, ix, iy, iz);
  });
}

template <bool MIXED, int DIM, int SH>
__device__ __forceinline__ void inner_tile(const BatchInst &I, uint32_t tile, double *sU) {
  int x0, y0, z0;
  tile_xyz<DIM, SH>(I, tile, x0, y0, z0);
  const InnerArgs &a = I.in;
  uint32_t il;
  int c;
  const bool own = tile_node<DIM, SH>(I.g, x0, y0, z0, il, c);
  const uint32_t i = I.off + il;
  InnerPoint<MIXED> pt{};
  if (own) pt = load_point<MIXED>(a, i);
  stage_halo<DIM, SH>(sU, a.t.uprev + I.off, I.g, x0, y0, z0);
  __syncthreads();
  if (!own) return;
  const double Fu = lds_stencil<DIM, SH>(sU, I.g, c);
  gptr(a.out)[i] = inner_point(a, sU[c], Fu, pt);
}

// Two tiles of an instance per block (tiles 2 pair and 2 pair + 1): the
// operands and halos of both are loaded before one barrier, so each wave
// keeps twice the loads in flight and the instance lookup serves two tiles.
template <bool MIXED, int DIM, int SH>
__device__ __forceinline__ void inner_tile_pair(const BatchInst &I, uint32_t pair, double *sU) {
  using T = Tile<DIM, SH>;
  const uint32_t ntz = DIM == 3 ? (I.g.n2 + T::TZ - 1) / T::TZ : 1u;
  const uint32_t ta = 2 * pair;
  const bool hasb = ta + 1 < I.ntx * I.nty * ntz;
  int xa, ya, za, xb, yb, zb;
  tile_xyz<DIM, SH>(I, ta, xa, ya, za);
  tile_xyz<DIM, SH>(I, hasb ? ta + 1 : ta, xb, yb, zb);
  const InnerArgs &a = I.in;
  uint32_t ila = 0, ilb = 0;
  int ca = 0, cb = 0;
  const bool owna = tile_node<DIM, SH>(I.g, xa, ya, za, ila, ca);
  const bool ownb = tile_node<DIM, SH>(I.g, xb, yb, zb, ilb, cb) && hasb;
  InnerPoint<MIXED> pa{}, pb{};
  if (owna) pa = load_point<MIXED>(a, I.off + ila);
  if (ownb) pb = load_point<MIXED>(a, I.off + ilb);
  Halo<DIM, SH> ha, hb;
  ha.load(a.t.uprev + I.off, I.g, xa, ya, za);
  if (hasb) hb.load(a.t.uprev + I.off, I.g, xb, yb, zb);
  ha.store(sU);
  if (hasb) hb.store(sU + T::NS);
  __syncthreads();
  const auto out = gptr(a.out + I.off);
  if (owna) out[ila] = inner_point(a, sU[ca], lds_stencil<DIM, SH>(sU, I.g, ca), pa);
  if (ownb) out[ilb] = inner_point(a, sU[T::NS + cb], lds_stencil<DIM, SH>(sU + T::NS, I.g, cb), pb);
}

// Inner stage of the batch, by the mode the tables were built for: LDS
// tiles, one per block (MODE 0) or two (MODE 2), or (MODE 1) z-marching
// columns of g.zc planes for the 3-D instances, whose table entries have
// inner_variant 1, and tiles for the others.  Each mode is its own kernel:
// the registers of one form would lower the occupancy of another.
template <bool MIXED, int SH, int MODE>
__global__ __launch_bounds__(kBlock) void k_inner_batch(const BatchInst *__restrict__ tab,
                                                        const uint16_t *__restrict__ map) {
  constexpr int NT = (MODE == 2 ? 2 : 1) * BatchLds<SH>::NS;
  constexpr int NL = MODE == 1 && NT < 3 * MPL ? 3 * MPL : NT;
  __shared__ double lds[NL];
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  BatchInst I = tab[batch_slot(map, lb)];
  if (MODE == 2) {
    if (I.g.dim == 3)
      inner_tile_pair<MIXED, 3, SH>(I, lb - I.tile0, lds);
    else
      inner_tile_pair<MIXED, 2, SH>(I, lb - I.tile0, lds);
  } else if (MODE == 1 && I.g.dim == 3 && I.g.inner_variant == 1) {
    inner_march_col<MIXED>(I.in, I.g, I.off, lb - I.tile0, I.ntx, I.nty, (double (*)[MPL])lds);
  } else if (I.g.dim == 3) {
    inner_tile<MIXED, 3, SH>(I, lb - I.tile0, lds);
  } else {
    inner_tile<MIXED, 2, SH>(I, lb - I.tile0, lds);
  }
}

// z between component planes and blocks of kZBlock nodes: element j of the
// block layout is component k of node i = b kZBlock + l with
// j = b kZBlock nz + k kZBlock + l.  Positions of the last block beyond N
// are written as zero and never copied back.  Consecutive threads take
// consecutive j, so both sides are read and written in runs of kZBlock.
template <class R, bool TO_BLOCKS>
__global__ __launch_bounds__(kBlock) void k_z_layout(const R *__restrict__ src, R *__restrict__ dst, uint32_t N,
                                                     uint32_t nz, size_t total) {
  const size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= total) return;
  const size_t per = (size_t)kZBlock * nz;
  const size_t b = j / per, r = j - b * per;
  const size_t k = r / kZBlock, i = b * kZBlock + r % kZBlock;
  if (TO_BLOCKS)
    dst[j] = i < N ? src[k * N + i] : R(0);
  else if (i < N)
    dst[k * N + i] = src[j];
}

__global__ void k_clock_set(Clock *c, int64_t step, double t0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->step = step;
    c->t0 = t0;
  }
}

__global__ __launch_bounds__(kBlock) void k_copy_tick(const double *src, double *dst, uint32_t N, Clock *tick,
                                                      int64_t tick_by) {
  const uint32_t i = node_index();
  if (tick != nullptr && blockIdx.x == 0 && threadIdx.x == 0) tick->step += tick_by;
  if (src != nullptr && i < N) dst[i] = src[i];
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_apply_diffusion(Mesh mesh, const double *V, double *out) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t i = node_index();
  if (i >= N) return;
  out[i] = apply_op<MIXED>(mesh, V, i);
}

// f_S(t, y) in double for the full state (component checks).
template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_eval_rhs_slow(uint32_t N, const double *V, const void *zv, double t,
                                                          StimArgs stim, double Cm, ModelParams mp, double *out) {
  using M = MathF64;
  using Mod = Model<M>;
  constexpr int NG = Mod::NG, NS = Mod::NS, NZ = NG + NS;
  const uint32_t i = node_index();
  if (i >= N) return;
  using Rs = typename std::conditional<MIXED, float, double>::type;
  const Rs *z = (const Rs *)zv;
  double zz[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) zz[k] = (double)z[(size_t)k * N + i];
  double dS[NS > 0 ? NS : 1];
  const double v = V[i];
  const double iion = Mod::eval(v, zz, zz + NG, dS, mp);
  out[i] = (stimulus(stim, i, t) - Cm * iion) / Cm;
#pragma unroll
  for (int g = 0; g < NG; ++g) out[(size_t)(1 + g) * N + i] = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) out[(size_t)(1 + NG + s) * N + i] = dS[s];
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
  }
  return s;  // valid in thread 0
}

// Each block sums a contiguous chunk of `per_block` items in a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce_final(const double *partials, uint32_t n, double *result) {
  double v = 0.0;
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) v += partials[k];
  v = block_sum(v);
  if (threadIdx.x == 0) *result = v;
}

// ||y||^2 over every component; z planes are `stride` apart.
template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_norm2_state(uint32_t N, int nz, const double *V, const void *zv,
                                                        size_t stride, double *partials) {
  using Rs = typename std::conditional<MIXED, float, double>::type;
  const Rs *z = (const Rs *)zv;
  double v = 0.0;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) {
    v = V[i] * V[i];
    for (int c = 0; c < nz; ++c) {
      const double x = (double)z[(size_t)c * stride + i];
      v += x * x;
    }
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void k_norm2_random(uint64_t seed, uint64_t total, double *partials) {
  double v = 0.0;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (uint64_t)gridDim.x * blockDim.x) {
    const double x = splitmix64_unit(seed, k);
    v += x * x;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void k_vec_diff_norm(uint64_t n, const double *a, const double *b, double *out,
                                                          double *partials) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double d = b != nullptr ? a[i] - b[i] : a[i];
    if (out != nullptr) out[i] = d;
    v = d * d;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// ---------------------------------------------------------------------------
// Conjugate gradients for (I - dt F) x = b, F = (chi Cm M_L)^{-1} A, in the
// inner product sum_i ML_i u_i v_i (in which I - dt F is symmetric positive
// definite), preconditioned by its diagonal 1 + dt D_i, D_i = sum of the
// node's neighbour weights (Dsum[i], or dconst on a uniform grid).  Always
// double precision.  The scalars live on the device (CgScalars): each
// vector kernel leaves per-block partial sums, a one-block kernel reduces
// them in a fixed order and updates the scalars, and once the solve has
// converged every later kernel of the solve returns at once, so the host
// can enqueue iterations ahead and look at the flag once per batch.
// ---------------------------------------------------------------------------
struct CgDiag {
  const double *Dsum;  // nullptr: every node has dconst
  double dconst;
  double dt;
  __device__ __forceinline__ double at(uint32_t i) const { return 1.0 + dt * (Dsum ? Dsum[i] : dconst); }
};

__device__ __forceinline__ double block_total(const double *partials, uint32_t n) {
  double v = 0.0;
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) v += partials[k];
  return block_sum(v);  // valid in thread 0
}

__global__ __launch_bounds__(kBlock) void k_cg_init(Mesh mesh, const double *ML, CgDiag dg, const double *x,
                                                    const double *b, double *r, double *z, double *partials) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, bb = 0.0;
  if (i < N) {
    const double Bx = x[i] - dg.dt * apply_op<false>(mesh, x, i);
    const double ri = b[i] - Bx;
    const double di = dg.at(i);
    const double zi = ri / di;
    r[i] = ri;
    z[i] = zi;
    rz = ML[i] * ri * zi;
    bb = ML[i] * b[i] * (b[i] / di);
  }
  rz = block_sum(rz);
  __syncthreads();  // block_sum's LDS slots are reused by the second sum
  bb = block_sum(bb);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = rz;
    partials[gridDim.x + blockIdx.x] = bb;
  }
}

__global__ __launch_bounds__(kBlock) void k_cg_init_final(const double *partials, uint32_t nb, double tol2,
                                                          CgScalars *s) {
  const double rz = block_total(partials, nb);
  __syncthreads();
  const double bb = block_total(partials + nb, nb);
  if (threadIdx.x == 0) {
    s->rz = rz;
    s->rz_prev = rz;
    s->pq = 0.0;
    s->stop = tol2 * bb;
    s->iters = 0;
    s->first = 1;
    s->done = rz <= s->stop ? 1 : (isfinite(rz) ? 0 : 2);
  }
}

// One iteration's first half: the new direction p = z + beta p_prev (p = z
// on the first iteration, where p_prev is not read), q = p - dt F p, and
// alpha = (r, z) / (p, q) in the lumped-mass inner product.
struct CgDirArgs {
  const double *ML, *z, *pprev;
  double *p, *q, *partials;
  CgScalars *s;
  double dt;
};

__device__ __forceinline__ double cg_beta(const CgScalars *s) { return s->first ? 0.0 : s->rz / s->rz_prev; }

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_cg_dir_apply_tiled(CgDirArgs a, Grid g, uint32_t ntx, uint32_t nty) {
  using T = Tile<DIM>;
  if (a.s->done) return;
  __shared__ double sP[T::NS];
  const bool first = a.s->first != 0;
  const double beta = cg_beta(a.s);
  int x0, y0, z0;
  tile_origin<DIM>(ntx, nty, x0, y0, z0);
  for (int r = threadIdx.x; r < T::NS; r += kBlock) {
    const int hx = r % T::SX, hy = (r / T::SX) % T::SY, hz = r / (T::SX * T::SY);
    const uint32_t gx = mirror_any(x0 + hx - 1, g.n0);
    const uint32_t gy = mirror_any(y0 + hy - 1, g.n1);
    const uint32_t gz = DIM == 3 ? mirror_any(z0 + hz - 1, g.n2) : 0u;
    const uint32_t j = gx + g.n0 * (gy + g.n1 * gz);
    sP[r] = first ? a.z[j] : a.z[j] + beta * a.pprev[j];
  }
  __syncthreads();
  uint32_t i;
  int c;
  double pq = 0.0;
  if (tile_node<DIM>(g, x0, y0, z0, i, c)) {
    const double pi = sP[c];
    const double qi = pi - a.dt * lds_stencil<DIM>(sP, g, c);
    a.p[i] = pi;
    a.q[i] = qi;
    pq = a.ML[i] * pi * qi;
  }
  pq = block_sum(pq);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = pq;
}

__global__ __launch_bounds__(kBlock) void k_cg_dir_apply_ell(CgDirArgs a, Ell e) {
  if (a.s->done) return;
  const bool first = a.s->first != 0;
  const double beta = cg_beta(a.s);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  double pq = 0.0;
  if (i < e.N) {
    auto pn = [&](uint32_t j) { return first ? a.z[j] : a.z[j] + beta * a.pprev[j]; };
    const double pi = pn(i);
    double acc = 0.0;
    for (uint32_t k = 0; k < e.width; ++k) {
      const uint32_t c = e.col[(size_t)k * e.N + i];
      acc = __builtin_fma(e.w64[(size_t)k * e.N + i], pn(c) - pi, acc);
    }
    const double qi = pi - a.dt * acc;
    a.p[i] = pi;
    a.q[i] = qi;
    pq = a.ML[i] * pi * qi;
  }
  pq = block_sum(pq);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = pq;
}

// Second half: x += alpha p, r -= alpha q, z = r/diag, rz' = (r, z); the
// last block rolls the scalars and sets the convergence flag.
__global__ __launch_bounds__(kBlock) void k_cg_update(uint32_t N, const double *ML, CgDiag dg, double *x, double *r,
                                                      double *z, const double *p, const double *q,
                                                      double *partials, CgScalars *s) {
  if (s->done) return;
  const double alpha = s->rz / s->pq;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0;
  if (i < N) {
    x[i] = x[i] + alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    const double zi = ri / dg.at(i);
    r[i] = ri;
    z[i] = zi;
    rz = ML[i] * ri * zi;
  }
  rz = block_sum(rz);
  if (threadIdx.x == 0) partials[blockIdx.x] = rz;
}

// One-block reductions of the partial sums, in index order: pq, then rz'
// with the scalars rolled and the convergence flag set.
__global__ __launch_bounds__(kBlock) void k_cg_pq_final(const double *partials, uint32_t nb, CgScalars *s) {
  if (s->done) return;
  const double t = block_total(partials, nb);
  if (threadIdx.x == 0) s->pq = t;
}

__global__ __launch_bounds__(kBlock) void k_cg_rz_final(const double *partials, uint32_t nb, CgScalars *s) {
  if (s->done) return;
  const double t = block_total(partials, nb);
  if (threadIdx.x == 0) {
    s->rz_prev = s->rz;
    s->rz = t;
    s->first = 0;
    s->iters = s->iters + 1;
    s->done = t <= s->stop ? 1 : (isfinite(t) ? 0 : 2);
  }
}

// Row sums of the ELL weights (the D_i of the preconditioner).
__global__ __launch_bounds__(kBlock) void k_ell_rowsum(Ell e, double *out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= e.N) return;
  double s = 0.0;
  for (uint32_t k = 0; k < e.width; ++k) s += e.w64[(size_t)k * e.N + i];
  out[i] = s;
}

__global__ __launch_bounds__(kBlock) void k_powF_shift(uint32_t N, const double *yV, const double *vin,
                                                       uint64_t seed, double q, double *zV) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double v = vin != nullptr ? vin[i] : splitmix64_unit(seed, i);
  zV[i] = yV[i] + q * v;
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_powF_diff(Mesh mesh, const double *zV, const double *yV, double *vout,
                                                      double *partials) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < N) {
    // the power iteration always differences in double
    const double d = apply_op<false>(mesh, zV, i) - apply_op<false>(mesh, yV, i);
    vout[i] = d;
    v = d * d;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// z and the vectors v have component planes `stride` apart; the random start
// vector is indexed as in a state of N nodes (component c at c*N + i).
template <template <class> class Model, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_powS_iter(uint32_t N, size_t stride, const double *V, const void *zv,
                                                      const double *vin, uint64_t seed, double q, double t,
                                                      StimArgs stim, double Cm, ModelParams mp, double *vout,
                                                      double *partials) {
  using M = MathF64;
  using Mod = Model<M>;
  constexpr int NG = Mod::NG, NS = Mod::NS, NZ = NG + NS;
  using Rs = typename std::conditional<MIXED, float, double>::type;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < N) {
    const Rs *z = (const Rs *)zv;
    double y[NZ], w[NZ];
    const double yv = V[i];
#pragma unroll
    for (int k = 0; k < NZ; ++k) y[k] = (double)z[(size_t)k * stride + i];
    // perturbed state z = y + q v; gate components of a warm vector are 0
    double wv;
    if (vin == nullptr) {
      wv = yv + q * splitmix64_unit(seed, i);
#pragma unroll
      for (int k = 0; k < NZ; ++k) w[k] = y[k] + q * splitmix64_unit(seed, (uint64_t)(1 + k) * N + i);
    } else {
      wv = yv + q * vin[i];
#pragma unroll
      for (int k = 0; k < NZ; ++k)
        w[k] = k < NG ? y[k] + q * 0.0 : y[k] + q * vin[(size_t)(1 + k - NG) * stride + i];
    }
    const double Is = stimulus(stim, i, t);
    double dSy[NS > 0 ? NS : 1], dSw[NS > 0 ? NS : 1];
    const double fy = (Is - Cm * Mod::eval(yv, y, y + NG, dSy, mp)) / Cm;
    const double fw = (Is - Cm * Mod::eval(wv, w, w + NG, dSw, mp)) / Cm;
    const double dv = fw - fy;
    vout[i] = dv;
    acc = dv * dv;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double d = dSw[s] - dSy[s];
      vout[(size_t)(1 + s) * stride + i] = d;
      acc += d * d;
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void k_finite_check(uint32_t N, const double *V, int *flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N && !isfinite(V[i])) *flag = 1;  // benign race: every writer stores 1
}

template <class M>
__global__ __launch_bounds__(kBlock) void k_elementary(int fn, const double *x, double *y, uint32_t n) {
  using R = typename M::R;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const R v = R(x[i]);
  y[i] = double(fn == 0 ? M::exp(v) : (fn == 1 ? M::expm1(v) : M::log(v)));
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

uint32_t reduce_blocks(uint32_t n) { return blocks_for(n); }

template <int DIM, int SH = 0>
static dim3 tile_grid(const Grid &g, uint32_t &ntx, uint32_t &nty) {
  using T = Tile<DIM, SH>;
  ntx = (g.n0 + T::TX - 1) / T::TX;
  nty = (g.n1 + T::TY - 1) / T::TY;
  const uint32_t ntz = DIM == 3 ? (g.n2 + T::TZ - 1) / T::TZ : 1;
  return dim3(ntx * nty * ntz);
}


template <template <class> class Model>
static hipError_t head_dispatch(bool mixed, const Mesh &mesh, const HeadArgs &a, hipStream_t st) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  // head shapes 5 and 6 on grids: the flat kernels below (one node per
  // thread in index order, stencil operands through the caches; no LDS
  // staging, no block barrier, no tile padding)
  const bool flat = mesh.kind != kGrid || mesh.flat || mesh.grid.head_variant >= 5;
  if (!flat) {
    uint32_t ntx, nty;
    const Grid &g = mesh.grid;
    if (g.dim == 3 && (g.head_variant == 1 || g.head_variant == 2)) {
      Grid gm = g;
      gm.zc = g.head_zc;
      const uint32_t ncx = (g.n0 + MX - 1) / MX, ncy = (g.n1 + MY - 1) / MY, ncz = (g.n2 + gm.zc - 1) / gm.zc;
      const dim3 grid(ncx * ncy * ncz);
      if (g.head_variant == 1) {
        if (mixed)
          EMRKC_LAUNCH((k_head_march<Model, true>), grid, dim3(kBlock), 0, st, a, gm, ncx, ncy);
        else
          EMRKC_LAUNCH((k_head_march<Model, false>), grid, dim3(kBlock), 0, st, a, gm, ncx, ncy);
      } else {
        if (mixed)
          EMRKC_LAUNCH((k_head_march_lds<Model, true>), grid, dim3(kBlock), 0, st, a, gm, ncx, ncy);
        else
          EMRKC_LAUNCH((k_head_march_lds<Model, false>), grid, dim3(kBlock), 0, st, a, gm, ncx, ncy);
      }
    } else if (g.dim == 3 && (g.head_variant == 3 || g.head_variant == 4)) {
      const dim3 grid = tile_grid<3>(g, ntx, nty);
      if (g.head_variant == 3) {
        if (mixed)
          EMRKC_LAUNCH((k_head_tiled_occ<Model, true, 3, 6>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
        else
          EMRKC_LAUNCH((k_head_tiled_occ<Model, false, 3, 6>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
      } else {
        if (mixed)
          EMRKC_LAUNCH((k_head_tiled_occ<Model, true, 3, 8>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
        else
          EMRKC_LAUNCH((k_head_tiled_occ<Model, false, 3, 8>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
      }
    } else if (g.dim == 3) {
      const dim3 grid = tile_grid<3>(g, ntx, nty);
      if (mixed)
        EMRKC_LAUNCH((k_head_tiled<Model, true, 3>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
      else
        EMRKC_LAUNCH((k_head_tiled<Model, false, 3>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
    } else {
      const dim3 grid = tile_grid<2>(g, ntx, nty);
      if (mixed)
        EMRKC_LAUNCH((k_head_tiled<Model, true, 2>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
      else
        EMRKC_LAUNCH((k_head_tiled<Model, false, 2>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
    }
    return hipGetLastError();
  }
  // shape 6 exists for mixed contexts only (the host rejects it for FP64)
  if (mixed && mesh.kind == kGrid && !mesh.flat && mesh.grid.head_variant == 6) {
    EMRKC_LAUNCH((k_head_occ<Model>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  } else if (mixed) {
    EMRKC_LAUNCH((k_head<Model, true>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  } else {
    EMRKC_LAUNCH((k_head<Model, false>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  }
  return hipGetLastError();
}

template <template <class> class Model>
static hipError_t init_dispatch(bool mixed, uint32_t N, double *V, void *z, ModelParams mp, hipStream_t st) {
  if (mixed)
    EMRKC_LAUNCH((k_init_state<Model, true>), dim3(blocks_for(N)), dim3(kBlock), 0, st, N, V, z, mp);
  else
    EMRKC_LAUNCH((k_init_state<Model, false>), dim3(blocks_for(N)), dim3(kBlock), 0, st, N, V, z, mp);
  return hipGetLastError();
}

template <template <class> class Model>
static hipError_t rhs_dispatch(bool mixed, uint32_t N, const double *V, const void *z, double t, StimArgs stim,
                               double Cm, ModelParams mp, double *out, hipStream_t st) {
  if (mixed)
    EMRKC_LAUNCH((k_eval_rhs_slow<Model, true>), dim3(blocks_for(N)), dim3(kBlock), 0, st, N, V, z, t,
                       stim, Cm, mp, out);
  else
    EMRKC_LAUNCH((k_eval_rhs_slow<Model, false>), dim3(blocks_for(N)), dim3(kBlock), 0, st, N, V, z, t,
                       stim, Cm, mp, out);
  return hipGetLastError();
}

template <template <class> class Model>
static hipError_t powS_dispatch(bool mixed, uint32_t N, size_t stride, const double *V, const void *z,
                                const double *vin, uint64_t seed, double q, double t, StimArgs stim, double Cm,
                                ModelParams mp, double *vout, double *partials, hipStream_t st) {
  if (mixed)
    EMRKC_LAUNCH((k_powS_iter<Model, true>), dim3(blocks_for(N)), dim3(kBlock), 0, st, N, stride, V, z, vin,
                       seed, q, t, stim, Cm, mp, vout, partials);
  else
    EMRKC_LAUNCH((k_powS_iter<Model, false>), dim3(blocks_for(N)), dim3(kBlock), 0, st, N, stride, V, z, vin,
                       seed, q, t, stim, Cm, mp, vout, partials);
  return hipGetLastError();
}

#define EMRKC_MODEL_SWITCH(model, CALL)          \
  switch (model) {                               \
    case 1: return CALL(HHModel);                \
    case 2: return CALL(LinearModel);            \
    case 3: return CALL(CrnSurrModel);           \
    case 4: return CALL(TtpSurrModel);           \
    default: return hipErrorInvalidValue;        \
  }

hipError_t launch_init_state(int model, bool mixed, uint32_t N, double *V, void *z, ModelParams mp, hipStream_t st) {
#define CALL(M) init_dispatch<M>(mixed, N, V, z, mp, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

hipError_t launch_head(int model, bool mixed, const Mesh &mesh, const HeadArgs &a, hipStream_t st) {
#define CALL(M) head_dispatch<M>(mixed, mesh, a, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

template <template <class> class Model>
static hipError_t exexrl_dispatch(bool mixed, const Mesh &mesh, const ExArgs &a, hipStream_t st) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  if (mixed)
    EMRKC_LAUNCH((k_exexrl<Model, true>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  else
    EMRKC_LAUNCH((k_exexrl<Model, false>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  return hipGetLastError();
}

hipError_t launch_exexrl(int model, bool mixed, const Mesh &mesh, const ExArgs &a, hipStream_t st) {
#define CALL(M) exexrl_dispatch<M>(mixed, mesh, a, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

template <template <class> class Model>
static hipError_t mrkc_head_dispatch(const Mesh &mesh, const MrkcHeadArgs &a, hipStream_t st) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  EMRKC_LAUNCH((k_mrkc_head<Model>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  return hipGetLastError();
}

hipError_t launch_mrkc_head(int model, const Mesh &mesh, const MrkcHeadArgs &a, hipStream_t st) {
#define CALL(M) mrkc_head_dispatch<M>(mesh, a, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

template <template <class> class Model>
static hipError_t mrkc_inner_dispatch(const Mesh &mesh, const MrkcInnerArgs &a, hipStream_t st) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  EMRKC_LAUNCH((k_mrkc_inner<Model>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  return hipGetLastError();
}

hipError_t launch_mrkc_inner(int model, const Mesh &mesh, const MrkcInnerArgs &a, hipStream_t st) {
#define CALL(M) mrkc_inner_dispatch<M>(mesh, a, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

template <template <class> class Model>
static hipError_t mrkc_rhs_dispatch(int which, const Mesh &mesh, uint32_t N, double t, const double *y, double *out,
                                    StimArgs stim, double Cm, ModelParams mp, hipStream_t st) {
  EMRKC_LAUNCH((k_mrkc_rhs<Model>), dim3(blocks_for(N)), dim3(kBlock), 0, st, which, mesh, N, t, y, out, stim, Cm,
               mp);
  return hipGetLastError();
}

hipError_t launch_mrkc_rhs(int model, int which, const Mesh &mesh, uint32_t N, double t, const double *y,
                           double *out, StimArgs stim, double Cm, ModelParams mp, hipStream_t st) {
#define CALL(M) mrkc_rhs_dispatch<M>(which, mesh, N, t, y, out, stim, Cm, mp, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

hipError_t launch_vec_diff_norm(uint64_t n, const double *a, const double *b, double *out, double *partials,
                                double *result, hipStream_t st) {
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  EMRKC_LAUNCH(k_vec_diff_norm, dim3(nb), dim3(kBlock), 0, st, n, a, b, out, partials);
  EMRKC_LAUNCH(k_reduce_final, dim3(1), dim3(kBlock), 0, st, partials, nb, result);
  return hipGetLastError();
}

template <template <class> class Model>
static hipError_t imexrl_dispatch(bool mixed, uint32_t N, const ImexArgs &a, hipStream_t st) {
  if (mixed)
    EMRKC_LAUNCH((k_imexrl_pre<Model, true>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, N);
  else
    EMRKC_LAUNCH((k_imexrl_pre<Model, false>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, N);
  return hipGetLastError();
}

hipError_t launch_imexrl_pre(int model, bool mixed, uint32_t N, const ImexArgs &a, hipStream_t st) {
#define CALL(M) imexrl_dispatch<M>(mixed, N, a, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

static inline uint32_t mesh_nodes(const Mesh &m) { return m.kind == kGrid ? m.grid.N : m.ell.N; }

hipError_t launch_cg_init(const Mesh &mesh, const double *ML, const double *Dsum, double dconst, double dt,
                          double tol2, const double *x, const double *b, double *r, double *z, double *partials,
                          CgScalars *s, hipStream_t st) {
  const uint32_t nb = blocks_for(mesh_nodes(mesh));
  EMRKC_LAUNCH(k_cg_init, dim3(nb), dim3(kBlock), 0, st, mesh, ML, CgDiag{Dsum, dconst, dt}, x, b, r, z, partials);
  EMRKC_LAUNCH(k_cg_init_final, dim3(1), dim3(kBlock), 0, st, partials, nb, tol2, s);
  return hipGetLastError();
}

// blocks of the direction/operator kernel (its partial sums)
uint32_t cg_apply_blocks(const Mesh &mesh) {
  if (mesh.kind == kEll) return blocks_for(mesh.ell.N);
  uint32_t ntx, nty;
  return grid_tiles(mesh.grid, ntx, nty, 0);
}

hipError_t launch_cg_step(int which, const Mesh &mesh, const double *ML, const double *Dsum, double dconst,
                          double dt, double *x, double *r, double *z, const double *pprev, double *p, double *q,
                          double *partials, CgScalars *s, hipStream_t st) {
  const uint32_t N = mesh_nodes(mesh);
  if (which == kCgApply) {
    const CgDirArgs a{ML, z, pprev, p, q, partials, s, dt};
    if (mesh.kind == kEll) {
      EMRKC_LAUNCH(k_cg_dir_apply_ell, dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh.ell);
    } else {
      uint32_t ntx, nty;
      const uint32_t nb = grid_tiles(mesh.grid, ntx, nty, 0);
      if (mesh.grid.dim == 3)
        EMRKC_LAUNCH(k_cg_dir_apply_tiled<3>, dim3(nb), dim3(kBlock), 0, st, a, mesh.grid, ntx, nty);
      else
        EMRKC_LAUNCH(k_cg_dir_apply_tiled<2>, dim3(nb), dim3(kBlock), 0, st, a, mesh.grid, ntx, nty);
    }
  } else if (which == kCgPqFinal) {
    EMRKC_LAUNCH(k_cg_pq_final, dim3(1), dim3(kBlock), 0, st, partials, cg_apply_blocks(mesh), s);
  } else if (which == kCgUpdate) {
    EMRKC_LAUNCH(k_cg_update, dim3(blocks_for(N)), dim3(kBlock), 0, st, N, ML, CgDiag{Dsum, dconst, dt}, x, r, z, p,
                 q, partials, s);
  } else if (which == kCgRzFinal) {
    EMRKC_LAUNCH(k_cg_rz_final, dim3(1), dim3(kBlock), 0, st, partials, blocks_for(N), s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cg_iterations(const Mesh &mesh, const double *ML, const double *Dsum, double dconst, double dt,
                                int64_t first_index, int count, double *x, double *r, double *z, double *const P[2],
                                double *q, double *partials, CgScalars *s, hipStream_t st) {
  for (int k = 0; k < count; ++k) {
    const int64_t it = first_index + k;
    double *pprev = P[it & 1], *p = P[(it + 1) & 1];
    for (int w = 0; w < kCgLaunches; ++w) {
      const hipError_t e = launch_cg_step(w, mesh, ML, Dsum, dconst, dt, x, r, z, pprev, p, q, partials, s, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_ell_rowsum(const Ell &e, double *out, hipStream_t st) {
  EMRKC_LAUNCH(k_ell_rowsum, dim3(blocks_for(e.N)), dim3(kBlock), 0, st, e, out);
  return hipGetLastError();
}

hipError_t launch_inner(bool mixed, const Mesh &mesh, const InnerArgs &a, hipStream_t st) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  if (mesh.kind == kGrid && !mesh.flat) {
    uint32_t ntx, nty;
    const Grid &g = mesh.grid;
    if (g.dim == 3 && g.inner_variant == 1) {
      const uint32_t ncx = (g.n0 + MX - 1) / MX, ncy = (g.n1 + MY - 1) / MY, ncz = (g.n2 + g.zc - 1) / g.zc;
      if (mixed)
        EMRKC_LAUNCH((k_inner_march<true>), dim3(ncx * ncy * ncz), dim3(kBlock), 0, st, a, g, ncx, ncy);
      else
        EMRKC_LAUNCH((k_inner_march<false>), dim3(ncx * ncy * ncz), dim3(kBlock), 0, st, a, g, ncx, ncy);
      return hipGetLastError();
    }
    if (g.dim == 3) {
      const dim3 grid = tile_grid<3>(g, ntx, nty);
      if (mixed)
        EMRKC_LAUNCH((k_inner_tiled<true, 3>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
      else
        EMRKC_LAUNCH((k_inner_tiled<false, 3>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
    } else {
      const dim3 grid = tile_grid<2>(g, ntx, nty);
      if (mixed)
        EMRKC_LAUNCH((k_inner_tiled<true, 2>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
      else
        EMRKC_LAUNCH((k_inner_tiled<false, 2>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
    }
    return hipGetLastError();
  }
  if (mixed)
    EMRKC_LAUNCH((k_inner<true>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  else
    EMRKC_LAUNCH((k_inner<false>), dim3(blocks_for(N)), dim3(kBlock), 0, st, a, mesh);
  return hipGetLastError();
}

bool fused_supported(const Mesh &mesh) { return mesh.kind == kGrid && !mesh.flat; }

bool split_supported(const Mesh &mesh) { return mesh.kind == kGrid && !mesh.flat && mesh.grid.dim == 3; }

bool inner_all_supported(const Mesh &mesh, int m) {
  return mesh.kind == kGrid && !mesh.flat && mesh.grid.dim == 2 && m >= 2 && m <= kInnerAllMaxM;
}

template <template <class> class Model>
static hipError_t step2d_dispatch(bool mixed, const Grid &g, const InnerAllArgs &a, const HeadArgs &h,
                                  hipStream_t st) {
  const uint32_t ntx = (g.n0 + 7) / 8, nty = (g.n1 + 7) / 8;
  if (mixed)
    EMRKC_LAUNCH((k_step2d<Model, true, 8>), dim3(ntx * nty), dim3(kBlock), 0, st, a, h, g, ntx);
  else
    EMRKC_LAUNCH((k_step2d<Model, false, 8>), dim3(ntx * nty), dim3(kBlock), 0, st, a, h, g, ntx);
  return hipGetLastError();
}

hipError_t launch_step2d(int model, bool mixed, const Mesh &mesh, const InnerAllArgs &a, const HeadArgs &h,
                         hipStream_t st) {
  if (!inner_all_supported(mesh, a.m)) return hipErrorInvalidValue;
#define CALL(M) step2d_dispatch<M>(mixed, mesh.grid, a, h, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

hipError_t launch_inner_all(bool mixed, const Mesh &mesh, const InnerAllArgs &a, hipStream_t st) {
  if (!inner_all_supported(mesh, a.m)) return hipErrorInvalidValue;
  const Grid &g = mesh.grid;
  const uint32_t T = g.inner_variant == 2 ? 16 : 8;  // shapes 3 and 4: 8 x 8 tiles
  const uint32_t ntx = (g.n0 + T - 1) / T, nty = (g.n1 + T - 1) / T;
  if (T == 8) {
    if (mixed)
      EMRKC_LAUNCH((k_inner_all2d<true, 8>), dim3(ntx * nty), dim3(kBlock), 0, st, a, g, ntx);
    else
      EMRKC_LAUNCH((k_inner_all2d<false, 8>), dim3(ntx * nty), dim3(kBlock), 0, st, a, g, ntx);
  } else if (mixed) {
    EMRKC_LAUNCH((k_inner_all2d<true, 16>), dim3(ntx * nty), dim3(kBlock), 0, st, a, g, ntx);
  } else {
    EMRKC_LAUNCH((k_inner_all2d<false, 16>), dim3(ntx * nty), dim3(kBlock), 0, st, a, g, ntx);
  }
  return hipGetLastError();
}

template <template <class> class Model>
static hipError_t head_pw_dispatch(bool mixed, uint32_t N, const HeadArgs &a, hipStream_t st) {
  // non-temporal z accesses with z in blocks (large arrays only)
  const dim3 grid(blocks_for(N));
  if (mixed && a.z_aos)
    EMRKC_LAUNCH((k_head_pw<Model, true, true>), grid, dim3(kBlock), 0, st, a, N);
  else if (mixed)
    EMRKC_LAUNCH((k_head_pw<Model, true, false>), grid, dim3(kBlock), 0, st, a, N);
  else if (a.z_aos)
    EMRKC_LAUNCH((k_head_pw<Model, false, true>), grid, dim3(kBlock), 0, st, a, N);
  else
    EMRKC_LAUNCH((k_head_pw<Model, false, false>), grid, dim3(kBlock), 0, st, a, N);
  return hipGetLastError();
}

hipError_t launch_head_pw(int model, bool mixed, const Mesh &mesh, const HeadArgs &a, hipStream_t st) {
  if (!split_supported(mesh)) return hipErrorInvalidValue;
#define CALL(M) head_pw_dispatch<M>(mixed, mesh.grid.N, a, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

hipError_t launch_inner12(bool mixed, const Mesh &mesh, const Inner12Args &a, hipStream_t st) {
  if (!split_supported(mesh)) return hipErrorInvalidValue;
  // columns of head_zc planes (the split head shape's plane count)
  Grid g = mesh.grid;
  g.zc = g.head_zc;
  const uint32_t ncx = (g.n0 + MX - 1) / MX, ncy = (g.n1 + MY - 1) / MY, ncz = (g.n2 + g.zc - 1) / g.zc;
  if (mixed) {
    EMRKC_LAUNCH((k_inner12_march<true>), dim3(ncx * ncy * ncz), dim3(kBlock), 0, st, a, g, ncx, ncy);
  } else {
    EMRKC_LAUNCH((k_inner12_march<false>), dim3(ncx * ncy * ncz), dim3(kBlock), 0, st, a, g, ncx, ncy);
  }
  return hipGetLastError();
}

uint32_t grid_tiles(const Grid &g, uint32_t &ntx, uint32_t &nty, int shape) {
  if (g.dim == 3)
    return shape == 1 ? tile_grid<3, 1>(g, ntx, nty).x
                      : shape == 2 ? tile_grid<3, 2>(g, ntx, nty).x : tile_grid<3, 0>(g, ntx, nty).x;
  return shape == 1 ? tile_grid<2, 1>(g, ntx, nty).x
                    : shape == 2 ? tile_grid<2, 2>(g, ntx, nty).x : tile_grid<2, 0>(g, ntx, nty).x;
}

template <template <class> class Model, int SH>
static hipError_t head_batch_launch(bool mixed, const BatchInst *tab, const uint16_t *map, uint32_t nb,
                                    uint32_t Ntot, int step_off, hipStream_t st) {
  if (mixed)
    EMRKC_LAUNCH((k_head_batch<Model, true, SH>), dim3(nb), dim3(kBlock), 0, st, tab, map, Ntot, step_off);
  else
    EMRKC_LAUNCH((k_head_batch<Model, false, SH>), dim3(nb), dim3(kBlock), 0, st, tab, map, Ntot, step_off);
  return hipGetLastError();
}

template <template <class> class Model>
static hipError_t head_batch_dispatch(bool mixed, int shape, const BatchInst *tab, const uint16_t *map, uint32_t nb,
                                      uint32_t Ntot, int step_off, hipStream_t st) {
  if (shape == 1) return head_batch_launch<Model, 1>(mixed, tab, map, nb, Ntot, step_off, st);
  if (shape == 2) return head_batch_launch<Model, 2>(mixed, tab, map, nb, Ntot, step_off, st);
  if (shape == kBatchFlatHead) {
    if (mixed)
      EMRKC_LAUNCH((k_head_batch_flat<Model, true>), dim3(nb), dim3(kBlock), 0, st, tab, map, Ntot, step_off);
    else
      EMRKC_LAUNCH((k_head_batch_flat<Model, false>), dim3(nb), dim3(kBlock), 0, st, tab, map, Ntot, step_off);
    return hipGetLastError();
  }
  return head_batch_launch<Model, 0>(mixed, tab, map, nb, Ntot, step_off, st);
}

hipError_t launch_head_batch(int model, bool mixed, int shape, const BatchInst *tab, const uint16_t *map,
                             uint32_t nblocks, uint32_t Ntot, int step_off, hipStream_t st) {
#define CALL(M) head_batch_dispatch<M>(mixed, shape, tab, map, nblocks, Ntot, step_off, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

template <int SH, int MODE>
static hipError_t inner_batch_mode(bool mixed, const BatchInst *tab, const uint16_t *map, uint32_t nblocks,
                                   hipStream_t st) {
  if (mixed)
    EMRKC_LAUNCH((k_inner_batch<true, SH, MODE>), dim3(nblocks), dim3(kBlock), 0, st, tab, map);
  else
    EMRKC_LAUNCH((k_inner_batch<false, SH, MODE>), dim3(nblocks), dim3(kBlock), 0, st, tab, map);
  return hipGetLastError();
}

template <int SH>
static hipError_t inner_batch_launch(bool mixed, int mode, const BatchInst *tab, const uint16_t *map,
                                     uint32_t nblocks, hipStream_t st) {
  if (mode == 1) return inner_batch_mode<SH, 1>(mixed, tab, map, nblocks, st);
  if (mode == 2) return inner_batch_mode<SH, 2>(mixed, tab, map, nblocks, st);
  return inner_batch_mode<SH, 0>(mixed, tab, map, nblocks, st);
}

hipError_t launch_inner_batch(bool mixed, int shape, int mode, const BatchInst *tab, const uint16_t *map,
                              uint32_t nblocks, uint32_t Ntot, hipStream_t st) {
  (void)Ntot;
  if (shape == 1) return inner_batch_launch<1>(mixed, mode, tab, map, nblocks, st);
  if (shape == 2) return inner_batch_launch<2>(mixed, mode, tab, map, nblocks, st);
  return inner_batch_launch<0>(mixed, mode, tab, map, nblocks, st);
}

template <template <class> class Model>
static hipError_t fused_dispatch(bool mixed, const Grid &g, const FusedArgs &a, hipStream_t st) {
  if (g.dim == 3) {
    using T = Tile<3>;
    const uint32_t ntx = (g.n0 + T::TX - 1) / T::TX, nty = (g.n1 + T::TY - 1) / T::TY,
                   ntz = (g.n2 + T::TZ - 1) / T::TZ;
    const dim3 grid(ntx * nty * ntz);
    if (mixed)
      EMRKC_LAUNCH((k_fused<Model, true, 3>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
    else
      EMRKC_LAUNCH((k_fused<Model, false, 3>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
  } else {
    using T = Tile<2>;
    const uint32_t ntx = (g.n0 + T::TX - 1) / T::TX, nty = (g.n1 + T::TY - 1) / T::TY;
    const dim3 grid(ntx * nty);
    if (mixed)
      EMRKC_LAUNCH((k_fused<Model, true, 2>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
    else
      EMRKC_LAUNCH((k_fused<Model, false, 2>), grid, dim3(kBlock), 0, st, a, g, ntx, nty);
  }
  return hipGetLastError();
}

hipError_t launch_fused(int model, bool mixed, const Mesh &mesh, const FusedArgs &a, hipStream_t st) {
  if (mesh.kind != kGrid) return hipErrorInvalidValue;
#define CALL(M) fused_dispatch<M>(mixed, mesh.grid, a, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

hipError_t launch_z_layout(bool mixed, const void *src, void *dst, uint32_t N, uint32_t nz, bool to_blocks,
                           hipStream_t st) {
  const size_t total = (size_t)((N + kZBlock - 1) / kZBlock) * kZBlock * nz;
  const size_t nb = (total + kBlock - 1) / kBlock;
  if (nb > 0x7fffffffu) return hipErrorInvalidValue;
  const dim3 grid((uint32_t)nb);
  if (mixed) {
    if (to_blocks)
      EMRKC_LAUNCH((k_z_layout<float, true>), grid, dim3(kBlock), 0, st, (const float *)src, (float *)dst, N, nz, total);
    else
      EMRKC_LAUNCH((k_z_layout<float, false>), grid, dim3(kBlock), 0, st, (const float *)src, (float *)dst, N, nz, total);
  } else if (to_blocks) {
    EMRKC_LAUNCH((k_z_layout<double, true>), grid, dim3(kBlock), 0, st, (const double *)src, (double *)dst, N, nz,
                 total);
  } else {
    EMRKC_LAUNCH((k_z_layout<double, false>), grid, dim3(kBlock), 0, st, (const double *)src, (double *)dst, N, nz,
                 total);
  }
  return hipGetLastError();
}

hipError_t launch_clock_set(Clock *c, int64_t step, double t0, hipStream_t st) {
  EMRKC_LAUNCH(k_clock_set, dim3(1), dim3(64), 0, st, c, step, t0);
  return hipGetLastError();
}

hipError_t launch_copy_tick(const double *src, double *dst, uint32_t N, Clock *tick, int64_t tick_by,
                            hipStream_t st) {
  const uint32_t nb = src != nullptr ? blocks_for(N) : 1;
  EMRKC_LAUNCH(k_copy_tick, dim3(nb), dim3(kBlock), 0, st, src, dst, N, tick, tick_by);
  return hipGetLastError();
}

hipError_t launch_apply_diffusion(bool mixed, const Mesh &mesh, const double *V, double *out, hipStream_t st) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  if (mixed)
    EMRKC_LAUNCH((k_apply_diffusion<true>), dim3(blocks_for(N)), dim3(kBlock), 0, st, mesh, V, out);
  else
    EMRKC_LAUNCH((k_apply_diffusion<false>), dim3(blocks_for(N)), dim3(kBlock), 0, st, mesh, V, out);
  return hipGetLastError();
}

hipError_t launch_eval_rhs_slow(int model, bool mixed, uint32_t N, const double *V, const void *z, double t,
                                StimArgs stim, double Cm, ModelParams mp, double *out, hipStream_t st) {
#define CALL(M) rhs_dispatch<M>(mixed, N, V, z, t, stim, Cm, mp, out, st)
  EMRKC_MODEL_SWITCH(model, CALL)
#undef CALL
}

static hipError_t finish_reduce(uint32_t nparts, double *partials, double *result, hipStream_t st) {
  EMRKC_LAUNCH(k_reduce_final, dim3(1), dim3(kBlock), 0, st, partials, nparts, result);
  return hipGetLastError();
}

hipError_t launch_norm2_state(bool mixed, uint32_t N, size_t stride, int nz, const double *V, const void *z,
                              double *partials, double *result, hipStream_t st) {
  const uint32_t nb = blocks_for(N);
  if (mixed)
    EMRKC_LAUNCH((k_norm2_state<true>), dim3(nb), dim3(kBlock), 0, st, N, nz, V, z, stride, partials);
  else
    EMRKC_LAUNCH((k_norm2_state<false>), dim3(nb), dim3(kBlock), 0, st, N, nz, V, z, stride, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish_reduce(nb, partials, result, st);
}

hipError_t launch_norm2_random(uint64_t seed, uint64_t count, double *partials, double *result, hipStream_t st) {
  // grid sized like the state reductions: count / nz items per block is fine
  const uint32_t nb = blocks_for(count) > 65536u ? 65536u : blocks_for(count);
  EMRKC_LAUNCH(k_norm2_random, dim3(nb), dim3(kBlock), 0, st, seed, count, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish_reduce(nb, partials, result, st);
}

hipError_t launch_powF_shift(uint32_t N, const double *yV, const double *vin, uint64_t seed, double q, double *zV,
                             hipStream_t st) {
  EMRKC_LAUNCH(k_powF_shift, dim3(blocks_for(N)), dim3(kBlock), 0, st, N, yV, vin, seed, q, zV);
  return hipGetLastError();
}

hipError_t launch_powF_diff(bool mixed, const Mesh &mesh, const double *zV, const double *yV, double *vout,
                            double *partials, double *result, hipStream_t st) {
  const uint32_t N = mesh.kind == kGrid ? mesh.grid.N : mesh.ell.N;
  const uint32_t nb = blocks_for(N);
  EMRKC_LAUNCH((k_powF_diff<false>), dim3(nb), dim3(kBlock), 0, st, mesh, zV, yV, vout, partials);
  (void)mixed;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish_reduce(nb, partials, result, st);
}

hipError_t launch_powS_iter(int model, bool mixed, uint32_t N, size_t stride, const double *V, const void *z,
                            const double *vin, uint64_t seed, double q, double t, StimArgs stim, double Cm,
                            ModelParams mp, double *vout, double *partials, double *result, hipStream_t st) {
  hipError_t e;
#define CALL(M) powS_dispatch<M>(mixed, N, stride, V, z, vin, seed, q, t, stim, Cm, mp, vout, partials, st)
  switch (model) {
    case 1: e = CALL(HHModel); break;
    case 2: e = CALL(LinearModel); break;
    case 3: e = CALL(CrnSurrModel); break;
    case 4: e = CALL(TtpSurrModel); break;
    default: return hipErrorInvalidValue;
  }
#undef CALL
  if (e != hipSuccess) return e;
  return finish_reduce(blocks_for(N), partials, result, st);
}

hipError_t launch_elementary(int fn, bool mixed, const double *x, double *y, uint32_t n, hipStream_t st) {
  if (mixed)
    EMRKC_LAUNCH(k_elementary<MathF32>, dim3(blocks_for(n)), dim3(kBlock), 0, st, fn, x, y, n);
  else
    EMRKC_LAUNCH(k_elementary<MathF64>, dim3(blocks_for(n)), dim3(kBlock), 0, st, fn, x, y, n);
  return hipGetLastError();
}

hipError_t launch_finite_check(uint32_t N, const double *V, int *flag, hipStream_t st) {
  EMRKC_LAUNCH(k_finite_check, dim3(blocks_for(N)), dim3(kBlock), 0, st, N, V, flag);
  return hipGetLastError();
}

}  // namespace emrkc
