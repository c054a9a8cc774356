// Device-side building blocks of the emRKC library: arithmetic policies for
// the two precisions, the ionic models, the structured Q1 diffusion stencil
// and the block-index remapping for the MI355X's eight XCDs.
//
// The ionic models follow the monodomain model's gate form
// dz/dt = alpha (1 - z) - beta z, rewritten as Lambda_E (z - z_inf) with
// Lambda_E = -(alpha + beta) and z_inf = alpha / (alpha + beta); their ionic
// current is per unit capacitance (mV/ms), so that I_ion = Cm * i_ion.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace emrkc {

// ---------------------------------------------------------------------------
// Elementary functions.  The ionic models spend most of their arithmetic in
// exp, expm1 and log; the device libm versions of the double functions cost
// 40 to 100 vector instructions each, so double precision uses the short
// forms below (all on finite arguments):
//   * exp / expm1: reduction x = k ln2 + r, |r| <= ln2/2, with ln2 split in
//     a rounded part and its remainder and both products taken with fused
//     multiply-adds (Cody and Waite); e^r - 1 = r + r^2 p(r) with p the
//     degree-9 minimax polynomial of (e^r - 1 - r)/r^2 on [-ln2/2, ln2/2]
//     (Remez exchange, coefficients from gen_exp_minimax.py: its error
//     1.0e-16 in p is at most 1.2e-17 relative in e^r; the degree-13 Taylor
//     form it replaces took two more fused multiply-adds) and reconstruction
//     e^x = 2^k (1 + q), e^x - 1 = 2^k q + (2^k - 1) (exact for k = 0, so
//     expm1 keeps full relative accuracy near 0).  About 1 ulp (exp) and 3
//     ulp (expm1); e^x underflows to 0 below -745 and overflows above 709.8;
//     an infinite argument yields NaN (non-finite in, non-finite out).
//   * log: x = 2^e m with m in [sqrt(1/2), sqrt(2)), log m = 2 atanh(s),
//     s = (m - 1)/(m + 1), |s| <= 0.172, from the odd series of atanh to
//     s^21 (remainder below 1e-17 relative); log x = e ln2 + log m.  About
//     2 ulp; 0 gives -inf, inf gives inf, negative or NaN gives NaN.
// The single precision forms use the native exp2/log2/rcp instructions and a
// degree-7 version of the reduced expm1 above.
// ---------------------------------------------------------------------------
namespace detail {
constexpr double kLn2Hi = 0.6931471805599453;       // ln 2 rounded to double
constexpr double kLn2Lo = 2.3190468138462996e-17;   // ln 2 - kLn2Hi
constexpr double kLog2E = 1.4426950408889634;
constexpr float kLn2HiF = 0.6931472f;
constexpr float kLn2LoF = -1.9046542e-09f;
constexpr float kLog2EF = 1.442695f;

// e^r - 1 for x = k ln2 + r; returns q and sets k.
__device__ __forceinline__ double expm1_reduced(double x, int &k) {
  const double kd = __builtin_rint(x * kLog2E);
  double r = __builtin_fma(-kd, kLn2Hi, x);
  r = __builtin_fma(-kd, kLn2Lo, r);
  // q = r + r^2 p(r), p the degree-9 minimax polynomial of (e^r - 1 - r)/r^2
  // on [-ln2/2, ln2/2] (Remez exchange; gen_exp_minimax.py)
  double p = 0x1.af631ec60423bp-26;
  p = __builtin_fma(p, r, 0x1.28917d2f3a399p-22);
  p = __builtin_fma(p, r, 0x1.71ddf6ba48e19p-19);
  p = __builtin_fma(p, r, 0x1.a019b913fad3ap-16);
  p = __builtin_fma(p, r, 0x1.a01a01b009f52p-13);
  p = __builtin_fma(p, r, 0x1.6c16c1788a1f2p-10);
  p = __builtin_fma(p, r, 0x1.111111110f808p-7);
  p = __builtin_fma(p, r, 0x1.5555555553d67p-5);
  p = __builtin_fma(p, r, 0x1.5555555555558p-3);
  p = __builtin_fma(p, r, 0x1.0000000000001p-1);
  k = (int)kd;  // saturates for |x| > 1.4e9, where 2^k is 0 or inf anyway
  return __builtin_fma(p * r, r, r);
}

__device__ __forceinline__ float expm1_reduced(float x, int &k) {
  const float kf = __builtin_rintf(x * kLog2EF);
  float r = __builtin_fmaf(-kf, kLn2HiF, x);
  r = __builtin_fmaf(-kf, kLn2LoF, r);
  float p = 1.0f / 5040.0f;
  p = __builtin_fmaf(p, r, 1.0f / 720.0f);
  p = __builtin_fmaf(p, r, 1.0f / 120.0f);
  p = __builtin_fmaf(p, r, 1.0f / 24.0f);
  p = __builtin_fmaf(p, r, 1.0f / 6.0f);
  p = __builtin_fmaf(p, r, 0.5f);
  k = (int)kf;
  return __builtin_fmaf(p * r, r, r);
}

__device__ __forceinline__ double exp_f64(double x) {
  int k;
  const double q = expm1_reduced(x, k);
  return __builtin_amdgcn_ldexp(q + 1.0, k);
}

__device__ __forceinline__ double expm1_f64(double x) {
  int k;
  const double q = expm1_reduced(x, k);
  return __builtin_amdgcn_ldexp(q, k) + (__builtin_amdgcn_ldexp(1.0, k) - 1.0);
}

__device__ __forceinline__ float expm1_f32(float x) {
  int k;
  const float q = expm1_reduced(x, k);
  return __builtin_amdgcn_ldexpf(q, k) + (__builtin_amdgcn_ldexpf(1.0f, k) - 1.0f);
}

__device__ __forceinline__ double rcp_f64(double b) {
  // hardware estimate refined by two Newton steps (within an ulp or two)
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double log_f64(double x) {
  int e = __builtin_amdgcn_frexp_exp(x);
  double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
  if (m < 0.70710678118654752) {
    m = m + m;
    e -= 1;
  }
  const double s = (m - 1.0) * rcp_f64(m + 1.0);
  const double s2 = s * s;
  // atanh(s)/s = sum_{j>=0} s^{2j}/(2j+1)
  double p = 1.0 / 21.0;
  p = __builtin_fma(p, s2, 1.0 / 19.0);
  p = __builtin_fma(p, s2, 1.0 / 17.0);
  p = __builtin_fma(p, s2, 1.0 / 15.0);
  p = __builtin_fma(p, s2, 1.0 / 13.0);
  p = __builtin_fma(p, s2, 1.0 / 11.0);
  p = __builtin_fma(p, s2, 1.0 / 9.0);
  p = __builtin_fma(p, s2, 1.0 / 7.0);
  p = __builtin_fma(p, s2, 1.0 / 5.0);
  p = __builtin_fma(p, s2, 1.0 / 3.0);
  const double lm = __builtin_fma(2.0 * s * s2, p, 2.0 * s);
  const double ed = (double)e;
  const double r = __builtin_fma(ed, kLn2Hi, __builtin_fma(ed, kLn2Lo, lm));
  const double inf = __builtin_inf();
  const double bad = (x == 0.0) ? -inf : (x > 0.0 ? x : __builtin_nan(""));
  return (x > 0.0 && x < inf) ? r : bad;
}
}  // namespace detail

// ---------------------------------------------------------------------------
// Arithmetic policies.  FP64 uses the elementary functions above and a
// Newton-refined hardware reciprocal for divisions; FP32 uses the native
// exp2/log2/rcp based fast paths (v_exp_f32, v_log_f32, v_rcp_f32) and the
// reduced expm1, whose relative accuracy near 0 carries the exponential Euler
// update of slow gates.
// ---------------------------------------------------------------------------
struct MathF64 {
  using R = double;
  static __device__ __forceinline__ R exp(R x) { return detail::exp_f64(x); }
  static __device__ __forceinline__ R expm1(R x) { return detail::expm1_f64(x); }
  static __device__ __forceinline__ R log(R x) { return detail::log_f64(x); }
  static __device__ __forceinline__ R rcp(R b) { return detail::rcp_f64(b); }
  static __device__ __forceinline__ R div(R a, R b) { return a * detail::rcp_f64(b); }
};

struct MathF32 {
  using R = float;
  static __device__ __forceinline__ R exp(R x) { return __expf(x); }
  static __device__ __forceinline__ R expm1(R x) { return detail::expm1_f32(x); }
  static __device__ __forceinline__ R log(R x) { return __logf(x); }
  static __device__ __forceinline__ R rcp(R b) { return __builtin_amdgcn_rcpf(b); }
  static __device__ __forceinline__ R div(R a, R b) { return a * __builtin_amdgcn_rcpf(b); }
};

// Runtime parameters of the models that have any (the linear test model).
struct ModelParams {
  double lin_a;      // i_ion = a V
  double lin_lamE;   // constant gate rate
};

// x / (e^x - 1) with its removable singularity: 1 - x/2 for |x| < 1e-7.
template <class M>
__device__ __forceinline__ typename M::R x_over_expm1(typename M::R x) {
  using R = typename M::R;
  return (x < R(1e-7) && x > R(-1e-7)) ? R(1) - R(0.5) * x : M::div(x, M::expm1(x));
}

template <class M>
__device__ __forceinline__ void gate_from_rates(typename M::R a, typename M::R b,
                                                typename M::R &lam, typename M::R &zinf) {
  using R = typename M::R;
  R s = a + b;
  lam = -s;
  zinf = a * M::rcp(s);
}

// Classical Hodgkin-Huxley gates m, h, n (modern sign convention, rest near
// -65 mV); the m rates are multiplied by km.
template <class M>
__device__ __forceinline__ void hh_m_gate(typename M::R V, typename M::R km, typename M::R &lam,
                                          typename M::R &zinf) {
  using R = typename M::R;
  R am = km * x_over_expm1<M>(-(V + R(40)) * R(0.1));
  R bm = km * (R(4) * M::exp(-(V + R(65)) * R(1.0 / 18.0)));
  gate_from_rates<M>(am, bm, lam, zinf);
}

template <class M>
__device__ __forceinline__ void hh_core_gates(typename M::R V, typename M::R km,
                                              typename M::R *lam, typename M::R *zinf) {
  using R = typename M::R;
  hh_m_gate<M>(V, km, lam[0], zinf[0]);
  R ah = R(0.07) * M::exp(-(V + R(65)) * R(0.05));
  R bh = M::div(R(1), R(1) + M::exp(-(V + R(35)) * R(0.1)));
  R an = R(0.1) * x_over_expm1<M>(-(V + R(55)) * R(0.1));
  R bn = R(0.125) * M::exp(-(V + R(65)) * R(1.0 / 80.0));
  gate_from_rates<M>(ah, bh, lam[1], zinf[1]);
  gate_from_rates<M>(an, bn, lam[2], zinf[2]);
}

// Surrogate extra gate: alpha = A/(1 + e^{-(V - Va)/sa}), beta = A/(1 + e^{(V - Vb)/sb}).
struct SigmoidGate {
  double A, Va, inv_sa, Vb, inv_sb;
};

// Lambda and z_inf of a surrogate gate from its two exponentials ep, eq in
// double (one reciprocal serves both: no overflow in double)
__device__ __forceinline__ void sigmoid_from_exps(double A, double ep, double eq, double &lam, double &zinf) {
  const double p = 1.0 + ep, q = 1.0 + eq;
  const double pq = p * q, spq = p + q;
  const double r = detail::rcp_f64(pq * spq);
  lam = -A * (spq * spq) * r;
  zinf = q * (pq * r);
}

template <class M>
__device__ __forceinline__ void sigmoid_gate(typename M::R V, const SigmoidGate &g,
                                             typename M::R &lam, typename M::R &zinf) {
  using R = typename M::R;
  // alpha = A/p, beta = A/q with p = 1 + e^{-(V-Va)/sa}, q = 1 + e^{(V-Vb)/sb}:
  // Lambda = -A (p+q)/(p q), z_inf = q/(p+q)
  const R ep = M::exp(-(V - R(g.Va)) * R(g.inv_sa));
  const R eq = M::exp((V - R(g.Vb)) * R(g.inv_sb));
  if constexpr (sizeof(R) == 8) {
    sigmoid_from_exps(g.A, ep, eq, lam, zinf);
  } else {
    const R p = R(1) + ep, q = R(1) + eq;
    lam = -R(g.A) * (p + q) * M::rcp(p * q);
    zinf = q * M::rcp(p + q);
  }
}

constexpr double kRTF = 25.69;
constexpr double kNaO = 140.0, kKO = 5.4, kCaO = 1.8;
constexpr double kNaI0 = 20.0, kKI0 = 108.0, kCaI0 = 1e-4;

// ---------------------------------------------------------------------------
// Models.  Each provides NG (gates), NS (other ionic variables), V_REST,
// gates(V) -> (Lambda_E, z_inf), eval(V, zE, zS) -> (i_ion, g_S) and the
// resting values of the non-gate variables.
// ---------------------------------------------------------------------------
template <class M>
struct HHModel {
  using R = typename M::R;
  static constexpr int NG = 3, NS = 0;
  static constexpr double V_REST = -65.0;
  static __device__ __forceinline__ void gates(R V, const ModelParams &, R *lam, R *zinf) {
    hh_core_gates<M>(V, R(1), lam, zinf);
  }
  // gate 0 alone (the stiffest: m), as gates() computes it
  static __device__ __forceinline__ void gate0(R V, const ModelParams &, R &lam, R &zinf) {
    hh_m_gate<M>(V, R(1), lam, zinf);
  }
  static __device__ __forceinline__ R eval(R V, const R *zE, const R *, R *, const ModelParams &) {
    R m = zE[0], h = zE[1], n = zE[2];
    R n2 = n * n;
    return R(120) * (m * m * m * h) * (V - R(50)) + R(36) * (n2 * n2) * (V + R(77)) +
           R(0.3) * (V + R(54.387));
  }
  static __host__ __device__ double slow_rest(int) { return 0.0; }
};

template <class M>
struct LinearModel {
  using R = typename M::R;
  static constexpr int NG = 1, NS = 0;
  static constexpr double V_REST = 0.0;
  static __device__ __forceinline__ void gates(R, const ModelParams &p, R *lam, R *zinf) {
    lam[0] = R(p.lin_lamE);
    zinf[0] = R(0);
  }
  static __device__ __forceinline__ void gate0(R, const ModelParams &p, R &lam, R &zinf) {
    lam = R(p.lin_lamE);
    zinf = R(0);
  }
  static __device__ __forceinline__ R eval(R V, const R *, const R *, R *, const ModelParams &p) {
    return R(p.lin_a) * V;
  }
  static __host__ __device__ double slow_rest(int) { return 0.0; }
};

// CRN-shaped surrogate: V, 15 gates (m, h, n, g3..g14), 5 slow variables
// (Na_i, K_i, Ca_i, Ca_up, Ca_rel).  Project-written; not the published
// Courtemanche-Ramirez-Nattel model.
static constexpr SigmoidGate kCrnGates[12] = {
    {2.0, -20.0, 1.0 / 10.0, -12.0, 1.0 / 13.0},
    {0.06, -50.0, 1.0 / -8.0, -58.0, 1.0 / -10.4},
    {0.4, -10.0, 1.0 / 12.0, -2.0, 1.0 / 15.6},
    {0.004, -40.0, 1.0 / -10.0, -48.0, 1.0 / -13.0},
    {1.0, -15.0, 1.0 / 6.0, -7.0, 1.0 / 7.8},
    {0.02, -30.0, 1.0 / -7.0, -38.0, 1.0 / -9.1},
    {0.02, -15.0, 1.0 / 8.0, -7.0, 1.0 / 10.4},
    {1.0, -40.0, 1.0 / -20.0, -48.0, 1.0 / -26.0},
    {0.006, 10.0, 1.0 / 15.0, 18.0, 1.0 / 19.5},
    {0.008, 5.0, 1.0 / 13.0, 13.0, 1.0 / 16.9},
    {0.2, -30.0, 1.0 / -10.0, -38.0, 1.0 / -13.0},
    {0.04, 0.0, 1.0 / 10.0, 8.0, 1.0 / 13.0},
};

// The gates of the CRN surrogate in double precision, the same rates as
// hh_core_gates (scaled by 15) and sigmoid_gate over kCrnGates; f(g, Lambda,
// z_inf) is called once per gate.  Each rate exponential is e^{aV + b}, and
// most slopes a recur (1/10, 1/13, 1/8, 1/10.4 and 1/20) or are twice
// another one (1/6, 1/7.8, 1/10 and 1/13 against 1/12, 1/15.6, 1/20 and
// 1/26).  So e^{aV + b} is formed as e^{aV} e^b, with e^b a compile-time
// constant, e^{2aV} as the square of e^{aV} and e^{-aV} as its reciprocal:
// 15 exponentials (the two expm1 of the x/(e^x - 1) rates among them) and 4
// reciprocals in place of 30 exponentials.  Each factor adds at most a
// rounding or two, so every rate stays within a few ulp of the direct form.
// The constants e^b are exp_f64 of constant arguments, which the compiler
// evaluates.  The gates are taken group by group of shared exponentials, so
// that each group is consumed (by f) before the next one is formed.
template <class F>
__device__ __forceinline__ void crn_gates_f64(double V, F f) {
  using detail::exp_f64;
  using detail::rcp_f64;
  auto sig = [&](int g, double ep, double eq) {
    double lam, zinf;
    sigmoid_from_exps(kCrnGates[g].A, ep, eq, lam, zinf);
    f(3 + g, lam, zinf);
  };
  auto hh = [&](int g, double al, double be) {
    double lam, zinf;
    gate_from_rates<MathF64>(al, be, lam, zinf);
    f(g, lam, zinf);
  };
  {  // slopes 1/20, 1/10, 1/26 and 1/13
    const double E20 = exp_f64(V * (1.0 / 20.0)), r20 = rcp_f64(E20);  // e^{+-V/20}
    const double E10 = E20 * E20, r10 = r20 * r20;                     // e^{+-V/10}
    const double E26 = exp_f64(V * (1.0 / 26.0)), r26 = rcp_f64(E26);  // e^{+-V/26}
    const double E13 = E26 * E26, r13 = r26 * r26;                     // e^{+-V/13}
    hh(1, r20 * (0.07 * exp_f64(-65.0 / 20.0)), rcp_f64(1.0 + r10 * exp_f64(-3.5)));  // h
    sig(0, r10 * exp_f64(-2.0), E13 * exp_f64(12.0 / 13.0));
    sig(3, E10 * exp_f64(4.0), r13 * exp_f64(-48.0 / 13.0));
    sig(7, E20 * exp_f64(2.0), r26 * exp_f64(-48.0 / 26.0));
    sig(10, E10 * exp_f64(3.0), r13 * exp_f64(-38.0 / 13.0));
    sig(11, r10, E13 * exp_f64(-8.0 / 13.0));
    sig(9, r13 * exp_f64(5.0 / 13.0), exp_f64((V - 13.0) * (1.0 / 16.9)));
  }
  {  // slopes 1/8 and 1/10.4
    const double E8 = exp_f64(V * 0.125), r8 = rcp_f64(E8);                  // e^{+-V/8}
    const double E104 = exp_f64(V * (1.0 / 10.4)), r104 = rcp_f64(E104);     // e^{+-V/10.4}
    sig(1, E8 * exp_f64(50.0 / 8.0), r104 * exp_f64(-58.0 / 10.4));
    sig(6, r8 * exp_f64(-15.0 / 8.0), E104 * exp_f64(7.0 / 10.4));
  }
  {  // slopes 1/12, 1/6, 1/15.6 and 1/7.8
    const double r12 = exp_f64(V * (-1.0 / 12.0)), r6 = r12 * r12;     // e^{-V/12}, e^{-V/6}
    const double E156 = exp_f64(V * (1.0 / 15.6)), E78 = E156 * E156;  // e^{V/15.6}, e^{V/7.8}
    sig(2, r12 * exp_f64(-10.0 / 12.0), E156 * exp_f64(2.0 / 15.6));
    sig(4, r6 * exp_f64(-15.0 / 6.0), E78 * exp_f64(7.0 / 7.8));
  }
  // slopes of one rate each
  sig(5, exp_f64((V + 30.0) * (1.0 / 7.0)), exp_f64(-(V + 38.0) * (1.0 / 9.1)));
  sig(8, exp_f64(-(V - 10.0) * (1.0 / 15.0)), exp_f64((V - 18.0) * (1.0 / 19.5)));
  hh(0, 15.0 * x_over_expm1<MathF64>(-(V + 40.0) * 0.1),
     15.0 * (4.0 * exp_f64(-(V + 65.0) * (1.0 / 18.0))));  // m
  hh(2, 0.1 * x_over_expm1<MathF64>(-(V + 55.0) * 0.1), 0.125 * exp_f64(-(V + 65.0) * (1.0 / 80.0)));  // n
}

template <class M>
struct CrnSurrModel {
  using R = typename M::R;
  static constexpr int NG = 15, NS = 5;
  static constexpr double V_REST = -65.0;
  static __device__ __forceinline__ void gate0(R V, const ModelParams &, R &lam, R &zinf) {
    hh_m_gate<M>(V, R(15), lam, zinf);
  }
  static __device__ __forceinline__ void gates(R V, const ModelParams &, R *lam, R *zinf) {
    if constexpr (std::is_same<R, double>::value) {
      crn_gates_f64(V, [&](int g, double l, double zi) {
        lam[g] = l;
        zinf[g] = zi;
      });
    } else {
      hh_core_gates<M>(V, R(15), lam, zinf);
#pragma unroll
      for (int g = 0; g < 12; ++g) sigmoid_gate<M>(V, kCrnGates[g], lam[3 + g], zinf[3 + g]);
    }
  }
  static __device__ __forceinline__ R eval(R V, const R *g, const R *zS, R *dS, const ModelParams &) {
    const R Na = zS[0], K = zS[1], Ca = zS[2], Cup = zS[3], Crel = zS[4];
    const R ENa = R(kRTF) * M::log(M::div(R(kNaO), Na));
    const R EK = R(kRTF) * M::log(M::div(R(kKO), K));
    const R ECa = R(0.5 * kRTF) * M::log(M::div(R(kCaO), Ca));
    const R VK = V - EK;
    const R n2 = g[2] * g[2];
    const R iNa = R(12) * (g[0] * g[0] * g[0] * g[1]) * (V - ENa);
    const R iK = R(3.6) * (n2 * n2) * VK;
    const R iL = R(0.03) * (V + R(54.387));
    const R ito = R(0.04) * (g[3] * g[3] * g[3] * g[4]) * VK;
    const R ikur = R(0.02) * (g[5] * g[5] * g[5] * g[6]) * VK;
    const R ical = R(0.03) * (g[7] * g[8]) * (V - ECa);
    const R ikr = R(0.02) * (g[9] * g[10]) * VK;
    const R iks = R(0.01) * (g[11] * g[12]) * VK;
    const R ik1 = M::div(R(0.005) * VK, R(1) + M::exp(R(0.07) * (V + R(80))));
    const R jrel = R(0.5) * (g[13] * g[13] * g[14]) * (Crel - Ca);
    const R jup = M::div(R(0.005) * Ca, Ca + R(0.001));
    const R jtr = (Cup - Crel) * R(1.0 / 50.0);
    constexpr double kJLeak = 0.005 * kCaI0 / (kCaI0 + 0.001);
    dS[0] = R(-1e-4) * iNa + (R(kNaI0) - Na) * R(1.0 / 500.0);
    dS[1] = R(-1e-4) * (iK + ito + ikur + ikr + iks + ik1) + (R(kKI0) - K) * R(1.0 / 500.0);
    dS[2] = R(-2e-6) * ical + R(0.02) * jrel - jup + R(kJLeak) + (R(kCaI0) - Ca) * R(1.0 / 100.0);
    dS[3] = R(0.05) * jup - R(0.05) * jtr;
    dS[4] = R(0.05) * jtr - R(0.001) * jrel;
    return iNa + iK + iL + ito + ikur + ical + ikr + iks + ik1;
  }
  static __host__ __device__ double slow_rest(int k) {
    return k == 0 ? kNaI0 : k == 1 ? kKI0 : k == 2 ? kCaI0 : 1.0;
  }
};

// TTP-shaped surrogate: V, 12 gates (m, h, n, g3..g11), 6 slow variables
// (Na_i, K_i, Ca_i, Ca_sr, Ca_ss, R).  Project-written; not the published
// ten Tusscher-Panfilov model.
__device__ __constant__ static const SigmoidGate kTtpGates[9] = {
    {3.0, -25.0, 1.0 / 9.0, -17.0, 1.0 / 11.7},
    {0.08, -45.0, 1.0 / -7.0, -53.0, 1.0 / -9.1},
    {0.03, -20.0, 1.0 / 9.0, -12.0, 1.0 / 11.7},
    {1.5, -45.0, 1.0 / -18.0, -53.0, 1.0 / -23.4},
    {0.01, 5.0, 1.0 / 14.0, 13.0, 1.0 / 18.2},
    {1.5, -12.0, 1.0 / 6.0, -4.0, 1.0 / 7.8},
    {0.03, -28.0, 1.0 / -7.0, -36.0, 1.0 / -9.1},
    {0.3, -35.0, 1.0 / -6.0, -43.0, 1.0 / -7.8},
    {0.5, -10.0, 1.0 / 8.0, -2.0, 1.0 / 10.4},
};

template <class M>
struct TtpSurrModel {
  using R = typename M::R;
  static constexpr int NG = 12, NS = 6;
  static constexpr double V_REST = -65.0;
  static __device__ __forceinline__ void gate0(R V, const ModelParams &, R &lam, R &zinf) {
    hh_m_gate<M>(V, R(110), lam, zinf);
  }
  static __device__ __forceinline__ void gates(R V, const ModelParams &, R *lam, R *zinf) {
    hh_core_gates<M>(V, R(110), lam, zinf);
#pragma unroll
    for (int g = 0; g < 9; ++g) sigmoid_gate<M>(V, kTtpGates[g], lam[3 + g], zinf[3 + g]);
  }
  static __device__ __forceinline__ R eval(R V, const R *g, const R *zS, R *dS, const ModelParams &) {
    const R Na = zS[0], K = zS[1], Ca = zS[2], Csr = zS[3], Css = zS[4], Rr = zS[5];
    const R ENa = R(kRTF) * M::log(M::div(R(kNaO), Na));
    const R EK = R(kRTF) * M::log(M::div(R(kKO), K));
    const R ECa = R(0.5 * kRTF) * M::log(M::div(R(kCaO), Css));
    const R VK = V - EK;
    const R n2 = g[2] * g[2];
    const R iNa = R(12) * (g[0] * g[0] * g[0] * g[1]) * (V - ENa);
    const R iK = R(3.6) * (n2 * n2) * VK;
    const R iL = R(0.03) * (V + R(54.387));
    const R ito = R(0.03) * (g[3] * g[3] * g[3] * g[4]) * VK;
    const R ikr = R(0.015) * (g[5] * g[6]) * VK;
    const R iks = R(0.01) * (g[7] * g[7]) * VK;
    const R ical = R(0.025) * (g[8] * g[9] * g[10]) * (V - ECa);
    const R ik1 = M::div(R(0.005) * VK, R(1) + M::exp(R(0.07) * (V + R(80))));
    const R jrel = R(0.4) * (g[11] * Rr) * (Csr - Css);
    const R jup = M::div(R(0.004) * Ca, Ca + R(0.00025));
    const R jxfer = (Css - Ca) * R(0.5);
    constexpr double kJLeak = 0.004 * kCaI0 / (kCaI0 + 0.00025);
    dS[0] = R(-1e-4) * iNa + (R(kNaI0) - Na) * R(1.0 / 500.0);
    dS[1] = R(-1e-4) * (iK + ito + ikr + iks + ik1) + (R(kKI0) - K) * R(1.0 / 500.0);
    dS[2] = R(0.1) * jxfer - jup + R(kJLeak) + (R(kCaI0) - Ca) * R(1.0 / 100.0);
    dS[3] = R(0.02) * (jup - R(kJLeak)) - R(0.002) * jrel;
    dS[4] = R(-2e-6) * ical + R(0.01) * jrel - jxfer;
    dS[5] = (R(0.98) - Rr) * R(1.0 / 200.0) - R(5) * (Css - R(1e-4)) * Rr;
    return iNa + iK + iL + ito + ikr + iks + ical + ik1;
  }
  static __host__ __device__ double slow_rest(int k) {
    return k == 0 ? kNaI0 : k == 1 ? kKI0 : k == 2 ? kCaI0 : k == 3 ? 1.0 : k == 4 ? 1e-4 : 0.98;
  }
};

// ---------------------------------------------------------------------------
// Index helpers.
// ---------------------------------------------------------------------------

// Exact unsigned division by a constant for x < 2^31: q = (x * M) >> shift
// with shift = 31 + ceil(log2 d) and M = ceil(2^shift / d).
struct FastDiv {
  uint32_t d;
  uint32_t shift;
  uint64_t mult;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv &f) {
  return (uint32_t)(((uint64_t)x * f.mult) >> f.shift);
}

// The hardware dispatches consecutive workgroups round-robin over the 8
// XCDs, each with its own L2.  Remap so that each XCD walks one contiguous
// range of the domain: neighbouring planes of a stencil then meet in the same
// L2.  Bijective for any grid size.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t kXcd = 8;
  uint32_t xcd = b % kXcd, idx = b / kXcd;
  uint32_t q = nb / kXcd, r = nb % kXcd;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Structured grid geometry passed to kernels.
struct Grid {
  uint32_t n0, n1, n2;   // nodes per axis (n2 = 1 in 2-D)
  uint32_t N;
  FastDiv div0, div1;    // division by n0 and by n1
  int dim;
  // inner-stage and head kernels for 3-D grids: 0 = 3-D tiles, 1 = z-marching
  // columns of zc (head_zc) planes per block (2.5-D); heads also 2 = columns
  // with the ionic state staged through LDS, 3/4 = tiles for 6/8 waves per
  // SIMD, 5 = flat (one node per thread), 6 = flat for 7 waves per SIMD
  // (mixed precision only), 7 and 8 = the split stage with a pointwise head
  // (7: one kernel for the first two inner stages in columns of head_zc
  // planes; 8: the first inner stage as a launch of the inner kernel);
  // on 2-D grids inner 2/3 = all inner stages of a stage in one launch
  // (16 x 16 / 8 x 8 tiles), 4 = one kernel per step (s == 1); chosen by
  // the host
  int inner_variant;
  uint32_t zc;
  int head_variant;
  uint32_t head_zc;
  // weights of (chi Cm M_L)^{-1} A on neighbour differences, by offset class
  // (|ox|, |oy|, |oz|): w[0]=100, w[1]=010, w[2]=001, w[3]=110, w[4]=101,
  // w[5]=011, w[6]=111 (2-D uses w[0], w[1], w[3]); w[7] = w[2] + 2 (w[4] +
  // w[5]) + 4 w[6], the total weight of one neighbouring plane (3-D).
  double w[8];
};

__device__ __forceinline__ uint32_t mirror_lo(uint32_t i) { return i > 0 ? i - 1 : 1; }
__device__ __forceinline__ uint32_t mirror_hi(uint32_t i, uint32_t n) { return i + 1 < n ? i + 1 : n - 2; }

// (chi Cm M_L)^{-1} (A u) at one node in difference form sum_o w_o (u_o - u_c),
// grouped by offset class.  get(dx, dy, dz) returns the neighbour value with
// the boundary already resolved: the zero-flux boundary of the lumped Q1
// operator equals the interior formula with mirrored neighbours.  Both
// precisions take it in double: the weights are kernel arguments, so a float
// form would save no memory traffic, and on gfx950 unpacked float arithmetic
// issues at the double rate, so its conversions would only add instructions.
//
// In 3-D every plane of the 3 x 3 x 3 neighbourhood enters through three
// numbers at the node's (x, y) (PlaneTerms): its centre value c, and the
// weighted in-plane differences to c (edges and corners) as the node's own
// plane (o) and as a neighbouring plane (t).  A difference to a neighbour in
// plane z +- 1 is split as (u_o - c_{z+-1}) + (c_{z+-1} - u_c), so
//   F = o_z + (t_{z-1} + t_{z+1}) + w[7] ((c_{z-1} - c_z) + (c_{z+1} - c_z)).
// A z-marching kernel forms each plane's terms once and keeps them, instead
// of reading 27 values per node.
//
// Written with explicit fused multiply-adds in a fixed order and no further
// contraction, so that the flat, LDS-tiled and z-marching kernels round
// identically.
struct PlaneTerms {
  double c, o, t;
};

template <class Get2>
__device__ __forceinline__ PlaneTerms plane_terms(const double *w, Get2 get) {
#pragma clang fp contract(off)
  const double c = get(0, 0);
  const double ex = (get(-1, 0) - c) + (get(1, 0) - c);
  const double ey = (get(0, -1) - c) + (get(0, 1) - c);
  const double cr = ((get(-1, -1) - c) + (get(1, -1) - c)) + ((get(-1, 1) - c) + (get(1, 1) - c));
  PlaneTerms p;
  p.c = c;
  p.o = __builtin_fma(w[3], cr, __builtin_fma(w[1], ey, w[0] * ex));
  p.t = __builtin_fma(w[6], cr, __builtin_fma(w[5], ey, w[4] * ex));
  return p;
}

__device__ __forceinline__ double plane_combine(const double *w, const PlaneTerms &m, const PlaneTerms &o,
                                                const PlaneTerms &p) {
#pragma clang fp contract(off)
  return __builtin_fma(w[7], (m.c - o.c) + (p.c - o.c), o.o + (m.t + p.t));
}

template <int DIM, class Get>
__device__ __forceinline__ double grid_stencil(const double *w, Get get) {
#pragma clang fp contract(off)
  if (DIM == 2) {
    const double uc = get(0, 0, 0);
    auto d = [&](int dx, int dy) { return get(dx, dy, 0) - uc; };
    const double f = d(-1, 0) + d(1, 0);
    const double e = d(0, -1) + d(0, 1);
    const double c = (d(-1, -1) + d(1, -1)) + (d(-1, 1) + d(1, 1));
    return __builtin_fma(w[3], c, __builtin_fma(w[1], e, w[0] * f));
  }
  const PlaneTerms m = plane_terms(w, [&](int dx, int dy) { return get(dx, dy, -1); });
  const PlaneTerms o = plane_terms(w, [&](int dx, int dy) { return get(dx, dy, 0); });
  const PlaneTerms p = plane_terms(w, [&](int dx, int dy) { return get(dx, dy, 1); });
  return plane_combine(w, m, o, p);
}

// The stencil on a global array at node (ix, iy, iz).
template <int DIM, class P>
__device__ __forceinline__ double grid_apply(P u, const Grid &g, uint32_t ix,
                                             uint32_t iy, uint32_t iz) {
  const uint32_t xs[3] = {mirror_lo(ix), ix, mirror_hi(ix, g.n0)};
  const uint32_t s1 = g.n0;
  const uint32_t ys[3] = {mirror_lo(iy) * s1, iy * s1, mirror_hi(iy, g.n1) * s1};
  const uint32_t s2 = g.n0 * g.n1;
  uint32_t zs[3] = {0, 0, 0};
  if (DIM == 3) {
    zs[0] = mirror_lo(iz) * s2;
    zs[1] = iz * s2;
    zs[2] = mirror_hi(iz, g.n2) * s2;
  }
  return grid_stencil<DIM>(g.w, [&](int dx, int dy, int dz) {
    return u[zs[dz + 1] + ys[dy + 1] + xs[dx + 1]];
  });
}

// splitmix64 (Steele, Lea and Flood, 2014): output number i (0-based) of
// the generator started at state `seed`, mapped to [-1, 1).
__host__ __device__ __forceinline__ double splitmix64_unit(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

}  // namespace emrkc
