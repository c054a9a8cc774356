// Internal interface between the host runtime (emrkc_host.hip) and the
// kernels (emrkc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "emrkc_device.h"

namespace emrkc {

// Device-resident time of the state: t_n = t0 + step * dt.  Kept on the
// device so that a captured sequence of steps can be replayed unchanged.
struct Clock {
  int64_t step;
  double t0;
};

struct StimArgs {
  const uint8_t *mask;  // nullptr: no stimulus
  double amp, t_on, t_off;
};

// Operator of the unstructured (P1) mesh: ELL rows of width `width`, column
// indices and weights of (chi Cm M_L)^{-1} A on neighbour differences; padded
// entries repeat the row's own index with weight 0.
struct Ell {
  uint32_t N;
  uint32_t width;
  const uint32_t *col;   // [width][N]
  const double *w64;     // [width][N]
  const float *w32;      // [width][N] (mixed form)
};

enum MeshKind : int { kGrid = 1, kEll = 2 };

struct Mesh {
  int kind;
  int flat;  // grids: use the flat global-load kernels only (a context's testing switch)
  Grid grid;
  Ell ell;
};

// Fused outer-stage head: exponential Euler on the gates, ionic evaluation
// at y_E, outer recurrence of z and the first inner stage of V.
struct HeadArgs {
  const double *Vin;    // V_{j-1}
  const double *Vin2;   // V_{j-2} (j >= 2)
  const void *zin;      // z_{j-1}
  const void *zin2;     // z_{j-2} (j >= 2)
  void *zout;           // z_j
  void *SV;             // S_V = Cm^{-1}(I_stim - I_ion) at y_E (m >= 2)
  double *uout;         // u_1 (m >= 2) or V_j (m == 1)
  const Clock *clock;   // chunk base step and t0
  int step_off;         // step index within the chunk
  StimArgs stim;
  ModelParams mp;
  double dt, eta, inv_eta, Cm;
  double c_prev;        // c_{j-1}: the stage is evaluated at t_n + c_{j-1} dt
  double mu_dt, nu, kappa;   // outer coefficients of stage j (times dt for mu)
  double mu1_eta;       // mu'_1 * eta of the inner iteration
  double cm_eta;        // c'_m * eta: inner end point of the frozen slow forcing
  int j1;               // stage j == 1
  int m_is_one;
  int progressive;      // progressive splitting: gates end at z + c'_m (z_E - z)
  double cm;            // c'_m
  int z_aos;            // z arrays in blocks of kZBlock nodes (else component planes); flat and pointwise heads
};

// z in blocks: component k of node i at (i / kZBlock) kZBlock n_z + k kZBlock
// + i % kZBlock, so that each wave's components are one contiguous run.
constexpr uint32_t kZBlock = 256;

// Last inner stage k = m of stage j together with the outer V update.
struct TailArgs {
  const double *uprev;   // u_{m-1} (read with neighbours)
  const double *uprev2;  // u_{m-2} (u_0 = V_{j-1} when m == 2)
  const void *SV;
  const double *Vin;     // V_{j-1}
  const double *Vin2;    // V_{j-2} (j >= 2)
  double nu, kappa, mu_eta;      // inner coefficients of stage m
  double inv_eta, mu_dt, nu_o, kappa_o;  // outer coefficients of stage j
  int j1;
};

// Inner stage k >= 2; at k == m (last) it also applies the outer V update.
struct InnerArgs {
  TailArgs t;            // uprev, uprev2, SV and the inner coefficients are used for every k
  double *out;           // u_k, or V_j when last
  int last;
  int first;             // k == 1 of the split stage: u_1 = u_0 + mu'_1 eta (f_F(u_0) + S_V), mu_eta = mu'_1 eta, uprev = u_0
  Clock *tick;           // when non-null, block 0 adds tick_by to the chunk base step
  int64_t tick_by;
};

// Every inner stage k = 2..m of one outer stage in one launch (2-D grids,
// 2 <= m <= kInnerAllMaxM): each block owns a 16 x 16 tile and recomputes
// u_k on the tile plus a halo of m - k nodes from u_1 on a halo of m - 1.
constexpr int kInnerAllMaxM = 9;
struct InnerAllArgs {
  TailArgs t;            // outer coefficients of stage j (inv_eta, mu_dt, nu_o, kappa_o, j1)
  const double *u1;      // u_1 (read on the tile and an m - 1 halo)
  const double *V;       // u_0 = V_{j-1} (read on an m - 2 halo)
  const double *Vin2;    // V_{j-2} (j >= 2)
  const void *SV;
  double *out;           // V_j
  double nu[kInnerAllMaxM + 1], kappa[kInnerAllMaxM + 1], mu_eta[kInnerAllMaxM + 1];  // inner stage k
  int m;
  Clock *tick;           // when non-null, block 0 adds tick_by to the chunk base step
  int64_t tick_by;
};

// First two inner stages of the split stage (3-D grids, m >= 2): u_1 from
// V_{j-1} and S_V, u_2 from u_1, and for m == 2 the outer V update.
struct Inner12Args {
  TailArgs t;            // coefficients of inner stage 2 and of the outer update (uprev unused)
  const double *V;       // V_{j-1} = u_0 (read with a two-node halo)
  const double *Vin2;    // V_{j-2} (m == 2, j >= 2)
  const void *SV;
  double mu1_eta;        // mu'_1 eta
  double *out;           // V_j (m == 2) or u_2
  double *u1out;         // u_1 (m >= 3)
  int last;              // m == 2
  Clock *tick;           // when non-null, block 0 adds tick_by to the chunk base step
  int64_t tick_by;
};

// Tail of the previous step (on the tile plus a one-node halo, staged in
// LDS) fused with the head of the next step (s == 1, m >= 2, grids).
struct FusedArgs {
  TailArgs t;
  double *Vout;          // V^n (tile nodes)
  HeadArgs h;            // h.Vin unused: V comes from the tail
};

// One step of the EXEX-RL reference method at every node.
struct ExArgs {
  const double *Vin;    // V^n (read with neighbours)
  double *Vout;         // V^{n+1}
  void *z;              // z^n, overwritten with z^{n+1}
  const Clock *clock;   // chunk base step and t0
  int step_off;         // step index within the chunk
  StimArgs stim;
  ModelParams mp;
  double dt, Cm;
};

// The pointwise part of an IMEX-RL step: gates by Rush-Larsen and the other
// ionic variables by explicit Euler (z updated in place), and the right-hand
// side V^n + dt Cm^{-1}(I_stim(t) - I_ion(V^n, z^{n+1})) of the diffusion line.
struct ImexArgs {
  const double *V;
  double *rhs;
  void *z;
  double t;
  StimArgs stim;
  ModelParams mp;
  double dt, Cm;
};

// mRKC (double precision): the head of outer stage j and the inner stages
// carry the stiffest gate (gate 0), which sits in the fast term, next to V.
struct MrkcHeadArgs {
  HeadArgs h;           // as for emRKC (no exponential stage); zout plane 0
                        // is written only when m == 1
  double *wout;         // w_1, gate 0 after the first inner stage (m >= 2)
};

struct MrkcInnerArgs {
  InnerArgs a;
  const double *wprev;  // w_{k-1}
  const double *wprev2; // w_{k-2} (w_0 = z_0 of stage j-1 when k == 2)
  double *wout;         // w_k (not last)
  const double *zq_in;  // gate 0 of z_{j-1}
  const double *zq_in2; // gate 0 of z_{j-2} (j >= 2)
  double *zq_out;       // gate 0 of z_j (last)
  ModelParams mp;
};

// One instance of a batched (ensemble) launch.  Instances are concatenated:
// node i of the instance is node off + i of every global array, component
// planes are N_total apart.  Logical blocks tile0 .. tile0 + ntiles - 1 of
// the launch belong to the instance.
struct BatchInst {
  Grid g;
  uint32_t off;
  uint32_t tile0;
  uint32_t ntx, nty;
  HeadArgs h;    // head launches: this instance's coefficients (pointers global)
  InnerArgs in;  // inner launches: this instance's coefficients (pointers global)
};

// Column cross-section (nodes in x and y) of the z-marching kernels.
constexpr int MX = 32, MY = 8;

// ---- launchers (emrkc_kernels.hip) ----------------------------------------
// Events recorded by the next kernel launches of this thread around the
// kernel's execution (profiling); nullptr to stop.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
// Tiles of a grid in the LDS-tiled layout of tile shape `shape` (0: 3-D
// 16x4x4 / 2-D 64x4, 1: 32x4x2 / 32x8, 2: 8x8x4 / 128x2).
uint32_t grid_tiles(const Grid &g, uint32_t &ntx, uint32_t &nty, int shape = 0);
// shape kBatchFlatHead: the flat head, whose table maps blocks of 256
// consecutive nodes of an instance (tile0 = the instance's first block)
constexpr int kBatchFlatHead = 3;
hipError_t launch_head_batch(int model, bool mixed, int shape, const BatchInst *tab, const uint16_t *map,
                             uint32_t nblocks, uint32_t Ntot, int step_off, hipStream_t st);
// mode: the tables' layout: 0 one tile per block, 1 z-marching columns for
// the 3-D instances (their entries have inner_variant 1), 2 two tiles per block
hipError_t launch_inner_batch(bool mixed, int shape, int mode, const BatchInst *tab, const uint16_t *map,
                              uint32_t nblocks, uint32_t Ntot, hipStream_t st);
hipError_t launch_init_state(int model, bool mixed, uint32_t N, double *V, void *z, ModelParams mp,
                             hipStream_t st);
hipError_t launch_head(int model, bool mixed, const Mesh &mesh, const HeadArgs &a, hipStream_t st);
hipError_t launch_inner(bool mixed, const Mesh &mesh, const InnerArgs &a, hipStream_t st);
hipError_t launch_exexrl(int model, bool mixed, const Mesh &mesh, const ExArgs &a, hipStream_t st);
hipError_t launch_mrkc_head(int model, const Mesh &mesh, const MrkcHeadArgs &a, hipStream_t st);
hipError_t launch_imexrl_pre(int model, bool mixed, uint32_t N, const ImexArgs &a, hipStream_t st);
// Conjugate gradients for (I - dt F) x = b in the inner product weighted by
// the lumped mass ML, preconditioned by the diagonal 1 + dt D_i (D_i from
// Dsum, or dconst for every node when Dsum is null), with its scalars on the
// device.  done: 0 running, 1 converged (preconditioned residual norm
// squared <= stop = tol2 * (b, b)), 2 non-finite residual.
struct CgScalars {
  double rz, rz_prev, pq, stop;
  int32_t iters, done, first, pad;
};
// r = b - (x - dt F x), z = r/diag; initialises the scalars (first
// iteration next); writes 2 x ceil(N/256) partial sums
hipError_t launch_cg_init(const Mesh &mesh, const double *ML, const double *Dsum, double dconst, double dt,
                          double tol2, const double *x, const double *b, double *r, double *z, double *partials,
                          CgScalars *s, hipStream_t st);
// the launches of an iteration, in order (each a no-op once the solve is
// done; the vector kernels leave block partial sums, the one-block kernels
// reduce them):
//   kCgApply:   p = z + beta pprev (p = z on the first), q = p - dt F p
//   kCgPqFinal: pq = (p, q)
//   kCgUpdate:  alpha = rz/pq; x += alpha p; r -= alpha q; z = r/diag
//   kCgRzFinal: rz' = (r, z), beta for the next direction, convergence flag
enum CgLaunch : int { kCgApply = 0, kCgPqFinal, kCgUpdate, kCgRzFinal, kCgLaunches };
hipError_t launch_cg_step(int which, const Mesh &mesh, const double *ML, const double *Dsum, double dconst,
                          double dt, double *x, double *r, double *z, const double *pprev, double *p, double *q,
                          double *partials, CgScalars *s, hipStream_t st);
// `count` iterations numbered from first_index; iteration k reads the
// direction from P[k % 2] and writes the new one to P[(k + 1) % 2]
hipError_t launch_cg_iterations(const Mesh &mesh, const double *ML, const double *Dsum, double dconst, double dt,
                                int64_t first_index, int count, double *x, double *r, double *z, double *const P[2],
                                double *q, double *partials, CgScalars *s, hipStream_t st);
// partial sums the kCgApply launch writes (one per block)
uint32_t cg_apply_blocks(const Mesh &mesh);
// out[i] = sum of row i's ELL weights
hipError_t launch_ell_rowsum(const Ell &e, double *out, hipStream_t st);
hipError_t launch_mrkc_inner(int model, const Mesh &mesh, const MrkcInnerArgs &a, hipStream_t st);
// The split terms of mRKC on a full double state y = [V | z planes]:
// which = 0: f~_F = (f_F, gate-0 rate, 0), which = 1: f~_S = (f_S's V part,
// 0, other gates' rates, g_S); out has the same layout.
hipError_t launch_mrkc_rhs(int model, int which, const Mesh &mesh, uint32_t N, double t, const double *y,
                           double *out, StimArgs stim, double Cm, ModelParams mp, hipStream_t st);
// out = a - b over n entries (b == nullptr: b = 0; out == nullptr: not
// stored), partial sums of out^2 per block (ceil(n/256) of them), final sum.
hipError_t launch_vec_diff_norm(uint64_t n, const double *a, const double *b, double *out, double *partials,
                                double *result, hipStream_t st);
hipError_t launch_fused(int model, bool mixed, const Mesh &mesh, const FusedArgs &a, hipStream_t st);
// The fused kernel stages its tile in LDS: grids only, and not under the
// flat-kernel switch (mesh.flat), which covers every grid kernel.
bool fused_supported(const Mesh &mesh);
// The split stage: the pointwise head k_head_pw (z and S_V only) and the
// two-stage inner kernel k_inner12_march; 3-D grids, not under mesh.flat.
bool split_supported(const Mesh &mesh);
// 2-D grids (not mesh.flat): all inner stages of a stage in one launch
bool inner_all_supported(const Mesh &mesh, int m);
hipError_t launch_inner_all(bool mixed, const Mesh &mesh, const InnerAllArgs &a, hipStream_t st);
// The inner stages of step n (s == 1, 8 x 8 tiles) and the head of step
// n + 1 in one kernel (2-D grids, inner shape 4)
hipError_t launch_step2d(int model, bool mixed, const Mesh &mesh, const InnerAllArgs &a, const HeadArgs &h,
                         hipStream_t st);
hipError_t launch_head_pw(int model, bool mixed, const Mesh &mesh, const HeadArgs &a, hipStream_t st);
hipError_t launch_inner12(bool mixed, const Mesh &mesh, const Inner12Args &a, hipStream_t st);
// z (nz components of N nodes, float when mixed) from component planes to
// blocks of kZBlock nodes (to_blocks) or back; dst of the block layout holds
// ceil(N / kZBlock) kZBlock nz values.
hipError_t launch_z_layout(bool mixed, const void *src, void *dst, uint32_t N, uint32_t nz, bool to_blocks,
                           hipStream_t st);
hipError_t launch_clock_set(Clock *c, int64_t step, double t0, hipStream_t st);
hipError_t launch_copy_tick(const double *src, double *dst, uint32_t N, Clock *tick, int64_t tick_by,
                            hipStream_t st);
hipError_t launch_apply_diffusion(bool mixed, const Mesh &mesh, const double *V, double *out,
                                  hipStream_t st);
hipError_t launch_eval_rhs_slow(int model, bool mixed, uint32_t N, const double *V, const void *z,
                                double t, StimArgs stim, double Cm, ModelParams mp, double *out,
                                hipStream_t st);

// Power iteration pieces.  Partial sums go to `partials` (one per block),
// the final sum to `result` (device double).
uint32_t reduce_blocks(uint32_t n);
hipError_t launch_norm2_state(bool mixed, uint32_t N, size_t stride, int nz, const double *V, const void *z,
                              double *partials, double *result, hipStream_t st);
hipError_t launch_norm2_random(uint64_t seed, uint64_t count, double *partials, double *result,
                               hipStream_t st);
hipError_t launch_powF_shift(uint32_t N, const double *yV, const double *vin, uint64_t seed, double q,
                             double *zV, hipStream_t st);
hipError_t launch_powF_diff(bool mixed, const Mesh &mesh, const double *zV, const double *yV, double *vout,
                            double *partials, double *result, hipStream_t st);
hipError_t launch_powS_iter(int model, bool mixed, uint32_t N, size_t stride, const double *V, const void *z,
                            const double *vin, uint64_t seed, double q, double t, StimArgs stim,
                            double Cm, ModelParams mp, double *vout, double *partials, double *result,
                            hipStream_t st);
hipError_t launch_elementary(int fn, bool mixed, const double *x, double *y, uint32_t n, hipStream_t st);
hipError_t launch_finite_check(uint32_t N, const double *V, int *flag, hipStream_t st);

}  // namespace emrkc
