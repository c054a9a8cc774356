/*
 * emrkc.h -- C ABI of the MI355X emRKC library (libemrkc.so).
 *
 * The library advances the semi-discrete monodomain model
 *
 *     Cm M dV/dt = chi^{-1} A V + M I_stim(t) - M I_ion(V, z_E, z_S)
 *     dz_E/dt    = Lambda_E(V) (z_E - z_inf(V))          (gating variables)
 *     dz_S/dt    = g_S(V, z_E, z_S)                      (other ionic variables)
 *
 * (paper: section "Space discretization", eq. sd_sys, with the F/S/E split of
 * eq. mono_in_FSE) by the explicit exponential multirate RKC method of the
 * emRKC algorithm: outer RKC stages on the averaged force, each averaged
 * force made of one exponential Euler step for the gates, one ionic
 * evaluation and an inner RKC iteration of lumped-mass diffusion products.
 * A is the negative semidefinite stiffness operator (A = -K) and M the
 * row-sum lumped mass.
 *
 * Conventions shared by every call:
 *  - Return value: EMRKC_OK (0) or a negative EMRKC_E* code.  No call throws
 *    or aborts; the text of the last error of a context is available from
 *    emrkc_last_error().
 *  - Host pointers passed to a call are read during the call only (they are
 *    copied); the caller keeps ownership.  Device pointers (state buffers,
 *    outputs of the evaluation calls) are owned by the caller; the library
 *    never frees them.
 *  - All GPU work of a context is queued on its stream (emrkc_set_stream;
 *    default: the null stream).  Calls return once the work is queued unless
 *    stated otherwise.  One context must not be used from two host threads
 *    at the same time.
 *  - State layout (structure of arrays, node index fastest):
 *      V : double[N]
 *      z : [n_v - 1][N] of double (EMRKC_FP64) or float (EMRKC_MIXED32),
 *          gates first (model order), then the other ionic variables.
 *  - Units are the caller's; the workloads use mm, ms, mV, uF/mm^2, mS/mm
 *    and uA/mm^2.  The ionic models compute their current per unit
 *    capacitance (mV/ms), so that I_ion = Cm * i_ion.
 */
#ifndef EMRKC_H
#define EMRKC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define EMRKC_OK 0
#define EMRKC_EINVAL (-1)       /* invalid argument or call order            */
#define EMRKC_ENOMEM (-2)       /* device or host allocation failed          */
#define EMRKC_EHIP (-3)         /* a HIP runtime call failed                 */
#define EMRKC_ENONFINITE (-4)   /* EMRKC_CHECK_FINITE found a NaN/Inf in V   */
#define EMRKC_ENOCONV (-5)      /* power iteration hit its iteration limit   */
#define EMRKC_EUNSUPPORTED (-6) /* valid but not implemented combination     */

/* ---- enumerations ------------------------------------------------------- */
#define EMRKC_MESH_Q1_GRID 1    /* structured Q1 grid, 2-D or 3-D            */
#define EMRKC_MESH_P1_TET 2     /* unstructured P1 tetrahedra                */
#define EMRKC_MESH_CSR 3        /* assembled operator A = -K in CSR form     */

#define EMRKC_MODEL_HH 1        /* classical Hodgkin-Huxley (N = 3 gates)     */
#define EMRKC_MODEL_LINEAR 2    /* linear test model: i_ion = a V, 1 gate     */
#define EMRKC_MODEL_CRN_SURR 3  /* CRN-shaped surrogate: 15 gates + 5 slow    */
#define EMRKC_MODEL_TTP_SURR 4  /* TTP-shaped surrogate: 12 gates + 6 slow    */

#define EMRKC_FP64 0            /* every quantity in double                  */
#define EMRKC_MIXED32 1         /* z, the ionic arithmetic and the tetrahedral
                                   operator's weights and products in float;
                                   V, grid stencils, recurrences, coefficients
                                   and spectral radii in double              */

#define EMRKC_CHECK_FINITE 1u   /* emrkc_step synchronises and checks V      */
/* Diagnostic flags (results are bit-identical with and without them):
 * EMRKC_EAGER — launch every kernel directly, never from a captured HIP graph;
 * EMRKC_FUSE — use the fused kernel (last inner stage + next head) where it
 *   applies, without asking the autotuner;
 * EMRKC_FLAT — structured grids use the flat (untiled) kernels only;
 * EMRKC_Z_PLANES — emrkc_step (and the autotuner's and profiler's steps)
 *   keep z in the state's component planes while stepping.  Without it, an
 *   emRKC context without rho_every (a single context whose head is not a
 *   z-marching one, 3-D kernel shapes 1 and 2, or a batch) whose z array
 *   holds at least 256 MiB converts z on entry into a library buffer that
 *   holds each block of 256 nodes' components contiguously (n_z x 256
 *   values per block), steps on that buffer and converts back before it
 *   returns; the buffer (the size of z, rounded up to whole blocks) is
 *   allocated on first use, and where that allocation fails the planes are
 *   kept.
 *   emrkc_step_noalloc always keeps the planes.
 * EMRKC_Z_BLOCKS — the block layout above also for z arrays below 256 MiB
 *   (EMRKC_Z_PLANES takes precedence).
 * The environment variables EMRKC_EAGER and EMRKC_FUSE (any value) act like
 * the flags for every context; EMRKC_VERBOSE makes emrkc_autotune print its
 * timings to stderr. */
#define EMRKC_EAGER 2u
#define EMRKC_FUSE 4u
#define EMRKC_FLAT 8u
#define EMRKC_Z_PLANES 0x400u
#define EMRKC_Z_BLOCKS 0x800u
/* Stepping variants (flags):
 * EMRKC_PROGRESSIVE — the progressive splitting of the auxiliary problem
 *   (remark after eq. auxp_exp): the inner problem starts from y and carries
 *   the exponential increment as a constant forcing; on the monodomain split
 *   the gates then end at z + c'_m (z_E - z) instead of z_E.
 * EMRKC_COND_A — (s, m, eta) from stability condition A of the stability
 *   lemma: eta = (6 dt / l_s) m^2/(m^2 - 1) with the smallest m >= 2 such
 *   that eta rho_F <= beta m^2 (single contexts only). */
/* Methods.  EMRKC_METHOD_MRKC is the mRKC method of the paper applied to
 * the monodomain model (section "The mRKC method for the monodomain model"):
 * the stiffest gate (gate 0 of every model here: the m gate, whose rates
 * are the largest) joins the diffusion in the fast term, the other gates
 * join f_S, and there is no exponential stage; emrkc_estimate_rho then
 * estimates the radii of these two terms.  Double precision single
 * contexts on the flat kernels only. */
#define EMRKC_METHOD_EMRKC 0
#define EMRKC_METHOD_MRKC 1
#define EMRKC_PROGRESSIVE 0x100u
#define EMRKC_COND_A 0x200u

/* ---- types -------------------------------------------------------------- */
typedef struct emrkc_ctx emrkc_ctx;

/* Mesh description.  For EMRKC_MESH_Q1_GRID: dim in {2, 3}, n[d] >= 2 nodes
 * per axis, h[d] > 0 spacing; node (i, j, k) has index i + n0*(j + n1*k).
 * The library derives the stiffness and lumped mass itself (exact Q1
 * integration, zero-flux boundary).  For EMRKC_MESH_P1_TET: n_nodes,
 * n_elems, coords[n_nodes][3], tets[n_elems][4] (0-based node indices,
 * any orientation) and fibres[n_elems][3] (fibre direction a_l, any
 * non-zero length); element conductivity D = sigma_l a a^T +
 * sigma_t (I - a a^T) (eq. def_D with sigma_n = sigma_t).
 * For EMRKC_MESH_CSR (the semi-discrete system of section "Space
 * discretization" with the matrices given): n_nodes = n, row_ptr[n + 1]
 * (row_ptr[0] = 0, non-decreasing), col_idx[row_ptr[n]] (0-based, any
 * order, duplicates summed) and values[row_ptr[n]] hold A = -K, already
 * assembled with the conductivity (the conductivity argument is ignored
 * and may be NULL); lumped_mass[n] > 0 is M_L.  f_F(V) = (chi Cm
 * M_L)^{-1} A V.  Every row must sum to zero within 1e-10 of the sum of
 * its magnitudes (A 1 = 0: a zero-flux stiffness operator), since the
 * library applies A in difference form, sum_j A_ij (V_j - V_i); at most 64
 * off-diagonal entries per row.  All arrays are host memory, copied. */
typedef struct {
  int32_t kind;
  int32_t dim;
  int64_t n[3];
  double h[3];
  int64_t n_nodes;
  int64_t n_elems;
  const double *coords;
  const int64_t *tets;
  const double *fibres;
  const int64_t *row_ptr;      /* EMRKC_MESH_CSR */
  const int32_t *col_idx;
  const double *values;
  const double *lumped_mass;
} emrkc_mesh;

/* Effective conductivities (eq. def_D).  Q1 grids use D = diag(sigma_l,
 * sigma_t, sigma_n): fibres along x, sheets along y. */
typedef struct {
  double sigma_l, sigma_t, sigma_n;
} emrkc_conductivity;

typedef struct {
  double chi;             /* surface-to-volume ratio, > 0                    */
  double Cm;              /* membrane capacitance, > 0                       */
  double eps;             /* RKC damping parameter (0.05)                    */
  double rho_safety;      /* factor applied to estimated radii (1.05)        */
  int32_t precision;      /* EMRKC_FP64 or EMRKC_MIXED32                     */
  uint32_t flags;         /* EMRKC_CHECK_FINITE                              */
  const uint8_t *stim_mask; /* host, N entries (nonzero = stimulated), or NULL */
  double stim_amp;        /* I_stim on stimulated nodes (per membrane area)  */
  double stim_t_on;       /* stimulus on for t_on <= t <= t_off              */
  double stim_t_off;
  double rho_F;           /* > 0: spectral radius of f_F used as given       */
  double rho_S;           /* > 0: spectral radius of f_S used as given       */
  double powiter_tol;     /* power-iteration tolerance (1e-2)                */
  double powiter_eps;     /* relative perturbation size (1e-8)               */
  int32_t powiter_max_iter; /* iteration limit per radius (100)             */
  int32_t rho_every;      /* > 0: emrkc_step re-estimates both radii, warm
                             started, before every step whose index is a
                             positive multiple of rho_every (0: never;
                             single contexts only)                         */
  uint64_t powiter_seed;  /* splitmix64 state of the start vector (0)        */
  double linear_a;        /* EMRKC_MODEL_LINEAR: i_ion = a V                 */
  double linear_lambda_E; /* EMRKC_MODEL_LINEAR: constant gate rate (< 0)    */
  int32_t method;         /* EMRKC_METHOD_EMRKC (0) or EMRKC_METHOD_MRKC    */
  int32_t reserved1;      /* 0                                              */
} emrkc_params;

/* Caller-owned state.  t0 and step define the time of the state as
 * t = t0 + step*dt (computed, never accumulated); emrkc_step advances step
 * and writes t.  A stepping call whose dt differs from the one the state
 * was advanced with (step != 0 and t != t0 + step*dt) first moves t0 to
 * t - step*dt, so the clock continues from t and step keeps counting.
 * V and z are device pointers laid out as described above. */
typedef struct {
  double t0;
  int64_t step;
  double t;
  void *V;
  void *z;
} emrkc_state;

/* Per-call statistics of the last emrkc_step. */
typedef struct {
  int32_t s, m;           /* outer and inner stage counts                     */
  double eta;             /* inner integration length                         */
  int64_t kernels_per_step;
  int32_t used_graph;     /* 1 if the steps were replayed from a HIP graph    */
  int32_t z_blocks;       /* 1 if z was held in blocks of 256 nodes while the
                             call stepped (see EMRKC_Z_PLANES)                */
} emrkc_stats;

/* ---- host-only helpers (no GPU needed) ---------------------------------- */

/* Fills *p with the defaults named above (chi = 140, Cm = 0.01, eps = 0.05,
 * rho_safety = 1.05, FP64, no stimulus, radii to be estimated, tol 1e-2,
 * eps 1e-8, 100 iterations, seed 0). */
void emrkc_default_params(emrkc_params *p);

/* Number of state variables including V (n_v) and of gates of a model, or
 * EMRKC_EINVAL for an unknown model. */
int emrkc_model_num_vars(int ionic_model);
int emrkc_model_num_gates(int ionic_model);

/* RKC coefficients of the RKC algorithm (get_coeffs): for j = 0..s the
 * arrays receive mu_j, nu_j, kappa_j, c_j (entries that the algorithm does
 * not define are 0).  Each array must hold s + 1 doubles.  s in [1, 10000],
 * eps > 0. */
int emrkc_rkc_coeffs(int s, double eps, double *mu, double *nu, double *kappa, double *c);

/* Stage counts under stability condition A (see EMRKC_COND_A); s as in
 * emrkc_stage_counts, m >= 2. */
int emrkc_stage_counts_a(double dt, double rho_F, double rho_S, double eps, int *s, int *m, double *eta);

/* Stage counts of the emRKC algorithm for given radii (get_stages twice):
 * s = max(1, ceil(sqrt(dt rho_S / beta))), eta = 2 dt / (beta s^2),
 * m = max(1, ceil(sqrt(eta rho_F / beta))), beta = 2 - 4 eps / 3. */
int emrkc_stage_counts(double dt, double rho_F, double rho_S, double eps,
                       int *s, int *m, double *eta);

/* ---- context ------------------------------------------------------------ */

/* Creates a context on the current HIP device: validates and copies the
 * inputs, builds the diffusion operator (with 1/(chi Cm M_ii) folded into
 * each row) and allocates the library's work buffers.  *out is set to NULL
 * on failure. */
int emrkc_create(const emrkc_mesh *mesh, const emrkc_conductivity *cond, int ionic_model,
                 const emrkc_params *params, emrkc_ctx **out);

/* Frees every buffer the library owns.  NULL is accepted. */
void emrkc_destroy(emrkc_ctx *ctx);

/* Routes all later work of ctx to the HIP stream `hip_stream` (a
 * hipStream_t; NULL selects the null stream). */
int emrkc_set_stream(emrkc_ctx *ctx, void *hip_stream);

int64_t emrkc_num_nodes(const emrkc_ctx *ctx);   /* N, or -1 for NULL */
int emrkc_num_vars(const emrkc_ctx *ctx);        /* n_v, or -1 for NULL */
/* Row width of the unstructured operator (ELL slots per node), 0 on grids,
 * -1 for NULL. */
int emrkc_ell_width(const emrkc_ctx *ctx);
const char *emrkc_last_error(const emrkc_ctx *ctx);

/* Writes the model's uniform resting state (V and every z) into the state
 * buffers and restarts its clock: step = 0, t = t0.  The initial values are
 * those the ionic model defines (section "Computational setup": the
 * simulations start from the model's own initial state; for the models
 * here that is their resting state, see the model list above). */
int emrkc_init_state(emrkc_ctx *ctx, emrkc_state *state);

/* Spectral radii of the Jacobians of f_F and f_S at `state` by the nonlinear
 * power iteration of the appendix (Compute_Rho), warm-started from the
 * context's previous vectors, then multiplied by rho_safety and stored in
 * the context.  Norms are Euclidean over every state component and
 * computed in double in both precisions.  Synchronises the stream.  Any of
 * the output pointers may be NULL.  Returns EMRKC_ENOCONV if either
 * iteration reached powiter_max_iter (the radii are still stored). */
int emrkc_estimate_rho(emrkc_ctx *ctx, const emrkc_state *state, double *rho_F, double *rho_S,
                       int *iters_F, int *iters_S);

/* Sets the radii used by emrkc_step (taken as given, no safety factor). */
int emrkc_set_rho(emrkc_ctx *ctx, double rho_F, double rho_S);
int emrkc_get_rho(const emrkc_ctx *ctx, double *rho_F, double *rho_S);

/* (s, m, eta) that emrkc_step would use for dt with the stored radii: the
 * two get_stages calls at the head of the emRKC algorithm ("One step of
 * the emRKC method"), s from dt rho_S, eta = 2 dt / (beta s^2) and m from
 * eta rho_F, under stability condition B (condition A with EMRKC_COND_A);
 * the formulas are those of emrkc_stage_counts. */
int emrkc_stages(const emrkc_ctx *ctx, double dt, int *s, int *m, double *eta);

/* Advances `state` by nsteps >= 0 emRKC steps of size dt > 0 (emRKC_Step of
 * the emRKC algorithm).  Requires radii (estimated or set).  Work is queued
 * on the context stream; state->step and state->t are updated on return.
 * With EMRKC_CHECK_FINITE the call synchronises and returns
 * EMRKC_ENONFINITE if V holds a NaN or infinity. */
int emrkc_step(emrkc_ctx *ctx, emrkc_state *state, double dt, int64_t nsteps);

/* emrkc_step for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops and harnesses that forbid
 * hipMalloc.  Advances the state exactly as emrkc_step does (same kernels,
 * same bits) and calls no hipMalloc, hipFree or other allocating routine:
 * the kernels' work buffers (the device clock, V_1, the inner values u_k,
 * S_V and, for s >= 2, z_1) live in a static array of 64 MiB per device that
 * the library holds until the process ends, and every kernel is launched
 * directly on the context stream (no graph is instantiated).  Needs
 * 8 B (4 B for S_V in the mixed precision) per node for each of V_1, u_1,
 * u_2 and S_V (plus one more u and S_V with EMRKC_FUSE, plus z_1 when
 * s >= 2) within the 64 MiB, i.e. about 2 million nodes at s = 1, and stage
 * counts up to 1024; larger problems return EMRKC_EINVAL (EMRKC_EUNSUPPORTED
 * for stage counts) with the reason in emrkc_last_error.  Single emRKC
 * contexts only, without rho_every or EMRKC_CHECK_FINITE (EMRKC_EUNSUPPORTED
 * otherwise); the current device must be the context's.  Every call on one
 * device shares that device's array and overwrites what the previous call
 * left there (each call sets its clock before use and writes every other
 * buffer before reading it), so calls that can overlap on one device --
 * contexts on concurrently running streams -- race and must be ordered by
 * the caller. */
int emrkc_step_noalloc(emrkc_ctx *ctx, emrkc_state *state, double dt, int64_t nsteps);

/* Diagnostic form of emrkc_step: advances the state the same way (same
 * kernels, same results) as one chunk of nsteps steps, but launches every
 * kernel directly on the context stream with a HIP event recorded before
 * and after it, synchronises, and writes the mean duration in ms and the
 * launch count of each kernel class: [0] outer-stage head, [1] inner stage
 * (including the last one of a chunk), [2] fused last-inner-stage + head.
 * 1 <= nsteps <= 1e5.  ms and counts (3 entries each) may be NULL. */
int emrkc_profile_step(emrkc_ctx *ctx, emrkc_state *state, double dt, int64_t nsteps, double *ms,
                       int64_t *counts);

/* Statistics of the last emrkc_step call. */
int emrkc_last_stats(const emrkc_ctx *ctx, emrkc_stats *out);

/* ---- batched ensembles ---------------------------------------------------- */

/* Creates one context for n_inst independent instances advanced together
 * (same ionic model, precision and time step; own Q1 grid, conductivity,
 * chi, Cm, stimulus and spectral radii).  meshes, conds and params are
 * arrays of n_inst entries; precision, eps, rho_safety, flags and the
 * power-iteration settings are taken from params[0].  Instances are
 * concatenated: instance k owns nodes [off_k, off_k + N_k) of V and of every
 * z plane, planes are N_total apart (offsets from emrkc_batch_info).  Every
 * call above accepts a batch context: the state holds N_total nodes,
 * emrkc_estimate_rho estimates each instance's radii (the outputs are the
 * largest ones), and emrkc_step advances all instances with one launch per
 * stage.  The outer stage count s is common (from the largest rho_S) and
 * must be 1 (EMRKC_EUNSUPPORTED otherwise); each instance uses its own
 * inner stage count m_k.  emrkc_eval_rhs_slow rejects batch contexts. */
int emrkc_create_batch(int n_inst, const emrkc_mesh *meshes, const emrkc_conductivity *conds, int ionic_model,
                       const emrkc_params *params, emrkc_ctx **out);

/* Number of instances (1 for a single context), -1 for NULL. */
int emrkc_batch_size(const emrkc_ctx *ctx);

/* offsets[n_inst + 1] (node offsets, last = N_total), m[n_inst] (inner stage
 * counts at dt; 0 before radii are known), rho_F[n_inst], rho_S[n_inst];
 * any output may be NULL. */
int emrkc_batch_info(const emrkc_ctx *ctx, double dt, int64_t *offsets, int *m, double *rho_F, double *rho_S);

/* Sets every instance's radii (taken as given). */
int emrkc_batch_set_rho(emrkc_ctx *ctx, const double *rho_F, const double *rho_S);

/* The two terms of the mRKC split (see EMRKC_METHOD_MRKC) at (t, state):
 * which = 0: f~_F = (f_F, rate of gate 0, 0 ...), which = 1: f~_S = (V part
 * of f_S, 0, rates of gates 1.., g_S).  out is a device double[n_v * N] in
 * the layout [V | z planes]; the context must be double precision and not a
 * batch.  Allocates a work copy of the state on first use. */
int emrkc_eval_mrkc_terms(emrkc_ctx *ctx, const emrkc_state *state, double t, int which, double *out);

/* ---- reference stepping ----------------------------------------------------
 * nsteps steps of EXEX-RL, the fine reference method of the error
 * measurements (IMEX-RL algorithm of the numerical experiments with its
 * diffusion solve replaced by an explicit update):
 *   z_E^{n+1} = z_E^n + (e^{dt Lambda_E(V^n)} - 1)(z_E^n - z_inf(V^n)),
 *   z_S^{n+1} = z_S^n + dt g_S(V^n, z_E^{n+1}, z_S^n),
 *   V^{n+1} = V^n + dt [f_F(V^n) + Cm^{-1}(I_stim(t_n) - I_ion(V^n, z^{n+1}))],
 * on the context's mesh, model and stimulus, t_n = t0 + n dt.  Needs no
 * radii (stable only for dt below the explicit limit of the diffusion).
 * Single contexts; same state layout and stream semantics as emrkc_step. */
int emrkc_exexrl_step(emrkc_ctx *ctx, emrkc_state *state, double dt, int64_t nsteps);

/* nsteps steps of IMEX-RL (algorithm "One step of the IMEX-RL method" of the
 * numerical experiments): z as in emrkc_exexrl_step, then V^{n+1} from the
 * implicit diffusion line
 *   (I - dt F) V^{n+1} = V^n + dt Cm^{-1}(I_stim(t_n) - I_ion(V^n, z^{n+1})),
 * F = (chi Cm M_L)^{-1} A with the lumped mass M_L.  The system is solved by
 * conjugate gradients in the M_L-weighted inner product (in which I - dt F is
 * symmetric positive definite), Jacobi preconditioned, started from V^n and
 * stopped when the preconditioned residual norm falls below 1e-13 times that
 * of the right-hand side; the solve is always in double precision.  Needs no
 * radii and is stable for any dt.  The host reads two reduced scalars per
 * iteration (a synchronisation each); V is updated in place and the context's
 * work vectors hold the solver's vectors.  Allocates the lumped mass (grids)
 * and the solver's extra vectors on first use.  Returns EMRKC_ENOCONV when a
 * solve takes more than 2000 iterations (the state is then part-way through
 * that step).  Single contexts; same state layout as emrkc_step. */
int emrkc_imexrl_step(emrkc_ctx *ctx, emrkc_state *state, double dt, int64_t nsteps);

/* Conjugate-gradient iterations summed over the steps of the last
 * emrkc_imexrl_step call; -1 for NULL. */
int64_t emrkc_imexrl_iterations(const emrkc_ctx *ctx);

/* nsteps IMEX-RL steps as emrkc_imexrl_step, launched one solver iteration
 * at a time with HIP events on each kernel; ms[4] receives the mean
 * duration and counts[4] the launch count of each kernel class: [0] the
 * pointwise step (gates, slow variables, right-hand side), [1] the solver's
 * initial residual, [2] the new direction p with the operator product
 * q = (I - dt F) p, [3] the update of x, r and z.  1 <= nsteps <= 1e4; ms
 * and counts may be NULL.  Synchronises after every iteration. */
int emrkc_profile_imexrl(emrkc_ctx *ctx, emrkc_state *state, double dt, int64_t nsteps, double *ms,
                         int64_t *counts);

/* ---- kernel shapes --------------------------------------------------------
 * variants[5] = {head kernel, head planes per column, inner kernel, inner
 * planes per column, fused}.
 * On 3-D structured grids, head kernel: 0 = 3-D tiles of 16x4x4 nodes, 1 =
 * z-marching columns of 32x8 nodes with the ionic state of the next plane
 * prefetched into registers, 2 = z-marching columns with that state staged
 * through LDS by direct global-to-LDS loads (grids with 8 N < 2^32 only),
 * 3 and 4 = the 3-D tiles compiled for at least 6 and 8 resident waves per
 * SIMD (fewer registers), 5 = flat: one node per thread in index order,
 * stencil operands read through the caches (the default on 3-D grids), 6 =
 * the flat head compiled for at least 7 resident waves per SIMD (mixed
 * precision only; EMRKC_EUNSUPPORTED in FP64, where it would spill); 7 and
 * 8 = the split stage (m >= 2): a pointwise head (exponential Euler, ionic
 * model, outer z recurrence and S_V, no stencil), with the first two inner
 * stages in one column kernel of `head planes` planes (7) or the first
 * inner stage as one more launch of the inner kernel (8, head planes 0).
 * Inner kernel: 0 = 3-D tiles, 1 = z-marching columns.  Planes per column
 * in [1, 64] and at most n[2] for the column kernels, else 0.
 * On 2-D structured grids (emRKC, single contexts) the head is the 2-D tile
 * kernel (entries 0, 1 and 3 are 0) and the inner kernel is 0 = 2-D tiles,
 * one launch per inner stage; 2 = all inner stages of an outer stage in one
 * launch (2 <= m <= 9; 16x16 tiles, u_1, V and S_V staged with halos of up
 * to m nodes); 3 = the same with 8x8 tiles; 4 = as 3 and, when s == 1, the
 * head of the next step in the same kernel (one launch per step); with m
 * outside [2, 9] the separate launches are used.  Shapes 2-4 exclude fused.
 * Other meshes have one head and one inner shape (entries 0..3 are 0), and
 * so do mRKC contexts (flat kernels, no fused kernel).  Batch contexts:
 * variants[0] is the tile shape of the batched head and inner kernels (0:
 * 16x4x4 in 3-D, 64x4 in 2-D; 1: 32x4x2 / 32x8; 2: 8x8x4 / 128x2),
 * variants[1] = 1 makes the head flat (blocks of 256 consecutive nodes of
 * an instance), variants[2] selects the inner stages' layout: 0 = one tile
 * per block, 1 = z-marching columns of variants[3] planes (1..64) for the
 * 3-D instances (tiles for the others), 2 = two tiles per block;
 * variants[3] is 0 unless variants[2] == 1, variants[4] is 0.
 * fused = 1 (structured grids, single contexts): when s == 1 and m >= 2,
 * the last inner stage of each step and the head of the next are one
 * kernel on 3-D or 2-D tiles.
 * Every variant gives bit-identical results; only speed differs. */

/* Times the candidate shapes for a few steps each (`reps` timed steps, on a
 * copy of `state`, which is not modified; every timing is the faster of two
 * repetitions) and keeps the fastest.  3-D grids: the head and inner kernels
 * by their own launch times (the flat head and the 3-D tiles first: a later
 * candidate must be at least 3% faster), then the split stage (shape 7 with
 * columns of 4..64 planes, shape 8 with each inner candidate, chosen by the
 * inner launches' time) against the separate kernels: where the summed
 * launch times put the split within 3% of them, the two run whole steps
 * head to head (alternating, fastest of three) and the faster is kept; then
 * the fused kernel (3%).  Head candidates: the
 * flat head (in the mixed precision also its 7-wave form), tiles (three
 * register budgets), and columns of 2, 3, 4, 8, 16 or 32 planes that leave
 * at least 256 blocks; inner candidates: tiles and those columns.  2-D
 * grids with 2 <= m <= 9: the 2-D shapes 0, 2, 3, 4 (4 when s == 1) and the
 * fused kernel by the wall time per step of eagerly launched steps.  A
 * batch: the three tile shapes by the time per step, the flat head by the
 * head's time, then two tiles per block and z-marching columns of 4, 8 or
 * 64 planes by the inner stage's time.  Needs the radii (the stage plan at
 * dt decides which shapes apply).  Writes the choice to `variants` (int[5])
 * when non-NULL.  Allocates a temporary copy of the state; synchronises the
 * stream.  Returns the fixed choice where nothing can be tuned. */
int emrkc_autotune(emrkc_ctx *ctx, const emrkc_state *state, double dt, int reps, int *variants);

int emrkc_get_variants(const emrkc_ctx *ctx, int *variants);   /* int[5] */

/* Sets the shapes (int[5]); EMRKC_EINVAL for values out of range,
 * EMRKC_EUNSUPPORTED for a shape this context cannot use. */
int emrkc_set_variants(emrkc_ctx *ctx, const int *variants);

/* ---- evaluation of single terms (component checks) ---------------------- */

/* out[i] = ((chi Cm M_L)^{-1} A V)_i for i < N: the V component of f_F
 * (eq. mono_in_FSE).  V and out are device double[N], distinct. */
int emrkc_apply_diffusion(emrkc_ctx *ctx, const double *V, double *out);

/* out = f_S(t, y) for the full state (eq. mono_in_FSE): V component
 * Cm^{-1}(I_stim(t) - I_ion), gate components 0, other components g_S.
 * out is device double[n_v * N] in the state layout; computed in double in
 * both precisions. */
int emrkc_eval_rhs_slow(emrkc_ctx *ctx, const emrkc_state *state, double t, double *out);

/* Elementary functions of the ionic models as the kernels evaluate them:
 * y[i] = f(x[i]) for i < n with f = exp (fn 0), expm1 (fn 1) or log (fn 2),
 * in double (precision EMRKC_FP64) or in single precision (EMRKC_MIXED32:
 * x rounded to float, result widened to double).  x and y are device
 * double[n]; the work is queued on `hip_stream` (NULL: null stream) and the
 * call waits for it.  EMRKC_EINVAL for an unknown fn or precision, n < 0 or
 * NULL pointers with n > 0. */
int emrkc_eval_elementary(int fn, int precision, const double *x, double *y, int64_t n, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* EMRKC_H */
