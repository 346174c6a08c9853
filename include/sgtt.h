/*
 * sgtt: low-rank (tensor-train) solver for one Picard step of the stochastic
 * Galerkin, all-at-once discretization of the unsteady Navier-Stokes
 * equations (Elman & Su, "A low-rank solver for the stochastic unsteady
 * Navier-Stokes problem"), on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes; no C++ or framework types cross it.
 * Every function returns an int status: 0 = OK, > 0 = warning, < 0 = error
 * (see SGTT_* codes).  No exception crosses the ABI.  After an error,
 * sgtt_last_error() on the context describes it.
 *
 * Vectors of the all-at-once system are pairs (u, p) of 3-way tensor trains
 * over (time, chaos, space) (sec. 4.1, eq. 4.1-4.2):
 *   z(i1,i2,i3) = sum_{a,b} core1[i1,a] core2[a,i2,b] core3'[b,i3]
 * with the memory layout of sgtt_tt below.  Velocity space dofs are
 * [x1-component on free nodes; x2-component on free nodes] (sec. 3.2), free
 * velocity nodes and pressure nodes sorted by (x1, x2).
 *
 * Threading / streams: calls on one context are ordered on the context's HIP
 * stream; calls are not thread-safe on one context.  Device buffers passed
 * in are owned by the caller and must stay valid for the call.
 */
#ifndef SGTT_H
#define SGTT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define SGTT_OK 0
#define SGTT_W_NOT_CONVERGED 1    /* solve stopped at max cycles; x = best iterate */
#define SGTT_E_INVALID -1         /* bad argument (null pointer, size mismatch)    */
#define SGTT_E_HIP -2             /* HIP runtime error                             */
#define SGTT_E_OOM -3             /* device allocation failed                      */
#define SGTT_E_RANK_CAP -4        /* result rank exceeds the output capacity;
                                     output left unchanged                         */
#define SGTT_E_NONFINITE -5       /* NaN/Inf met in a reduction                    */
#define SGTT_E_SETUP -6           /* problem setup failed (mesh / factorization)   */
#define SGTT_E_IO -7              /* checkpoint file missing, unreadable, of another
                                     format, or failing its hash                    */

typedef struct sgtt_context sgtt_context;
typedef struct sgtt_system sgtt_system;
typedef struct sgtt_host_problem sgtt_host_problem;

/* element type of the cores of an sgtt_tt */
#define SGTT_DTYPE_F64 0

/* A tensor train with three cores in device memory (caller-owned buffers).
 *   core1: n1 x r1, row-major, leading dimension r1     (n1 * cap1 doubles)
 *   core2: r1 x n2 x r2, row-major [a][i][b]            (cap1 * n2 * cap2)
 *   core3: n3 x r2, row-major (node-major), ld r2       (n3 * cap2 doubles)
 * core3 is the transpose of the paper's third core (eq. 4.2): row = space
 * index, so that sparse products over space read contiguous rank vectors.
 * r1, r2 are the live ranks: inputs read them, outputs write them.
 * The cores must be device, managed or pinned host memory (as
 * hipPointerGetAttributes reports it); any other pointer is refused with
 * SGTT_E_INVALID before a kernel runs.
 * dtype: element type of the cores.  The boundary exchanges FP64 tensor
 *   trains only (SGTT_DTYPE_F64); any other value is refused with
 *   SGTT_E_INVALID.  Reduced-precision copies (precision options of
 *   sgtt_solve_opts) live inside the library.
 * d_ranks: optional device pointer to 2 ints (NULL: none), caller-owned;
 *   memory HIP does not know (e.g. plain host memory) is refused with
 *   SGTT_E_INVALID before anything is written.
 *   Every call that writes this TT as an output also stores (r1, r2) there,
 *   ordered on the context stream after the cores, so that work queued
 *   later on that stream can read the live ranks from device memory without
 *   a host round trip.  Inputs are always read from r1, r2 above, never
 *   from d_ranks. */
typedef struct {
  int n1, n2, n3;
  int r1, r2;
  int cap1, cap2;
  double* core1;
  double* core2;
  double* core3;
  int dtype;
  int* d_ranks;
} sgtt_tt;

/* velocity TT (n3 = n_u) and pressure TT (n3 = n_p) of one all-at-once vector */
typedef struct {
  sgtt_tt u;
  sgtt_tt p;
} sgtt_tt_pair;

/* Problem description (sec. 6.1).  Viscosity law 0: nu0 (1 + nu_coef
 * sum_k xi_k/k^2), xi_k ~ U[-1,1]; law 1: the paper's truncated KL expansion
 * nu0 (1 + nu_coef sum_k sqrt(beta_k) a_k(x) xi_k) of the covariance
 * exp(-||x - y||_1 / corr_length), xi_k ~ U[-sqrt 3, sqrt 3] (sec. 6.1, its
 * m + 1 distinct stiffness matrices in eq. 3.6; meshes up to h = 1/8).
 * Legendre chaos of total degree <= p in m variables. */
typedef struct {
  double h;          /* mesh size: 1/h even integer                         */
  double L;          /* channel length (12 in the paper)                    */
  int m;             /* number of random variables                          */
  int p;             /* total chaos degree                                  */
  int nt;            /* time steps                                          */
  double tau;        /* time step                                           */
  double nu0;        /* mean viscosity                                      */
  double nu_coef;    /* relative amplitude of the viscosity expansion       */
  double ramp;       /* inflow ramp rate: u_D = (1-4 x2^2)(1-exp(-ramp t))  */
  double eps_conv;   /* truncation of the convection field (eq. 4.13)       */
  double eps_rhs;    /* truncation of a Picard residual right-hand side     */
  int viscosity_law; /* 0 or 1, see above                                   */
  double corr_length;/* KL correlation length b (law 1)                     */
} sgtt_problem_desc;

typedef struct {
  int n_s, n_u, n_p, n_xi, nt, n_all;
  int conv_r1, conv_r2;   /* ranks of the convection field w~ (0 for Stokes) */
  int rhs_r1u, rhs_r2u, rhs_r1p, rhs_r2p;
  double setup_seconds;
  double rhs_norm;     /* ||f|| (Stokes) or the norm of the untruncated
                          nonlinear residual of the prior iterate (Picard) */
} sgtt_system_info;

typedef struct {
  double tol;          /* exact relative residual target (1e-8)             */
  double eps_krylov;   /* truncation of Krylov vectors (1e-6)               */
  double tol_cycle;    /* relative tolerance of one flexible GMRES cycle    */
  int restart;         /* iterations per cycle                              */
  int max_cycles;      /* refinement cycles                                 */
  double inner_tol;    /* mean-matrix inner solve tolerance (1e-1)          */
  double inner_eps;    /* truncation inside the inner solve (1e-3)          */
  int inner_maxit;     /* inner iterations                                  */
  int verbose;         /* 1: per-iteration line on stderr                   */
  int outer_explicit;  /* 1: Alg. 4.2 literally, z_k and s_k = T(b - L z_k)
                          every outer iteration; 0: stop a cycle on the
                          least-squares residual estimate, form z at its end */
  int inner_explicit;  /* same choice for the inner mean-matrix solve       */
  int relax;           /* 0: fixed eps_krylov (Alg. 4.2); 1: truncate the
                          k-th Krylov vectors with eps_krylov ||b||/||r_k-1||
                          (capped at 1e-2), an inexact-Krylov relaxation    */
  int precision;       /* arithmetic of the velocity block of the
                          preconditioner: 0 FP64.  inner_mode 0: 1 FP32 and 2
                          BF16 operands on the matrix cores with FP32
                          accumulation for the dense products of the inner
                          solve (eq. 5.22-5.23).  inner_mode 1: 1 or 2 run
                          the time-stepped mean solve in FP32 (full tensor,
                          mass products and block cyclic reduction passes in
                          FP32 on the matrix cores, FP32 accumulation; its
                          TT-SVD in FP64).  The outer iteration, operator,
                          truncation eigen-solves, Hessenberg least squares
                          and the exact residual stay FP64, so the flexible
                          outer solve and the refinement still reach tol.
                          3 (relaxed): the velocity block runs in FP32 (as
                          with 1) only in the outer iterations whose
                          residual, relative to the right-hand side of the
                          whole solve, is at most 0.05 tol / 1e-5 (1e-5
                          bounds the FP32 mean solve's relative error), in
                          FP64 before; so the FP32 error an application adds
                          to the solution stays below what the refinement
                          cycle's right-hand side is compressed at, and
                          does not raise its ranks.  Outside sgtt_solve
                          (sgtt_precondition) 3 means FP64                   */
  double inner_rhs_eps;    /* truncation of the inner solve's right-hand side
                              (0: inner_eps); the inner solve only has to
                              reach inner_tol                              */
  double cycle_rhs_factor; /* a refinement cycle's right-hand side r_j is
                              compressed at max(eps_krylov, min(1e-3,
                              factor tol ||b|| / ||r_j||)); 0 means 0.05    */
  int inner_mode;          /* velocity block of the preconditioner:
                              0: inner low-rank GMRES on (F_0 + C) with M
                                 (eq. 5.22-5.23);
                              1: block forward substitution in time on the
                                 full velocity tensor with F_avg (eq. 5.23)
                                 on the diagonal and -tau^-1 M below, then
                                 TT-SVD at inner_eps: (F_0 + C)^-1 exactly
                                 without convection; with convection the
                                 time-averaged convection of F_avg stands
                                 for N_0 (an approximation, as is M);
                              2: M^-1 of eq. 5.23 applied once in place of
                                 the inner solve (prefix sum in time on
                                 core 1, one F_avg solve of the core-3
                                 columns), then truncation at inner_eps   */
  int schur;               /* Schur complement approximation of the
                              preconditioner: 0 mean-based LSC (eq. 5.19);
                              1 mean-based PCD (eq. 5.17) with the Q1
                              pressure-space mass, stiffness and mean
                              convection (natural boundary conditions)    */
  int graph;               /* 1: inner_mode 1 runs the time loop of its mean
                              solve (a mass product and a block cyclic
                              reduction solve per time step) as one HIP
                              graph launch, captured once per system and
                              arithmetic on two full-tensor buffers the
                              system allocates on first use and keeps (2 n_t
                              n_xi n_u doubles); until the spatial solve's
                              kernel choices are tuned, the loop runs as
                              plain launches; the results are those of the
                              plain launches; inner modes 0 and 2 ignore
                              it.  0: plain launches                      */
} sgtt_solve_opts;

typedef struct {
  int cycles, outer_iters, inner_iters;
  double rel_residual;       /* exact ||b - L x|| / ||b|| at return          */
  double seconds;
  int max_rank_krylov_u, max_rank_krylov_p;
  int roundings;
  double t_apply, t_round, t_precond, t_residual;   /* seconds by phase     */
  int learned_calls;         /* mean solves done by an attached network      */
  int learned_fallback;      /* 1 if the solve switched back to the exact one */
  long device_allocs;        /* device allocations (hipMalloc) made during the
                                solve: 0 once the context's reservation
                                (sgtt_context_reserve) covers its working set
                                and the spatial-solve kernel choices for its
                                column counts are tuned                     */
  int f32_applications;      /* precision 3: preconditioner applications whose
                                velocity block ran in FP32                  */
  long graph_launches;       /* graph option: mean-solve time loops run as a
                                graph launch                                */
} sgtt_solve_stats;

/* ------------------------------------------------------------- context */
/* One device, one stream.  hip_stream may be NULL (the library creates a
 * default-priority stream) or an existing hipStream_t (e.g. torch's).
 * Calls are ordered on that stream.  Inside a solve, the pressure TT of a
 * vector pair is rounded on a second, default-priority stream driven by a
 * second host thread of the context (created on first use, with its own
 * memory pool), forked from and joined back into the context's stream; the
 * results are the same as rounding both on one stream.  The environment
 * variable SGTT_SIDE_LANE=0 at context creation keeps both on the calling
 * thread and stream. */
int sgtt_context_create(int device, void* hip_stream, sgtt_context** out);
/* Ends the caller's use of the context.  Systems and networks made on it
 * keep it alive: when any remain, its memory, threads and (own) stream are
 * released with the last of them, in any order of destruction. */
int sgtt_context_destroy(sgtt_context* ctx);
/* Device memory of a context.  The library takes temporaries from a
 * stream-ordered caching pool.  sgtt_context_reserve allocates an arena of
 * `bytes` up front (and the largest split-K workspace of the context's
 * stream): later temporaries are carved out of it while it suffices, so a
 * solve whose working set fits allocates no device memory (what callers
 * that must not allocate inside a solve need; the peak of an earlier solve
 * of the same system, from sgtt_context_memory, is a size that fits).
 * Fails with SGTT_E_INVALID while temporaries of an earlier arena are in use,
 * SGTT_E_OOM if the arena cannot be allocated; bytes = 0 drops the arena. */
typedef struct {
  size_t arena_bytes;       /* reserved arena                                 */
  size_t arena_peak_bytes;  /* most of it in use at once since the reserve    */
  size_t cached_bytes;      /* blocks allocated outside the arena (cached)    */
  long device_allocs;       /* hipMalloc calls of the context's pool so far   */
} sgtt_memory_info;
int sgtt_context_reserve(sgtt_context* ctx, size_t bytes);
int sgtt_context_memory(const sgtt_context* ctx, sgtt_memory_info* out);
/* last error of the context; with ctx == NULL, the last failed context creation */
const char* sgtt_last_error(const sgtt_context* ctx);
/* build identification string (static storage) */
const char* sgtt_version(void);
/* sizeof of the public structs, in this order: sgtt_tt, sgtt_tt_pair,
 * sgtt_problem_desc, sgtt_system_info, sgtt_solve_opts, sgtt_solve_stats,
 * sgtt_memory_info, sgtt_picard_opts, sgtt_picard_stats, sgtt_iter_record;
 * the first min(n, 10) go to sizes.  Returns the number of structs (10).
 * For bindings
 * that mirror the structs (host only, no device call). */
int sgtt_abi_sizes(long* sizes, int n);

/* ------------------------------------------------------------- system */
/* Assemble the Picard-step system eq. 3.14: operator L(w~) with
 * w~ = T_eps_conv(w) (eq. 4.13), right-hand side r = f - L(w)[w; p_w]
 * (eq. 3.15) truncated with eps_rhs, preconditioner factorizations
 * (eq. 5.19, 5.23).  prior = NULL gives the Stokes system (N = 0, r = f).
 * Host setup runs on the CPU; device data are uploaded on the context
 * stream.  The system owns its workspace until sgtt_system_destroy. */
int sgtt_assemble(sgtt_context* ctx, const sgtt_problem_desc* desc, const sgtt_tt_pair* prior,
                  sgtt_system** out);
int sgtt_system_destroy(sgtt_system* sys);
int sgtt_system_info_get(const sgtt_system* sys, sgtt_system_info* info);

/* Write the right-hand side of the system into caller buffers b: for the
 * Stokes system the lifted Dirichlet data f (sec. 3.2 with the inflow of
 * eq. 6.1; exact TT of ranks <= 2), for a Picard step the nonlinear residual
 * r = f - L(w)[w; p_w] of eq. 3.15 (the untruncated prior, sec. 4.3),
 * truncated with desc->eps_rhs.  Capacities of b are checked
 * (SGTT_E_RANK_CAP, b unchanged); ranks are written to b. */
int sgtt_rhs(sgtt_system* sys, sgtt_tt_pair* b);

/* y = L x (eq. 3.11-3.12 with eq. 4.4 and eq. 4.12), exact when eps == 0,
 * else followed by T_eps on u and p separately. */
int sgtt_apply(sgtt_system* sys, const sgtt_tt_pair* x, sgtt_tt_pair* y, double eps);

/* z = P^-1 r for the mean-based LSC block-triangular preconditioner
 * (eq. 5.2, 5.19, 5.22-5.23).  opts supplies eps_krylov and the inner solve
 * parameters; NULL uses defaults.  stats (may be NULL) gets the inner
 * iteration count (inner_iters) of this application; its other fields are
 * zero. */
int sgtt_precondition(sgtt_system* sys, const sgtt_tt_pair* r, sgtt_tt_pair* z,
                      const sgtt_solve_opts* opts, sgtt_solve_stats* stats);

/* Spatial solves of the preconditioner on the device, by block cyclic
 * reduction: which = 0 solves F_avg v = b (eq. 5.23; both velocity
 * components, 2 n_s rows, component 2 after component 1), which = 1 solves
 * X q = b with X = B M*^-1 B^T (eq. 5.19; n_p rows).  b and x are device
 * buffers owned by the caller, row-major with ncols columns (ld = ncols);
 * b is not modified.  variant = -1 uses the tuned kernel choice of every
 * pass; 0 <= variant < sgtt_bcr_variant_count() runs every pass with that
 * kernel variant (SGTT_E_INVALID if it does not take the factor's block
 * size).  Runs on the context's stream and waits for it. */
int sgtt_bcr_apply(sgtt_system* sys, int which, int variant, int ncols, const double* b, double* x);
int sgtt_bcr_variant_count(void);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * spatial solve as sgtt_bcr_apply, allocating nothing.  The reduction's
 * working copy of b lives in a fixed device array that the library holds on
 * every GPU it runs on until the process ends, of
 * SGTT_NOALLOC_SCRATCH_DOUBLES doubles (32 MiB): it takes
 * ncomp * rows * ncols <= SGTT_NOALLOC_SCRATCH_DOUBLES (ncomp = 2 for
 * which = 0, else 1; rows = n_s or n_p), else SGTT_E_INVALID with nothing
 * launched.  variant >= 0 runs that kernel variant in every pass; -1 takes
 * the choice an earlier sgtt_bcr_apply or solve tuned for this column count
 * (power-of-two bucket), else the first variant that takes the blocks: no
 * timing runs.  Stream-ordered on the context's stream and does NOT wait for
 * it (the caller synchronizes before reading x).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other contexts or
 * streams, other threads) race.  Each call overwrites the part of the array
 * it uses before reading it. */
#define SGTT_NOALLOC_SCRATCH_DOUBLES (4 * 1024 * 1024)
int sgtt_bcr_apply_noalloc(sgtt_system* sys, int which, int variant, int ncols, const double* b, double* x);

/* In-place truncation T_eps (eq. 4.5-4.7): ||round(x) - x|| <= eps ||x||
 * (up to the accuracy of FP64 Gram matrices, about 1e-8 relative).  If a
 * rank would exceed max_rank (> 0; 0 means 4096) or the capacity of x, the
 * call fails with SGTT_E_RANK_CAP.  The first rank is at most 512.  A second
 * rank above 96 is truncated by a blocked pivoted Cholesky of the Gram
 * matrix with a skeleton (interpolative) factor: the bound above still
 * holds, core 2 is then not orthonormal. */
int sgtt_round(sgtt_context* ctx, sgtt_tt* x, double eps, int max_rank);

/* Euclidean inner product of two all-at-once vectors over all free (time,
 * chaos, space) coefficients, <x, y> = <x.u, y.u> + <x.p, y.p> (the norm of
 * the residual and the Gram-Schmidt products of Alg. 4.2), computed from the
 * cores by contraction over the TT modes (sec. 4.1, eq. 4.4 applied to the
 * identity), never expanding the tensors.  x and y must have the same mode
 * sizes (SGTT_E_INVALID otherwise); ranks may differ.  Result to host memory
 * (synchronizes the context stream); SGTT_E_NONFINITE for a NaN/Inf result. */
int sgtt_dot(sgtt_context* ctx, const sgtt_tt_pair* x, const sgtt_tt_pair* y, double* out);

/* y = alpha x + beta y as an exact TT by core concatenation (sec. 4.1: the
 * ranks of a sum add, and the sum is not truncated; Alg. 4.2 rounds such
 * sums with sgtt_round).  Core 1 of the result is [alpha X1, beta Y1], core 2
 * is block diagonal, core 3 is [X3, Y3] (in the layout of sgtt_tt).  The
 * result ranks (x.r1 + y.r1, x.r2 + y.r2) must fit y's capacities, else
 * SGTT_E_RANK_CAP with y unchanged; mode sizes must match (SGTT_E_INVALID).
 * y is overwritten on success (its ranks updated). */
int sgtt_axpby(sgtt_context* ctx, double alpha, const sgtt_tt_pair* x, double beta, sgtt_tt_pair* y);

/* Solve L x = b (Alg. 4.2 with refinement to an exact relative residual).
 * x is output only (z_0 = 0).  opts = NULL uses defaults.  Returns
 * SGTT_W_NOT_CONVERGED with the best iterate in x when max_cycles run out,
 * SGTT_E_NONFINITE (x untouched) for a right-hand side with a NaN or Inf,
 * checked before any rounding, or for a non-finite residual later. */
int sgtt_solve(sgtt_system* sys, const sgtt_tt_pair* b, sgtt_tt_pair* x, const sgtt_solve_opts* opts,
               sgtt_solve_stats* stats);

/* Solve n independent systems (b[i], x[i] as in sgtt_solve).  Systems
 * assembled on different contexts run concurrently (one host worker per
 * context driving that context's stream; the streams share the device);
 * systems on the same context run in order.  status[i] gets each solve's
 * return code and stats[i] (may be NULL) its statistics.  Returns the worst
 * status, or SGTT_E_INVALID if any solve failed (see status[i] and
 * sgtt_last_error of that system's context).  A context must not be used by
 * other calls while the batch runs.  With more than one context the solves
 * of the batch run without the contexts' side lanes (second streams and
 * host threads), whose work would queue behind the other contexts' streams
 * on the process's few hardware queues; results are the same. */
int sgtt_solve_batched(sgtt_system* const* systems, int n, const sgtt_tt_pair* const* b,
                       sgtt_tt_pair* const* x, const sgtt_solve_opts* opts, sgtt_solve_stats* stats,
                       int* status);

/* ------------------------------------------------------------- Picard */
#define SGTT_PICARD_MAX_STEPS 16

typedef struct {
  int max_steps;          /* Picard steps after the Stokes solve (Alg. 3.1, maxit) */
  double tol_picard;      /* stop when ||r^(i)|| <= tol_picard ||f|| (Alg. 3.1)    */
  double eps_soln;        /* truncation of the updated iterates (eq. 4.8); 0 keeps  */
                          /* u^(i-1) + du as the exact sum (ranks add)            */
  sgtt_solve_opts solve;  /* options of every linear solve                        */
  int update_mode;        /* 0: u^(i) = T_eps_soln(u^(i-1) + du) (eq. 4.8);        */
                          /* 1: u^(i) = u^(i-1) + T_eps_soln(du), the update       */
                          /* truncated relative to its own norm and the sum kept   */
                          /* exact (ranks add; see sgtt_picard)                    */
} sgtt_picard_opts;

typedef struct {
  int steps;                                            /* Picard steps taken     */
  double nonlinear_residual[SGTT_PICARD_MAX_STEPS + 1]; /* ||r^(i)|| / ||f||      */
  double linear_residual[SGTT_PICARD_MAX_STEPS + 1];    /* solve i (0 = Stokes)   */
  int outer_iters[SGTT_PICARD_MAX_STEPS + 1];
  int inner_iters[SGTT_PICARD_MAX_STEPS + 1];
  double solve_seconds[SGTT_PICARD_MAX_STEPS + 1];
  double assemble_seconds[SGTT_PICARD_MAX_STEPS + 2];
  int rank_u[SGTT_PICARD_MAX_STEPS + 1][2];             /* iterate ranks after    */
  int rank_p[SGTT_PICARD_MAX_STEPS + 1][2];             /* solve i and eq. 4.8    */
  double seconds;
  /* ranks of the iterate as stored: equal to rank_u / rank_p with
   * update_mode 0; with update_mode 1 the exact sum's ranks, while rank_u /
   * rank_p give the ranks of that sum rounded at eps_soln */
  int stored_rank_u[SGTT_PICARD_MAX_STEPS + 1][2];
  int stored_rank_p[SGTT_PICARD_MAX_STEPS + 1][2];
} sgtt_picard_stats;

/* Picard's method (Alg. 3.1) with the low-rank variant of sec. 4.3: the
 * Stokes solve gives u^(0), p^(0); each step assembles the system with the
 * convection of w~ = T_eps_conv(u^(i-1)) (eq. 4.13), takes the nonlinear
 * residual r^(i-1) = f - L(u^(i-1)) [u^(i-1); p^(i-1)] of the untruncated
 * iterate (truncated at desc->eps_rhs for the right-hand side), solves for
 * (du, dp) with opts->solve, and sets u^(i) = T_eps_soln(u^(i-1) + du),
 * p^(i) likewise (eq. 4.8).  The rounding is Gram-based, so its result is
 * accurate to about sqrt(machine epsilon) ||u|| whatever eps_soln asks; the
 * residual of such an error stalls the nonlinear residual near 1e-5 ||f||
 * on the step-domain problems.  update_mode 1 truncates the update alone
 * (error eps_soln ||du||) and keeps the sum exact, so the iterate's ranks
 * grow by the update's at every step.  Stops when ||r^(i)|| <= tol_picard ||f|| or
 * after max_steps (<= SGTT_PICARD_MAX_STEPS) steps; the residual of the
 * returned iterate is always evaluated (nonlinear_residual[steps]).  x:
 * caller buffers for the last iterate (capacity checked).  Returns
 * SGTT_W_NOT_CONVERGED if a linear solve missed its tolerance. */
int sgtt_picard(sgtt_context* ctx, const sgtt_problem_desc* desc, const sgtt_picard_opts* opts,
                sgtt_tt_pair* x, sgtt_picard_stats* stats);

/* ------------------------------------------------------------- dense products */
/* C = alpha A B + beta C in FP64 with the library's product kernels (the
 * ones the TT cores, Grams, projections and full-tensor expansions use):
 * row-major device matrices, A m x k (leading dimension lda >= k), B k x n
 * (ldb >= n), C m x n (ldc >= n).  m, n >= 1, k >= 0 (A and B may be NULL
 * for k = 0, which scales C by beta); SGTT_E_INVALID otherwise.  Stream-ordered on the context stream; synchronizes.  For
 * checks of the kernels against a reference product. */
int sgtt_gemm(sgtt_context* ctx, int m, int n, int k, double alpha, const double* A, long lda, const double* B,
              long ldb, double beta, double* C, long ldc);

/* ------------------------------------------------------------- solve history */
/* One record per outer FGMRES iteration of the last sgtt_solve on a system
 * (iter = 1, 2, ... within refinement cycle `cycle`), and one closing each
 * refinement cycle (iter = -1).  For an iteration, rel is the relative
 * residual of the cycle's correction system (the explicit one when
 * outer_explicit is set, else the Hessenberg estimate of Alg. 4.2), rank_v
 * the (r1, r2) of the newest Krylov vector of each component, rank_z those
 * of the cycle's current solution (explicit residuals only, else 0).  For a
 * cycle's end, rel is the exact ||b - L x|| / ||b|| of the accumulated
 * solution and rank_z its ranks.  seconds: since the solve began. */
typedef struct {
  int cycle, iter;
  double rel;
  int rank_v_u[2], rank_v_p[2];
  int rank_z_u[2], rank_z_p[2];
  double seconds;
} sgtt_iter_record;
/* Copies the first min(max_records, n) records to out; *nrecords gets n. */
int sgtt_solve_history(const sgtt_system* sys, int max_records, sgtt_iter_record* out, int* nrecords);

/* ------------------------------------------------------------- checkpoints */
/* The Picard iterate (Alg. 3.1) is the natural restart point of a nonlinear
 * solve; it is small (eq. 6.6).  A checkpoint file holds one TT pair: a
 * magic tag, a format version, the sizes and ranks (n1, n2, n3, r1, r2 of
 * the velocity TT, then of the pressure TT), the six cores in the layout of
 * sgtt_tt with the live ranks as leading dimensions, as little-endian
 * float64, and a 64-bit FNV-1a hash of all of it.  Files are written to
 * "<path>.tmp" and renamed, so a failed write leaves no torn file behind.
 *
 * sgtt_pair_save: copies x's live cores to the host (synchronizes the
 * context stream) and writes them.  SGTT_E_IO if the file cannot be
 * written.
 * sgtt_pair_load: reads a file into x's buffers (sizes must match x's n1,
 * n2, n3: SGTT_E_INVALID; ranks above x's capacities: SGTT_E_RANK_CAP;
 * missing, damaged or foreign files: SGTT_E_IO) and sets x's ranks; x is
 * unchanged unless the call returns SGTT_OK.  Synchronizes. */
int sgtt_pair_save(sgtt_context* ctx, const sgtt_tt_pair* x, const char* path);
int sgtt_pair_load(sgtt_context* ctx, const char* path, sgtt_tt_pair* x);
/* Host-only forms (no device call): dims[10] = n1, n2, n3, r1, r2 of the
 * velocity TT then of the pressure TT; cores[6] = core 1, 2, 3 of each,
 * compact, in host memory.  sgtt_pair_file_info reads the dims of a file
 * (header checked, the hash is not); sgtt_pair_file_read_host reads into
 * host buffers whose sizes caps[10] = n1, n2, n3, cap1, cap2 per TT give,
 * with the checks of sgtt_pair_load, and writes the file's dims. */
int sgtt_pair_file_write_host(const char* path, const int* dims, const double* const* cores);
int sgtt_pair_file_info(const char* path, int* dims);
int sgtt_pair_file_read_host(const char* path, const int* caps, double* const* cores, int* dims);

/* Exact ||b - L x|| / ||b|| evaluated in full format on the device
 * (synchronizes; result to host). */
int sgtt_residual(sgtt_system* sys, const sgtt_tt_pair* b, const sgtt_tt_pair* x, double* rel);

/* The same exact residual r = b - L x, also written out in full format:
 * ru (device, n_t * n_xi * n_u doubles) and rp (device, n_t * n_xi * n_p),
 * C order (time slowest, space fastest; eq. 4.1), caller-owned.  *rel gets
 * ||r|| / ||b||.  For checking a solve at sizes where a full tensor still
 * fits in HBM (2 GB per velocity tensor at the 64 x 192 grid). */
int sgtt_residual_tensor(sgtt_system* sys, const sgtt_tt_pair* b, const sgtt_tt_pair* x, double* ru,
                         double* rp, double* rel);

/* Expand a TT to the full tensor out (n1*n2*n3 doubles, device, C order). */
int sgtt_expand(sgtt_context* ctx, const sgtt_tt* x, double* out);

/* Least squares argmin_y || beta e1 - H y || for the (k+1) x k upper
 * Hessenberg matrix H (host, column-major, leading dimension k+1), solved by
 * Givens rotations on the device (Alg. 4.2, line 12).  y: host, length k. */
int sgtt_hessenberg_lsq(sgtt_context* ctx, const double* H, int k, double beta, double* y,
                        double* resid);

/* ------------------------------------------------ learned mean solve
 * A correction of the mean spatial solve used inside the inner
 * preconditioner M^-1 = (I - C)^-1 (x) I (x) F_avg^-1 (eq. 5.23).  The
 * paper's inner solve only needs to be approximate (sec. 5.2) and the outer
 * solve is flexible (sec. 4.2), so F_avg^-1 may be replaced there by
 *     z = D^-1 r + ||r|| MLP(r / ||r||),   D = diag(F_avg),
 * applied to every spatial column (each velocity component separately).
 * MLP: n -> width -> width -> n with ReLU; weights FP16, activations and
 * accumulation FP32 on the matrix cores; trained on the device with Adam on
 * FP32 masters, minimizing the mean relative squared error against the
 * exact correction (F_avg^-1 r - D^-1 r) / ||r|| over pairs that the solver
 * records from its own exact mean solves.  The exact solve remains the
 * fallback: after two inner solves that miss their tolerance with the
 * network, the rest of that solve uses the exact one (learned_fallback). */
typedef struct sgtt_mlp sgtt_mlp;

/* n = spatial size of one component (n_s of the system), capacity = pairs
 * that can be recorded (2 per velocity column of a mean solve). */
int sgtt_mlp_create(sgtt_context* ctx, int n, int width, long capacity, unsigned seed, sgtt_mlp** out);
int sgtt_mlp_destroy(sgtt_mlp* mlp);   /* SGTT_E_INVALID while a system refers to it */
/* number of parameters (W1 w x n, b1 w, W2 w x w, b2 w, W3 n x w, b3 n, in
 * this order, row-major) and of recorded pairs */
int sgtt_mlp_size(const sgtt_mlp* mlp, long* nparam, long* npairs);
/* host FP32 parameter vectors in the order above (set rounds the working
 * weights to FP16 and resets the optimizer state) */
int sgtt_mlp_set_params(sgtt_mlp* mlp, const float* host);
int sgtt_mlp_get_params(sgtt_mlp* mlp, float* host);
/* Parameter files of a trained network (a learned correction is trained once
 * and reused): magic tag, version, n, width, nparam, the FP32 parameters in
 * the order above, an FNV-1a hash; written under a temporary name and
 * renamed.  sgtt_mlp_load checks the shape (SGTT_E_INVALID for a network of
 * another n or width) and the hash (SGTT_E_IO, also for a missing, cut or
 * foreign file) before it changes the network; it then sets the parameters
 * as sgtt_mlp_set_params does.  Host-only forms need no context:
 * sgtt_mlp_file_info reads the header (hash not checked),
 * sgtt_mlp_file_read_host reads the parameters of a network of the given
 * shape into host memory (unchanged on error). */
int sgtt_mlp_save(sgtt_mlp* mlp, const char* path);
int sgtt_mlp_load(sgtt_mlp* mlp, const char* path);
int sgtt_mlp_file_write_host(const char* path, int n, int width, const float* params);
int sgtt_mlp_file_info(const char* path, int* n, int* width, long* nparam);
int sgtt_mlp_file_read_host(const char* path, int n, int width, float* params);
/* y = MLP(x) for batch host columns (column s at x + s*n): FP16 weights
 * widened to FP32 against FP32 activations on the FP32 matrix cores (the
 * form training differentiates) */
int sgtt_mlp_forward(sgtt_mlp* mlp, const float* x, int batch, float* y);
/* the same with every product on the FP16 matrix cores: inputs and hidden
 * activations rounded to FP16, FP32 accumulation (the form the correction
 * takes inside the preconditioner, where each right-hand side column is
 * scaled to unit norm before rounding) */
int sgtt_mlp_forward_f16(sgtt_mlp* mlp, const float* x, int batch, float* y);
/* loss (mean relative squared error) and its gradient (host, nparam floats,
 * may be NULL) for host inputs x and targets t */
int sgtt_mlp_loss_grad(sgtt_mlp* mlp, const float* x, const float* t, int batch, double* loss, float* grad);
/* append host training pairs (x_s, t_s at x + s*n, t + s*n) while capacity
 * lasts; *added gets how many were stored */
int sgtt_mlp_add_pairs(sgtt_mlp* mlp, const float* x, const float* t, long count, long* added);
/* steps Adam minibatches of batch recorded pairs (uniform with replacement,
 * seeded; batch >= the number of pairs uses all pairs in order every step);
 * losses: host array of steps values or NULL */
int sgtt_mlp_train(sgtt_mlp* mlp, int steps, int batch, double lr, unsigned seed, double* losses);
/* record (r, F_avg^-1 r) pairs from this system's exact mean solves during
 * later solves (NULL stops recording); network and system must share the
 * context and the spatial size */
int sgtt_mlp_collect(sgtt_system* sys, sgtt_mlp* mlp);
/* use the network for the mean solves of this system (NULL: exact solve)
 * Ownership: a system refers to the network it collects for or uses; it does
 * not own it.  sgtt_mlp_destroy fails with SGTT_E_INVALID (network kept)
 * while any system still refers to it; detaching (NULL) or destroying the
 * system releases the reference. */
int sgtt_mlp_attach(sgtt_system* sys, sgtt_mlp* mlp);

/* ------------------------------------------------------------- profiling */
/* Per-launch timing of the library's kernels with HIP events recorded on the
 * context stream (process-wide switch; enabling clears earlier records).
 * Adds two event records per launch while enabled. */
int sgtt_profile_enable(sgtt_context* ctx, int enable);
/* The same switch restricted to the kernel classes whose bit is set in
 * class_mask (bit c = class id c; 0 turns profiling off), so that a timed
 * run pays the event records of the classes it reports only. */
int sgtt_profile_enable_classes(sgtt_context* ctx, unsigned class_mask);
/* Sampling of the event scopes: of the scopes of each class opened since
 * this call (or since profiling was last enabled), the 1st, (period+1)th,
 * (2 period+1)th ... are recorded; the others run without events.  A scope
 * brackets one launch, or one spatial solve's passes for the block cyclic
 * reduction.  period 1 (the default) records every scope; period < 1 is
 * SGTT_E_INVALID.  The sums of sgtt_profile_read then cover the sampled
 * scopes only, so their ratios (bytes or flops per second, seconds per
 * launch) stay averages over the run while the event records cost 1/period
 * of what they cost unsampled.  Synchronizes the context stream. */
int sgtt_profile_sample(sgtt_context* ctx, int period);
/* Sums since enabling, per kernel class (index = class id, see
 * sgtt_profile_class_name): event seconds, algorithmic bytes and flops (what
 * each launch's operation must read/write and compute, from its arguments),
 * launch counts.  Arrays of length max_classes; *nclasses gets the number of
 * classes.  Synchronizes the context stream. */
int sgtt_profile_read(sgtt_context* ctx, int max_classes, double* seconds, double* bytes, double* flops,
                      long* launches, int* nclasses);
/* kernel symbol name of a class id (static storage) */
const char* sgtt_profile_class_name(int cls);
/* The same event seconds split by phase of the solve (outer apply, outer
 * Gram-Schmidt, outer solution/residual sums, LSC pressure part, inner
 * right-hand side, inner M^-1, inner apply, inner Gram-Schmidt, inner
 * solution, exact residual, other): seconds[r * max_classes + c] for
 * r < max_regions, c < max_classes.  *nregions gets the number of phases.
 * Synchronizes the context stream. */
int sgtt_profile_read_regions(sgtt_context* ctx, int max_regions, int max_classes, double* seconds,
                              int* nregions);
/* name of a phase id (static storage) */
const char* sgtt_profile_region_name(int region);

/* ------------------------------------------------------------- host setup */
/* Host-only problem setup (no device calls), for inspection and checks:
 * mesh sizes, CSR matrices and chaos matrices. */
int sgtt_host_problem_create(const sgtt_problem_desc* desc, sgtt_host_problem** out);
int sgtt_host_problem_destroy(sgtt_host_problem* hp);
/* sizes[0..5] = n_s, n_u, n_p, n_xi, nt, n_all */
int sgtt_host_sizes(const sgtt_host_problem* hp, int* sizes);
/* CSR export.  which: 0 = M (free x free), 1 = A unit viscosity (free x free),
 * 2 = B (n_p x n_u), 3 = B M*^-1 B^T (n_p x n_p), 4 = B M*^-1 M M*^-1 B^T,
 * 5 = B M*^-1 A M*^-1 B^T, 6 = Q1 pressure mass M_p (n_p x n_p), 7 = Q1
 * pressure stiffness A_p, unit viscosity, natural boundary conditions (the
 * pressure-space matrices of eq. 5.17), 8 + t = the stiffness A_t of the
 * t-th viscous term of eq. 3.6 on the free x free pattern (t < nvisc, see
 * sgtt_host_kl; t = 0 is the unit-viscosity A).  Call with NULL arrays to
 * get nrows/ncols/nnz. */
int sgtt_host_csr(const sgtt_host_problem* hp, int which, int* nrows, int* ncols, int* nnz,
                  int* rowptr, int* col, double* val);
/* chaos: which 0 = G (m+1 x n_xi x n_xi), 1 = H (n_xi^3), 2 = G_nu (n_xi^2),
 * 3 = the chaos matrices of the viscous terms (nvisc x n_xi x n_xi) */
int sgtt_host_gpc(const sgtt_host_problem* hp, int which, double* out);
/* Viscous terms and KL expansion (sec. 6.1): *nvisc gets the number of
 * viscous terms sum_t Gv_t (x) A_t of eq. 3.6 (1 for law 0, m + 1 for the
 * KL law), *nmodes the KL modes (0 for law 0); beta (nmodes) and modes
 * (nmodes x n_p, values at the pressure vertices, int a^2 = 1) may be NULL. */
int sgtt_host_kl(const sgtt_host_problem* hp, int* nmodes, int* nvisc, double* beta, double* modes);
/* Dirichlet lift g over all velocity nodes (2 n_all) and node coordinates
 * (n_all x 2), free node list (n_s) */
int sgtt_host_mesh(const sgtt_host_problem* hp, double* coords, int* free_nodes, double* g_all);
/* Host check of the block cyclic reduction that the spatial solves run on the
 * device (the F_avg solve of eq. 5.23 and the X solve of eq. 5.19): factor
 * which = 0: F = M / tau + nu A on the velocity slabs (n_s rows), or
 * which = 1: X = B M*^-1 B^T on the pressure slabs (n_p rows), and apply its
 * op lists on the host to ncols right-hand sides b (row-major, n x ncols),
 * x = A^-1 b (same layout).  *npass gets the number of passes.  Host memory
 * only; the caller owns b and x.  SGTT_E_INVALID on bad arguments, -6 on a
 * singular block. */
int sgtt_host_bcr_solve(const sgtt_host_problem* hp, int which, double tau, double nu, int ncols, const double* b,
                        double* x, int* npass);

#ifdef __cplusplus
}
#endif
#endif /* SGTT_H */
