// Device kernels for the tensor-train Picard-step solver (gfx950).
// Launch wrappers only; every numeric step of the solve runs in these kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

namespace sgtt {

// ---------------------------------------------------------------- profiling
// Optional per-launch timing with HIP events on the launch stream, with the
// algorithmic bytes / flops of each launch (what the operation must move and
// compute, not what the hardware counted).  Kernel classes:
enum KernelClass {
  KC_GEMM = 0, KC_GEMM_PTR, KC_SPMM, KC_BCR, KC_TRUNC, KC_REDUCE, KC_OTHER, KC_GEMM_LOWP,
  KC_GRAM,   // tall-skinny Gram products (truncations, inner products): k_gemm<0, 1>
  KC_ELL,    // the ELL mass product of the time-stepped mean solve: k_ell_grouped
  KC_PROJ,   // projections of core 3 onto kept ranks (truncations): k_gemm<0, 2>
  KC_COUNT
};
const char* kernel_class_name(int cls);
// hipMalloc calls made by this file's launchers (split-K workspaces, tuning
// copies of the block cyclic reduction) since the process started
long kernel_device_allocs();
// grow the stream's split-K workspace to the largest any launch uses
void splitk_reserve(hipStream_t s);
// frees the split-K workspace of a stream that is about to be destroyed
void splitk_release(hipStream_t s);
// what a gemm() call computes, for the profiler's classes and the kernel's name
enum GemmTag { GEMM_PLAIN = 0, GEMM_GRAM = 1, GEMM_PROJ = 2 };
struct GemmTagScope {
  int old;
  explicit GemmTagScope(int tag);
  ~GemmTagScope();
};
void prof_enable(bool on);
void prof_enable_mask(unsigned class_mask);   // bit c records class c; 0 = off
unsigned prof_mask();                          // classes recorded now (0 when off)
void prof_sample_period(int period);          // record one scope in every `period` per class
bool prof_enabled();
// sums since the last reset: seconds (from events), bytes, flops, launches
void prof_read(double* seconds, double* bytes, double* flops, long* launches);
void prof_reset();
// Phases of the solve that launches are attributed to (prof_region sets the
// current one and returns the previous one).
enum Region {
  RG_OTHER = 0, RG_OUT_APPLY, RG_OUT_MGS, RG_OUT_SOL, RG_LSC, RG_IN_RHS, RG_IN_MINV, RG_IN_APPLY, RG_IN_MGS,
  RG_IN_SOL, RG_RESIDUAL, RG_COUNT
};
const char* region_name(int r);
int prof_region(int r);
// hold: the calling host thread records no profiler scopes (while it
// captures a stream into a graph, where event records would be captured too)
void prof_hold_thread(bool hold);
// seconds[r * KC_COUNT + c] since the last reset
void prof_read_regions(double* seconds);
struct RegionScope {
  int old;
  explicit RegionScope(int r) : old(prof_region(r)) {}
  ~RegionScope() { prof_region(old); }
};

// Arithmetic of the dense products (gemm, gemm_batched, gram): FP64 matrix
// cores, or FP32 / BF16 operands on the matrix cores with FP32 accumulation
// (operands and results stay FP64 in memory).  gemm_precision sets the mode
// for later launches and returns the previous one.
enum GemmPrecision { GP_F64 = 0, GP_F32 = 1, GP_BF16 = 2 };
int gemm_precision(int p);
struct GemmPrecisionScope {
  int old;
  explicit GemmPrecisionScope(int p) : old(gemm_precision(p)) {}
  ~GemmPrecisionScope() { gemm_precision(old); }
};

// C[b](i,j) = alpha * sum_k A[b](i,k) B[b](k,j) + beta * C[b](i,j)
// element (i,k) of A[b] at A + b*sAb + i*sAi + k*sAk (likewise B, C).
// If klimit > 0, batch b only sums k < min(k, klimit - b*kstep) (split-K).
void gemm(hipStream_t s, int batch, int m, int n, int k, double alpha, const double* A, long sAb,
          long sAi, long sAk, const double* B, long sBb, long sBk, long sBj, double beta, double* C,
          long sCb, long sCi, long sCj, int kstep = 0, long klimit = 0);

// Descriptor of one GEMM of a pointer-array batch (same convention as gemm).
struct GemmDesc {
  int m, n, k;
  double alpha, beta;
  const double* A;
  long sAi, sAk;
  const double* B;
  long sBk, sBj;
  double* C;
  long sCi, sCj;
};
// Run nb independent GEMMs described by d_desc (device array of GemmDesc);
// max_m / max_n bound the grid.
void gemm_batched(hipStream_t s, int nb, const GemmDesc* d_desc, int max_m, int max_n);

// out (nx x ny, row-major) = X^T Y over `rows` rows; X(r,i) at X + r*sXr + i*sXc.
// ws: scratch of ws_doubles doubles for split-K partial sums.
void gram(hipStream_t s, long rows, int nx, int ny, const double* X, long sXr, long sXc,
          const double* Y, long sYr, long sYc, double* out, double* ws, size_t ws_doubles);
// Scratch that gram() can use for its partial sums: nx ny doubles per row
// chunk of at least 128 rows, with at most 1024 output tiles of 64 x 64 in
// flight (a larger scratch is never touched).
inline size_t gram_ws_doubles(long rows, int nx, int ny) {
  const long tiles = (long)((nx + 63) / 64) * ((ny + 63) / 64);
  long nch = rows / 128;
  if (nch > 1024 / tiles) nch = 1024 / tiles;
  if (nch < 1) nch = 1;
  return (size_t)nx * ny * nch;
}

// Sum of squares of n doubles into *out (single value, device) -- deterministic.
void sumsq(hipStream_t s, const double* x, long n, double* out, double* ws, size_t ws_doubles);

void fill(hipStream_t s, double* p, long n, double v);
// d[0] = r1, d[1] = r2 (device ints), ordered on s
void store_ranks(hipStream_t s, int* d, int r1, int r2);
// 2-D strided copy with scale: dst[i*ldd + j] = alpha * (*dscale if dscale) * src[i*lds + j]
void copy2d(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst, long ldd,
            double alpha, const double* dscale = nullptr, int dscale_inv = 0);

// dst[j*ldd + i] = src[i*lds + j] for i < rows, j < cols
void transpose_copy(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst, long ldd);
// the same transpose from FP32 to FP64
void transpose_widen(hipStream_t s, int rows, int cols, const float* src, long lds, double* dst, long ldd);
// batch transposes: source b at src + b*sbatch, destination at dst + b*dbatch
// Many independent 2-D block copies in one launch: block z copies a
// rows x cols row-major block, dst[i][j] = a src[i][j] (transpose 0) or
// dst[j][i] = a src[i][j] (transpose 1), with a = alpha, times *dalpha when
// dalpha is set.  The descriptors live in device memory (n of them).
struct BlockCopy {
  const double* src;
  double* dst;
  const double* dalpha;
  long lds, ldd;
  int rows, cols, transpose, pad_;
  double alpha;
};
void block_copy_batched(hipStream_t s, const BlockCopy* d_descs, int n, int max_rows, int max_cols);
void transpose_copy_batched(hipStream_t s, int batch, int rows, int cols, const double* src, long sbatch, long lds,
                            double* dst, long dbatch, long ldd);
void transpose_widen_batched(hipStream_t s, int batch, int rows, int cols, const float* src, long sbatch, long lds,
                             double* dst, long dbatch, long ldd);

// CSR SpMM over the space index with several value arrays sharing a pattern
// and `ncomp` velocity components:
//  y[(c*ocs + r)*ldy + ycol0 + v*yvstep + j] =
//     alpha * sum_t vals[v*vstride + t] * x[(c*ics + col[t])*ldx + xcol0 + j]
//     (+ beta * the old value)
// for rows r < nrows, components c < ncomp, v < nv (<= 16), columns j < ncols.
// max_row_nnz (> 0 when known) bounds the entries of a row; with one value
// array and at most 32 entries a row's loads are all issued at once.
void spmm(hipStream_t s, int nrows, int ncomp, int ics, int ocs, const int* rowptr, const int* col,
          const double* vals, int nv, long vstride, const double* x, int ldx, int xcol0, int ncols,
          double* y, int ldy, int ycol0, int yvstep, double alpha, double beta = 0.0, int max_row_nnz = 0);

// The same product for a square matrix with one value array in padded-row
// (ELL) form: row r has ELL_WIDTH value slots at eval[r * ELL_WIDTH ...], its
// entries first, zeros after them.  The rows are cut into groups of
// consecutive rows (ell_groups_build) whose distinct input rows are staged in
// LDS; rows of the input x are at (c*ics + col)*ldx + xcol0, of y at
// (c*ocs + r)*ldy + ycol0.  y = alpha * A x + beta * y.
constexpr int ELL_WIDTH = 32;
constexpr int ELL_GROUP_ROWS = 16;   // rows per group, at most
constexpr int ELL_GROUP_UMAX = 96;   // distinct input rows per group, at most
constexpr int ELL_CHUNK = 16;        // entries read per step
// Group g covers rows row0[g] .. row0[g+1]-1 and reads input rows
// ucols[uptr[g] .. uptr[g+1]-1] (ascending); lidx[r * ELL_WIDTH + q] is the
// position of row r's q-th entry in its group's list (0 past the entries),
// rlen[r] the row's entry count rounded up to a multiple of ELL_CHUNK.
struct EllGroups {
  int ngroups = 0;
  int umax = 0;                  // largest distinct-row count of a group
  int* row0 = nullptr;           // device, ngroups + 1
  int* uptr = nullptr;           // device, ngroups + 1
  int* ucols = nullptr;          // device
  int* lidx = nullptr;           // device, nrows * ELL_WIDTH
  int* rlen = nullptr;           // device, nrows
};
// host: greedy groups of a CSR pattern (a row joins the current group while
// the group has fewer than ELL_GROUP_ROWS rows and at most ELL_GROUP_UMAX
// distinct columns with it); throws when a row has more than ELL_WIDTH entries
void ell_groups_build(int nrows, const int* rowptr, const int* col, std::vector<int>& row0, std::vector<int>& uptr,
                      std::vector<int>& ucols, std::vector<int>& lidx, std::vector<int>& rlen, int& umax);
void ell_spmm(hipStream_t s, int nrows, int ncomp, int ics, int ocs, const EllGroups& G, const double* eval, long nnz,
              const double* x, int ldx, int xcol0, int ncols, double* y, int ldy, int ycol0, double alpha,
              double beta);
// the same product in FP32 (values, input and output)
void ell_spmm32(hipStream_t s, int nrows, int ncomp, int ics, int ocs, const EllGroups& G, const float* eval,
                long nnz, const float* x, int ldx, int xcol0, int ncols, float* y, int ldy, int ycol0, float alpha,
                float beta);
// C = A B (m x n) with output column j stored at C[i*sCi + (j / csplit)*sCt +
// j % csplit]: a column index (t, xi) of csplit values of xi written as one
// block per t.  gemm_csplit computes at the current product precision,
// gemm_csplit_f32out in FP64 rounded to FP32 on the store.
void gemm_csplit(hipStream_t s, int m, int n, int k, const double* A, long sAi, long sAk, const double* B, long sBk,
                 long sBj, double* C, long sCi, int csplit, long sCt);
void gemm_csplit_f32out(hipStream_t s, int m, int n, int k, const double* A, long sAi, long sAk, const double* B,
                        long sBk, long sBj, float* C, long sCi, int csplit, long sCt);
// C (float, m x n) = A B computed in FP64 on the matrix cores and rounded
// to FP32 on the store (strides as for gemm, batch 1)
void gemm_f32out(hipStream_t s, int m, int n, int k, const double* A, long sAi, long sAk, const double* B, long sBk,
                 long sBj, float* C, long sCi, long sCj);

// core1 block ops on row-major n1 x r matrices
// out[t, col0 + a] = scale*(in[t,a] - in[t-1,a])          (kind 0: (I - C)/tau)
// out[t, col0 + a] = scale*in[t,a] (times *dscale)          (kind 1: copy)
// out[t, col0 + a] = scale*sum_{s<=t} in[s,a]               (kind 2: (I - C)^-1)
void core1_op(hipStream_t s, int kind, int n1, int r, const double* in, int ldi, double* out, int ldo,
              int col0, double scale, const double* dscale = nullptr);
// out[t, col0 + a*r + al] = w[t*ldw + a] * in[t*ldi + al] for a < k
void core1_diag(hipStream_t s, int n1, int r, int k, const double* w, int ldw, const double* in, int ldi,
                double* out, int ldo, int col0);

// core2 block: out[(row0 + a*r1 + al), i, (col0 + b*r2 + be)] =
//   sum_j X_ab(i,j) in[al, j, be]  for a < k1, b < k2, with X_ab at
//   X + (a*k2 + b)*n2*n2 (row-major n2 x n2), or identity if X == nullptr.
// out is R1 x n2 x R2 row-major.
void core2_block(hipStream_t s, int r1, int n2, int r2, const double* in, const double* X, int k1, int k2,
                 double* out, int R1, int R2, int row0, int col0);

// Truncated eigen-decomposition of a symmetric PSD Gram matrix S (N x N
// row-major), following the TT-SVD rank rule, in stages (the full routine
// is trunc_sym in tt_core):
//  trunc_pc: one-workgroup pivoted Cholesky S ~ L L^T (L column-major, ld N)
//    until the remaining trace is <= delta^2 / 16.  delta^2 = eps^2 normsq / 2
//    where normsq = *normsq_in if given, else trace(S) (written to
//    *normsq_out).  *info = 1 when kmax pivots were not enough and kmax <
//    rank_bound (rank capacity exceeded); *info = 2 when more than 96 pivots
//    are needed and large_ok is set (the caller runs the blocked path);
//    without large_ok the pivoted Cholesky subspace (orthonormalized) is the
//    truncation, up to 512 columns, written to U (N x k, ld kmax) with *k_out
//    and the kept trace *kept_out.  A zero matrix gives k = 1, U = e_1.
//    Otherwise *kp_out = kp > 0 pivots for the next stage; *kp_out = 0 when
//    the stage finished the truncation (or *info = 2).  Always state[0..3] =
//    {residual trace, delta^2, zero threshold, trace} (the layout pc_panel
//    uses) and piv_out[j] = the j-th pivot (j < 96), so that after *info = 2
//    the blocked path can resume from the 96 pivots in L and the remaining
//    Schur diagonal in the N doubles after L.  L: scratch N x kmax (+ N).
//    In mode 0 the columns kp .. km-1 of L are zeroed (km = min(96, kmax)).
//  The later stages read kp (and k) from device memory and do nothing when
//  the first stage finished, so the whole chain is queued without a host
//  round trip:
//  trunc_jacobi: for T = L^T L (km x km, ld 96), cyclic Jacobi on its
//    leading kp x kp block, rank k = smallest r >= 1 with discarded
//    eigenvalues + residual <= delta^2, writes *k_out, the kept eigenvalue
//    sum *kept_out and W = V_k diag(lambda^-1/2) (km x km, zero outside
//    kp x k, ld 96), so that L W has orthonormal columns.
//  chol_inv_upper: R = C^-T (km x km, zero outside k x k, ld 96) for the
//    Cholesky factor C of the leading k x k block of G (ld 96): U R has
//    orthonormal columns when G = U^T U; *info = 3 when G is not
//    numerically positive definite.
//  take_basis: U[i][c] = X[i][c] (ld ldx) for c < k when the eigen stage ran.
constexpr int TRUNC_KSMALL = 96;
// Second-bond Grams of at least this order go straight to the blocked
// pivoted Cholesky (panels of pc_panel_width pivots, device-wide Schur
// updates): their ranks mostly exceed TRUNC_KSMALL, and the panels' products
// are shorter than the one-workgroup stage's.
constexpr int TRUNC_BLOCKED_N = 512;
void trunc_pc(hipStream_t s, int N, double* S, double eps, const double* normsq_in, double* normsq_out, double* U,
              int kmax, double* L, int* k_out, double* kept_out, int* info, int rank_bound, int large_ok,
              int* kp_out, double* state, int* piv_out);
void trunc_jacobi(hipStream_t s, int km, const int* kp_dev, const double* T, const double* state, double* W,
                  int* k_out, double* kept_out);
void chol_inv_upper(hipStream_t s, int km, const int* kp_dev, const int* k_dev, const double* G, double* R,
                    int* info);
void take_basis(hipStream_t s, const int* kp_dev, const int* k_dev, int N, const double* X, int ldx, double* U,
                int kmax);

// Blocked pivoted Cholesky of a symmetric PSD Gram matrix S (N x N),
// used when more than 96 pivots are needed.  pc_init: d = diag(S),
// state = {trace, delta^2 = eps^2 normsq / 2, zero threshold}; pc_panel: up
// to nsteps (<= 64) pivots on the current Schur complement into the panel Lp
// (N x nsteps, column-major), out = {pivots taken, finished}.  The caller
// subtracts Lp Lp^T from S between panels (GEMM).
void pc_init(hipStream_t s, int N, const double* S, double eps, const double* normsq_in, double* normsq_out,
             double* d, double* state);
// Panel width of pc_panel for Grams of order N: up to order 4096 the panel
// lives in registers (24 pivots up to 1024, 16 up to 2048, 8 up to 4096);
// beyond, 32-pivot panels run from global memory.
int pc_panel_width(int N);
void pc_panel(hipStream_t s, int N, const double* S, double* d, double* Lp, int* piv, int nsteps, double* state,
              int* out, double* kept);
// Skeleton (interpolative) factor F = L L_P^{-1} of the pivoted Cholesky
// factor L (N x k, column-major), L_P = L[piv, :] lower triangular: then
// S[:, piv] S[piv, piv]^{-1} = F.  F is N x k column-major; LP: k*k scratch.
void skeleton_factor(hipStream_t s, int N, int k, const double* L, const int* piv, double* LP, double* F);
// out[a, :] = in[piv[a], :] for a < k
void gather_rows(hipStream_t s, int k, int cols, const double* in, long ld_in, const int* piv, double* out,
                 long ld_out);

// Stochastic Galerkin convection N(w) w in full format (eq. 3.7, eq. 4.12):
// out[t, i, c*ns + f] += sign * (SG convection of the wind with itself),
// with the wind = ufree (n_t x n_xi x n_u, free dofs [comp1; comp2]) plus the
// Dirichlet lift ramp(t) e_1 gall (gall: 2 n_all).  conn: 9 Q2 nodes per
// element; free_id: node -> free index or -1; H_{ilk} as rows i (hrow,
// hl, hk, hv); ref: reference tables (252 doubles); hh = h / 2.  n_xi <= 64.
void sg_convection_full(hipStream_t s, int nt, int nxi, int n_u, int ns, int nall, int nelem, const int* conn,
                        const int* free_id, const double* ufree, const double* ramp, const double* gall,
                        const int* hrow, const int* hl, const int* hk, const double* hv, const double* ref, double hh,
                        double sign, double* out);

// Block cyclic reduction solve (factor built on the host): device copies of
// the op lists and block data; pass_begin stays on the host.
// One op of a block cyclic reduction pass: output block rows [r0, r0 + bo)
// <- [own rows of B if flags & 1] + sum_t coef[t] * M_t * (rows
// [in_r0[t], in_r0[t] + in_bi[t]) of X if bit t of in_x, else of B), with
// the bo x in_bi[t] block M_t at data + off[t] in matrix-core fragment order
// (bcr_fragment_order); the output goes to X if flags & 2, else to B.
constexpr int BCR_NT = 16;
constexpr int BCR_DATA_PAD = 64 * 64;   // doubles of padding behind the block data
// Element (i, k) of a rows x cols block in fragment order: row tile i / 16,
// k-step k / 4, lane (i % 16) + 16 (k % 4), at ((i/16) nq + k/4) 64 + lane
// with nq = ceil(cols / 4); the tiles are zero-padded.
inline long bcr_fragment_size(int rows, int cols) { return (long)((rows + 15) / 16) * ((cols + 3) / 4) * 64; }
inline long bcr_fragment_index(int i, int k, int cols) {
  return ((long)(i / 16) * ((cols + 3) / 4) + k / 4) * 64 + (i % 16) + 16 * (k % 4);
}
struct BcrOpDesc {
  int r0, bo, nterm, flags;
  int in_r0[BCR_NT];
  int in_bi[BCR_NT];
  int in_x, pad_[3];
  long off[BCR_NT];
  double coef[BCR_NT];
};
// Tuned kernel variant per pass, per (column bucket, components), of one
// factor.  Owned by the factor (shared between copies of its BcrDev), so a
// choice never outlives the factor it was timed on.
struct BcrChoices {
  std::mutex mu;
  std::map<std::pair<int, int>, std::vector<int>> by_key;
};
struct BcrDev {
  int n = 0, nblk = 0, maxbs = 0, npass = 0;
  double ndata = 0;                 // doubles of block data (for the profiler)
  std::vector<int> pass_begin;      // host: ops of pass p are [pass_begin[p], pass_begin[p + 1])
  // host, per pass, for the profiler: sum over ops and terms of rows x cols
  // (flops = 2 * that * columns), doubles of block data, and rows of the
  // right-hand side read or written (times columns)
  std::vector<double> pass_mk, pass_data, pass_rows;
  BcrOpDesc* ops = nullptr;
  double* data = nullptr;
  float* data32 = nullptr;          // the same blocks in FP32 (reduced-precision mean solve)
  std::shared_ptr<BcrChoices> choices = std::make_shared<BcrChoices>();
};
// X <- A^-1 B for ncols columns of ncomp components (rows of one component;
// component z of B at B + z * n * ldb, of X at X + z * n * ldx).  B is
// overwritten (reduced right-hand sides); X must not overlap B.
void bcr_solve(hipStream_t s, const BcrDev& f, int ncomp, double* B, long ldb, double* X, long ldx, int ncols);
// The same solve with one kernel variant for every pass (0 .. count - 1);
// throws when the variant does not take the factor's block size.
int bcr_variant_count();
bool bcr_variant_takes(const BcrDev& f, int variant);
// whether bcr_solve (f32: bcr_solve32) has its pass variants for this
// component and column count already, so that it launches kernels only
bool bcr_is_tuned(const BcrDev& f, int ncomp, int ncols, bool f32);
void bcr_solve_variant(hipStream_t s, const BcrDev& f, int ncomp, double* B, long ldb, double* X, long ldx, int ncols,
                       int variant);
// The same solve in FP32 (blocks data32, right-hand sides and solutions in
// FP32, FP32 accumulation on the matrix cores), kernel variant tuned per pass.
void bcr_solve32(hipStream_t s, const BcrDev& f, int ncomp, float* B, long ldb, float* X, long ldx, int ncols);
// The same solve without timing variants: variant >= 0 for every pass, or
// -1 for the choice an earlier bcr_solve tuned for this column bucket, else
// the first variant that takes the blocks.  Launches only (no allocation).
void bcr_solve_untuned(hipStream_t s, const BcrDev& f, int ncomp, double* B, long ldb, double* X, long ldx, int ncols,
                       int variant);



// Givens least squares for the (k+1) x k Hessenberg H (column-major, ld),
// y = argmin || beta e1 - H y ||; resid = |final rotated rhs entry|.
void hessenberg_lsq(hipStream_t s, const double* H, int ld, int k, const double* beta, double* y,
                    double* resid);

// Modified Gram-Schmidt coefficients from <x, v_i> (d, i < k) and the basis
// Gram matrix GV (ld): h_i = d_i - sum_{j<i} h_j GV[j, i].  Writes h into
// Hcol[0..k-1] and coef[0] = 1, coef[1+i] = -h_i.
void mgs_coef(hipStream_t s, int k, const double* d, const double* GV, int ldg, double* Hcol, double* coef);

// small scalar helpers on device values
// out = sqrt(a + b) (kind 0), out = 1/a (kind 1), out = a * b (kind 2),
// out = a + b (kind 3), out = -a (kind 4), out = sqrt(a) (kind 5)
void scalar_op(hipStream_t s, int kind, const double* a, const double* b, double* out);

// sum_i w[i] * k[i] over n entries -> out (or out += if accumulate)
void dot_reduce(hipStream_t s, long n, const double* w, const double* k, double* out, int accumulate);

// scale n doubles by *dscale (or 1 / *dscale if inv)
void scale_by(hipStream_t s, double* p, long n, const double* dscale, int inv);

// full residual helper: out[i] = a[i] - b[i]
void sub_arrays(hipStream_t s, const double* a, const double* b, double* out, long n);

// check finite: *flag = 1 if any non-finite in x[0..n)
void check_finite(hipStream_t s, const double* x, long n, int* flag);

}  // namespace sgtt
