// Device kernels for the tensor-train Picard-step solver on gfx950.
// See kernels.h for the contract of each launcher.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <stdexcept>
#include <type_traits>
#include <vector>
#include <unordered_map>
#include <utility>

#include "kernels.h"

namespace sgtt {

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRec {
  int cls, region;
  hipEvent_t a, b;
  double bytes, flops;
  long launches;
};
struct Profiler {
  bool on = false;
  unsigned mask = ~0u;   // kernel classes recorded while on
  int period = 1;        // one scope in every `period` of a class is recorded
  long seen[KC_COUNT] = {};
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t ev() {
    if (used == pool.size()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
};
Profiler g_prof;
std::mutex g_prof_mu;
thread_local int g_region = 0;   // per host thread (workers of batched solves)
thread_local bool g_prof_held = false;   // this thread records no scopes (stream capture)

// Brackets launches of one kernel class with HIP events on their stream.
// A scope may cover several dependent launches of the class (launches > 1);
// its time then includes the dispatch gaps between them.
struct ProfScope {
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  double bytes, flops;
  long launches;
  ProfScope(int c, hipStream_t st, double by, double fl, long nl = 1)
      : cls(c), s(st), bytes(by), flops(fl), launches(nl) {
    if (g_prof_held || !g_prof.on || !((g_prof.mask >> c) & 1u)) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof.seen[c]++ % g_prof.period != 0) return;
    a = g_prof.ev();
    (void)hipEventRecord(a, s);
  }
  void add(double by, double fl, long nl) {
    bytes += by;
    flops += fl;
    launches += nl;
  }
  ~ProfScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t b = g_prof.ev();
    (void)hipEventRecord(b, s);
    g_prof.recs.push_back(ProfRec{cls, g_region, a, b, bytes, flops, launches});
  }
};
}  // namespace

const char* kernel_class_name(int cls) {
  static const char* names[] = {"k_gemm", "k_gemm_ptr", "k_spmm", "k_bcr", "k_trunc_eig",
                                "k_reduce_partials", "other", "k_gemm_lowp", "k_gram", "k_ell_spmm", "k_proj"};
  return (cls >= 0 && cls < KC_COUNT) ? names[cls] : "?";
}
const char* region_name(int r) {
  static const char* names[] = {"other",       "outer_apply", "outer_mgs", "outer_solution", "lsc_pressure",
                                "inner_rhs",   "inner_minv",  "inner_apply", "inner_mgs",    "inner_solution",
                                "residual"};
  return (r >= 0 && r < RG_COUNT) ? names[r] : "?";
}
int prof_region(int r) {
  int old = g_region;
  g_region = (r >= 0 && r < RG_COUNT) ? r : 0;
  return old;
}
void prof_hold_thread(bool hold) { g_prof_held = hold; }
void prof_read_regions(double* seconds) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int i = 0; i < RG_COUNT * KC_COUNT; ++i) seconds[i] = 0.0;
  for (auto& r : g_prof.recs) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    seconds[r.region * KC_COUNT + r.cls] += ms * 1e-3;
  }
}
void prof_enable(bool on) { prof_enable_mask(on ? ~0u : 0u); }
void prof_enable_mask(unsigned mask) {
  const bool on = mask != 0;
  if (on) {
    // create the events before the profiled region: creating them while
    // kernels are queued would add host time to what is measured
    std::lock_guard<std::mutex> lk(g_prof_mu);
    constexpr size_t kReserve = 1 << 17;
    while (g_prof.pool.size() < kReserve) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) break;
      g_prof.pool.push_back(e);
    }
  }
  g_prof.mask = mask;
  g_prof.on = on;
  for (long& n : g_prof.seen) n = 0;
}
void prof_sample_period(int period) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.period = period < 1 ? 1 : period;
  for (long& n : g_prof.seen) n = 0;
}

namespace {
thread_local int g_gemm_prec = GP_F64;
}
int gemm_precision(int p) {
  int old = g_gemm_prec;
  g_gemm_prec = (p == GP_F32 || p == GP_BF16) ? p : GP_F64;
  return old;
}
bool prof_enabled() { return g_prof.on; }
unsigned prof_mask() { return g_prof.on ? g_prof.mask : 0u; }
void prof_reset() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.recs.clear();
  g_prof.used = 0;
}
void prof_read(double* seconds, double* bytes, double* flops, long* launches) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int c = 0; c < KC_COUNT; ++c) {
    seconds[c] = bytes[c] = flops[c] = 0.0;
    launches[c] = 0;
  }
  for (auto& r : g_prof.recs) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    seconds[r.cls] += ms * 1e-3;
    bytes[r.cls] += r.bytes;
    flops[r.cls] += r.flops;
    launches[r.cls] += r.launches;
  }
}

namespace {
constexpr int WAVE = 64;

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// ------------------------------------------------------------------ GEMM
constexpr int TM = 64, TN = 64, TK = 16;
constexpr int LQ = TM * TK / 256;   // staged elements per thread and operand

// Tiled FP64 GEMM: global -> register -> LDS staging of 64 x 16 (A) and
// 16 x 64 (B) slices, 4 elements per thread.
__device__ __forceinline__ void gemm_load_tile(const double* __restrict__ A, long sAi, long sAk, int m, const double* __restrict__ B,
                                               long sBk, long sBj, int n, long kb, int i0, int j0, long kk, bool a_kfast,
                                               bool b_kfast, int tid, double ra[LQ], double rb[LQ]) {
#pragma unroll
  for (int q = 0; q < LQ; ++q) {
    int e = tid + 256 * q;
    int ii, kx;
    if (a_kfast) { kx = e % TK; ii = e / TK; } else { ii = e % TM; kx = e / TM; }
    long gi = i0 + ii, gk = kk + kx;
    ra[q] = (gi < m && gk < kb) ? A[gi * sAi + gk * sAk] : 0.0;
    int jj, kx2;
    if (b_kfast) { kx2 = e % TK; jj = e / TK; } else { jj = e % TN; kx2 = e / TN; }
    long gj = j0 + jj, gk2 = kk + kx2;
    rb[q] = (gj < n && gk2 < kb) ? B[gk2 * sBk + gj * sBj] : 0.0;
  }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// 64 x 64 output tile per 256-thread workgroup on the matrix cores: each wave
// owns a 32 x 32 quarter as 2 x 2 MFMA tiles of 16 x 16.  PREC selects the
// arithmetic: GP_F64 v_mfma_f64_16x16x4 (lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator item v is D[4v + l/16][l%16]); GP_F32
// v_mfma_f32_16x16x4f32 (same inputs; item v is D[4(l/16) + v][l%16]);
// GP_BF16 v_mfma_f32_16x16x16_bf16 (lane l supplies A[l%16][4(l/16)+j] and
// B[4(l/16)+j][l%16], j < 4; output as GP_F32).  The reduced precisions
// round the FP64 operands when they are staged and accumulate in FP32.
// K is staged through LDS in slices of 16, the next slice prefetched into
// registers while the current one is consumed.
// With CSPLIT the output column j is stored at (j / csplit) * sCt +
// (j % csplit) * sCj: a column index (t, xi) laid out as blocks per t.
template <int PREC, typename CT = double, bool CSPLIT = false>
__device__ __forceinline__ void gemm_core(int m, int n, long kb, double alpha, const double* __restrict__ A, long sAi,
                                          long sAk, const double* __restrict__ B, long sBk, long sBj, double beta,
                                          CT* __restrict__ C, long sCi, long sCj, int i0, int j0, int csplit = 1,
                                          long sCt = 0) {
  typedef typename std::conditional<PREC == GP_F64, double, float>::type st_t;
  typedef typename std::conditional<PREC == GP_F64, dbl4, flt4>::type acc_t;
  __shared__ st_t As[TK][TM + 1];
  __shared__ st_t Bs[TK][TN + 1];
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane % 16, lk = lane / 16;
  acc_t acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c] = acc_t{0, 0, 0, 0};
  const bool a_kfast = (sAk == 1);
  const bool b_kfast = (sBk == 1);
  double ra[LQ], rb[LQ];
  if (kb > 0) gemm_load_tile(A, sAi, sAk, m, B, sBk, sBj, n, kb, i0, j0, 0, a_kfast, b_kfast, tid, ra, rb);
  for (long kk = 0; kk < kb; kk += TK) {
#pragma unroll
    for (int q = 0; q < LQ; ++q) {
      int e = tid + 256 * q;
      int ii, kx;
      if (a_kfast) { kx = e % TK; ii = e / TK; } else { ii = e % TM; kx = e / TM; }
      As[kx][ii] = (st_t)ra[q];
      int jj, kx2;
      if (b_kfast) { kx2 = e % TK; jj = e / TK; } else { jj = e % TN; kx2 = e / TN; }
      Bs[kx2][jj] = (st_t)rb[q];
    }
    __syncthreads();
    if (kk + TK < kb) gemm_load_tile(A, sAi, sAk, m, B, sBk, sBj, n, kb, i0, j0, kk + TK, a_kfast, b_kfast, tid, ra, rb);
    if constexpr (PREC == GP_BF16) {
#pragma unroll
      for (int kh = 0; kh < TK / 16; ++kh) {
      bf16x4 a0, a1, b0, b1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int kr = kh * 16 + 4 * lk + j;
        a0[j] = to_bf16(As[kr][wr + lr]);
        a1[j] = to_bf16(As[kr][wr + 16 + lr]);
        b0[j] = to_bf16(Bs[kr][wc + lr]);
        b1[j] = to_bf16(Bs[kr][wc + 16 + lr]);
      }
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc[1][1], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kq = 0; kq < TK / 4; ++kq) {
        const int kr = kq * 4 + lk;
        const st_t a0 = As[kr][wr + lr], a1 = As[kr][wr + 16 + lr];
        const st_t b0 = Bs[kr][wc + lr], b1 = Bs[kr][wc + 16 + lr];
        if constexpr (PREC == GP_F64) {
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        } else {
          acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int tr = 0; tr < 2; ++tr)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = (PREC == GP_F64) ? (4 * v + lk) : (4 * lk + v);
      const long gi = i0 + wr + tr * 16 + row;
      if (gi >= m) continue;
#pragma unroll
      for (int tc = 0; tc < 2; ++tc) {
        const long gj = j0 + wc + tc * 16 + lr;
        if (gj >= n) continue;
        CT* cp = C + gi * sCi + (CSPLIT ? (gj / csplit) * sCt + (gj % csplit) * sCj : gj * sCj);
        double val = alpha * (double)acc[tr][tc][v];
        if (beta != 0.0) val += beta * (double)(*cp);
        *cp = (CT)val;
      }
    }
}

// TAG only names the instantiation (GEMM_GRAM for the tall-skinny Gram
// products of truncations and inner products, GEMM_PROJ for the projections
// of core 3 onto the kept ranks), so that a kernel trace tells them apart
// from the other products.
template <int PREC, int TAG = 0>
__global__ __launch_bounds__(256) void k_gemm(int m, int n, int k, double alpha, const double* __restrict__ A,
                                              long sAb, long sAi, long sAk, const double* __restrict__ B, long sBb,
                                              long sBk, long sBj, double beta, double* __restrict__ C, long sCb,
                                              long sCi, long sCj, int kstep, long klimit) {
  const int b = blockIdx.z;
  long kb = k;
  if (klimit > 0) {
    long rem = klimit - (long)b * kstep;
    kb = rem < k ? rem : k;
  }
  gemm_core<PREC>(m, n, kb, alpha, A + b * sAb, sAi, sAk, B + b * sBb, sBk, sBj, beta, C + b * sCb, sCi, sCj,
                  blockIdx.y * TM, blockIdx.x * TN);
}

// C (float) = A B computed in FP64 and rounded once on the store: the
// full-tensor expansion of the reduced-precision mean solve (the TT cores of
// a sum can cancel in the product, so the product itself stays FP64)
__global__ __launch_bounds__(256) void k_gemm_f32out(int m, int n, int k, const double* __restrict__ A, long sAi,
                                                     long sAk, const double* __restrict__ B, long sBk, long sBj,
                                                     float* __restrict__ C, long sCi, long sCj) {
  gemm_core<GP_F64, float>(m, n, k, 1.0, A, sAi, sAk, B, sBk, sBj, 0.0, C, sCi, sCj, blockIdx.y * TM, blockIdx.x * TN);
}

// C = A B with the output columns split into blocks (see gemm_core): the
// full-tensor expansion written time-major for the time-stepped mean solve
template <int PREC, typename CT>
__global__ __launch_bounds__(256) void k_gemm_csplit(int m, int n, int k, const double* __restrict__ A, long sAi,
                                                     long sAk, const double* __restrict__ B, long sBk, long sBj,
                                                     CT* __restrict__ C, long sCi, int csplit, long sCt) {
  gemm_core<PREC, CT, true>(m, n, k, 1.0, A, sAi, sAk, B, sBk, sBj, 0.0, C, sCi, 1, blockIdx.y * TM, blockIdx.x * TN,
                            csplit, sCt);
}

template <int PREC>
__global__ __launch_bounds__(256) void k_gemm_ptr(const GemmDesc* __restrict__ descs) {
  const GemmDesc d = descs[blockIdx.z];
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  if (i0 >= d.m || j0 >= d.n) return;
  gemm_core<PREC>(d.m, d.n, d.k, d.alpha, d.A, d.sAi, d.sAk, d.B, d.sBk, d.sBj, d.beta, d.C, d.sCi, d.sCj, i0, j0);
}

// out[e] = sum_b ws[b*ne + e]: 64 elements per 256-thread block, the
// four waves split the partial sums and combine through LDS
__global__ __launch_bounds__(256) void k_reduce_partials(int nb, long ne, const double* __restrict__ ws,
                                                         double* __restrict__ out) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x % 64, grp = threadIdx.x / 64;
  const long e = (long)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (e < ne)
    for (int b = grp; b < nb; b += 4) s += ws[(long)b * ne + e];
  sh[grp][lane] = s;
  __syncthreads();
  if (grp == 0 && e < ne) out[e] = sh[0][lane] + sh[1][lane] + sh[2][lane] + sh[3][lane];
}

// ------------------------------------------------------------------ reductions
__device__ double block_sum(double v, double* sh) {
  // 1024 threads max; sh has >= 32 entries
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_down(v, o, WAVE);
  int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  int nw = (blockDim.x + WAVE - 1) / WAVE;
  double t = 0.0;
  if (threadIdx.x < WAVE) {
    t = (l < nw) ? sh[l] : 0.0;
    for (int o = WAVE / 2; o > 0; o >>= 1) t += __shfl_down(t, o, WAVE);
  }
  __syncthreads();
  if (threadIdx.x == 0) sh[0] = t;
  __syncthreads();
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_sumsq_stage1(const double* __restrict__ x, long n, double* __restrict__ ws) {
  __shared__ double sh[32];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double v = x[i];
    s = fma(v, v, s);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) ws[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_sum_stage2(const double* __restrict__ ws, int nb, double* out) {
  __shared__ double sh[32];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += ws[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(1024) void k_dot_reduce(long n, const double* __restrict__ w, const double* __restrict__ k,
                                                    double* out, int acc) {
  __shared__ double sh[32];
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) s = fma(w[i], k[i], s);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = acc ? (*out + s) : s;
}

// ------------------------------------------------------------------ elementwise
__global__ void k_fill(double* p, long n, double v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_store_ranks(int* d, int r1, int r2) {
  if (threadIdx.x == 0) d[0] = r1;
  if (threadIdx.x == 1) d[1] = r2;
}

__global__ void k_copy2d(int rows, int cols, const double* __restrict__ src, long lds, double* __restrict__ dst,
                         long ldd, double alpha, const double* dscale, int inv) {
  double a = alpha;
  if (dscale) a *= inv ? 1.0 / (*dscale) : (*dscale);
  long total = (long)rows * cols;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long i = e / cols, j = e % cols;
    dst[i * ldd + j] = a * src[i * lds + j];
  }
}

// Batched block copies (BlockCopy): grid (column tiles, row tiles, block),
// 32 x 32 tiles through LDS so that a transposed block is read and written
// along its rows; tiles past a block's extent leave at once.
__global__ __launch_bounds__(256) void k_block_copy(const BlockCopy* __restrict__ descs) {
  __shared__ double tile[32][33];
  const BlockCopy d = descs[blockIdx.z];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  if (i0 >= d.rows || j0 >= d.cols) return;   // uniform per workgroup
  const double a = d.dalpha ? d.alpha * (*d.dalpha) : d.alpha;
  if (!d.transpose) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + ty + 8 * q, j = j0 + tx;
      if (i < d.rows && j < d.cols) d.dst[(long)i * d.ldd + j] = a * d.src[(long)i * d.lds + j];
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + ty + 8 * q, j = j0 + tx;
    if (i < d.rows && j < d.cols) tile[ty + 8 * q][tx] = d.src[(long)i * d.lds + j];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + ty + 8 * q, i = i0 + tx;
    if (i < d.rows && j < d.cols) d.dst[(long)j * d.ldd + i] = a * tile[tx][ty + 8 * q];
  }
}

// dst[j][i] = src[i][j] through a 32 x 32 LDS tile: both the reads (along j)
// and the writes (along i) are coalesced.  blockDim (32, 8); tiles walk the
// rows with a grid stride so any row count fits the grid.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_transpose_copy(int rows, int cols, const TI* __restrict__ src, long lds,
                                                        long sbatch, TO* __restrict__ dst, long ldd, long dbatch) {
  __shared__ TO tile[32][33];
  src += blockIdx.z * sbatch;   // batch of independent transposes along grid z
  dst += blockIdx.z * dbatch;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int j0 = blockIdx.x * 32;
  for (long i0 = (long)blockIdx.y * 32; i0 < rows; i0 += (long)gridDim.y * 32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long i = i0 + ty + 8 * q;
      const int j = j0 + tx;
      if (i < rows && j < cols) tile[ty + 8 * q][tx] = (TO)src[i * lds + j];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + ty + 8 * q;
      const long i = i0 + tx;
      if (i < rows && j < cols) dst[(long)j * ldd + i] = tile[tx][ty + 8 * q];
    }
    __syncthreads();
  }
}

__global__ void k_scale_by(double* p, long n, const double* ds, int inv) {
  double a = inv ? 1.0 / (*ds) : (*ds);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] *= a;
}

__global__ void k_sub(const double* a, const double* b, double* o, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    o[i] = a[i] - b[i];
}

__global__ void k_check_finite(const double* x, long n, int* flag) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) *flag = 1;
}

__global__ void k_scalar(int kind, const double* a, const double* b, double* out) {
  double va = a ? *a : 0.0, vb = b ? *b : 0.0, r = 0.0;
  switch (kind) {
    case 0: r = sqrt(fmax(va + vb, 0.0)); break;
    case 1: r = 1.0 / va; break;
    case 2: r = va * vb; break;
    case 3: r = va + vb; break;
    case 4: r = -va; break;
    case 5: r = sqrt(fmax(va, 0.0)); break;
  }
  *out = r;
}

// ------------------------------------------------------------------ SpMM
constexpr int NVMAX = 16;

// CSR SpMM with nv value arrays sharing one pattern: one row per wave, one
// output column per lane.  The row index is made wave-uniform, so the row's
// pattern and values are read with scalar loads; its input rows are loaded
// eight entries at a time before their products, so eight loads are in
// flight per lane instead of one.  Products are accumulated in entry order.
__global__ __launch_bounds__(256) void k_spmm(int nrows, int ics, int ocs, const int* __restrict__ rowptr,
                                              const int* __restrict__ col, const double* __restrict__ vals, int nv,
                                              long vstride, const double* __restrict__ x, int ldx, int xcol0,
                                              int ncols, double* __restrict__ y, int ldy, int ycol0, int yvstep,
                                              double alpha, double beta) {
  constexpr int EB = 8;   // entries per batch of loads
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
  const int r = blockIdx.x * (blockDim.x / WAVE) + wave;
  const int c = blockIdx.y;
  if (r >= nrows) return;
  const int t0 = rowptr[r], t1 = rowptr[r + 1];
  const double* xb = x + (long)c * ics * ldx + xcol0;
  double* yb = y + ((long)c * ocs + r) * ldy + ycol0;
  for (int j0 = 0; j0 < ncols; j0 += WAVE) {
    const int j = j0 + lane;
    const bool act = j < ncols;
    const int jc = act ? j : ncols - 1;   // idle lanes read a valid column
    double acc[NVMAX];
#pragma unroll
    for (int v = 0; v < NVMAX; ++v) acc[v] = 0.0;
    int t = t0;
    for (; t + EB <= t1; t += EB) {
      double xv[EB];
#pragma unroll
      for (int q = 0; q < EB; ++q) xv[q] = xb[(long)col[t + q] * ldx + jc];
      // value array outside, entries inside: a value array's EB values are
      // contiguous (one wide scalar load), and each sum keeps entry order
#pragma unroll
      for (int v = 0; v < NVMAX; ++v) {
        if (v >= nv) break;
        const double* vv = vals + v * vstride + t;
#pragma unroll
        for (int q = 0; q < EB; ++q) acc[v] = fma(vv[q], xv[q], acc[v]);
      }
    }
    for (; t < t1; ++t) {
      const double xv = xb[(long)col[t] * ldx + jc];
#pragma unroll
      for (int v = 0; v < NVMAX; ++v)
        if (v < nv) acc[v] = fma(vals[v * vstride + t], xv, acc[v]);
    }
    if (act) {
#pragma unroll
      for (int v = 0; v < NVMAX; ++v)
        if (v < nv) yb[v * yvstep + j] = alpha * acc[v] + (beta != 0.0 ? beta * yb[v * yvstep + j] : 0.0);
    }
  }
}

// lane l's value, as a wave-uniform (scalar) value
__device__ inline double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline double readlane_val(double v, int l) { return readlane_f64(v, l); }
__device__ inline float readlane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// One value array, rows of at most NZ entries: each lane holds one entry of
// its wave's row, broadcast across the wave, so all the row's input loads
// are issued back to back (one memory round trip per row instead of one per
// entry).
template <int NZ>
__global__ __launch_bounds__(256) void k_spmm_short(int nrows, int ics, int ocs, const int* __restrict__ rowptr,
                                                    const int* __restrict__ col, const double* __restrict__ vals,
                                                    const double* __restrict__ x, int ldx, int xcol0, int ncols,
                                                    double* __restrict__ y, int ldy, int ycol0, double alpha,
                                                    double beta) {
  static_assert(NZ <= WAVE, "one entry per lane");
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int r = blockIdx.x * (blockDim.x / WAVE) + wave;
  const int c = blockIdx.y;
  if (r >= nrows) return;
  const int t0 = __builtin_amdgcn_readfirstlane(rowptr[r]);   // uniform per wave
  const int n = __builtin_amdgcn_readfirstlane(rowptr[r + 1]) - t0;
  double* yb = y + ((long)c * ocs + r) * ldy + ycol0;
  if (n == 0) {
    for (int j = lane; j < ncols; j += WAVE) yb[j] = beta != 0.0 ? beta * yb[j] : 0.0;
    return;
  }
  // lanes past the row's end repeat its first column with value 0, so every
  // load below is valid and none is predicated
  int my_col = lane < n ? col[t0 + lane] : 0;
  my_col = lane < n ? my_col : __builtin_amdgcn_readfirstlane(my_col);
  const double my_val = lane < n ? vals[t0 + lane] : 0.0;
  const double* xb = x + (long)c * ics * ldx + xcol0;
  for (int j0 = 0; j0 < ncols; j0 += WAVE) {
    const int j = j0 + lane;
    const bool act = j < ncols;
    const int jc = act ? j : ncols - 1;   // idle lanes read a valid column
    double xv[NZ];
#pragma unroll
    for (int q = 0; q < NZ; ++q) xv[q] = xb[(long)__builtin_amdgcn_readlane(my_col, q) * ldx + jc];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < NZ; ++q) acc = fma(readlane_f64(my_val, q), xv[q], acc);
    if (act) yb[j] = alpha * acc + (beta != 0.0 ? beta * yb[j] : 0.0);
  }
}

// Padded-row (ELL) SpMM over row groups.  A workgroup takes one group of
// consecutive rows (at most ELL_GROUP_ROWS) and first copies the group's
// distinct input rows (at most ELL_GROUP_UMAX, listed in ascending order) into
// LDS with coalesced loads: neighbouring rows share most of their inputs, so
// an input row leaves L2 once per group instead of once per entry that uses
// it.  Each wave then forms rows wave, wave + 4, ... of the group with one
// lane per output column.  A row's entries (LDS positions and values) are
// wave-uniform and read with scalar loads, ELL_CHUNK at a time: the row
// length is rounded up to whole chunks (the extra slots hold value 0 and a
// valid position), so a chunk's LDS reads are issued together with no
// branches between them.  Columns are processed in chunks of cw (the LDS holds
// umax x cw values).  Workgroups are remapped so that each XCD (ids are dealt
// round-robin over the 8 XCDs) takes a contiguous range of groups; the grid
// is a multiple of 8.
template <typename T>
__global__ __launch_bounds__(256) void k_ell_grouped(int ngroups, int ics, int ocs, const int* __restrict__ row0,
                                                     const int* __restrict__ uptr, const int* __restrict__ ucols,
                                                     const int* __restrict__ lidx, const int* __restrict__ rlen,
                                                     const T* __restrict__ eval, const T* __restrict__ x, int ldx,
                                                     int xcol0, int ncols, int cw, T* __restrict__ y, int ldy,
                                                     int ycol0, T alpha, T beta) {
  constexpr int RPW = ELL_GROUP_ROWS / 4;   // rows per wave
  constexpr int UNR = 24;                   // staging loads in flight per thread
  static_assert(ELL_GROUP_ROWS % 4 == 0 && ELL_WIDTH % ELL_CHUNK == 0, "group shape");
  extern __shared__ __align__(16) unsigned char ell_smem[];
  T* xs = reinterpret_cast<T*>(ell_smem);
  __shared__ int us[ELL_GROUP_UMAX];
  const unsigned per = gridDim.x / 8;
  const unsigned g = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (g >= (unsigned)ngroups) return;   // whole workgroup: before any barrier
  const int c = blockIdx.y;
  const int ra = row0[g], rb = row0[g + 1];
  const int ua = uptr[g], U = uptr[g + 1] - ua;
  // the wave index as a scalar, so that row addresses (and the entry loads
  // through them) are uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x % WAVE;
  for (int u = threadIdx.x; u < U; u += blockDim.x) us[u] = ucols[ua + u];
  __syncthreads();
  const T* xb = x + (long)c * ics * ldx + xcol0;
  for (int j0 = 0; j0 < ncols; j0 += cw) {
    const int w = min(cw, ncols - j0);
    if (j0 > 0) __syncthreads();   // every read of the previous chunk is done
    const int jc = lane < w ? lane : w - 1;   // idle lanes read a valid value
    // this chunk's old outputs, loaded now so that their latency overlaps the
    // staging below
    T yo[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = ra + wave + 4 * i;
      yo[i] = (r < rb && lane < w && beta != (T)0) ? y[((long)c * ocs + r) * ldy + ycol0 + j0 + jc] : (T)0;
    }
    // element i of the U x w chunk is (i / w, i % w); thread t takes
    // i = t, t + 256, ..., with the quotient and remainder advanced in steps;
    // up to UNR loads per thread are issued before the first LDS store
    const int tot = U * w;
    const int du = 256 / w, dj = 256 - du * w;
    int u = threadIdx.x / w, j = threadIdx.x - u * w;
    for (int i0 = threadIdx.x; i0 < tot; i0 += 256 * UNR) {
      T v[UNR];
#pragma unroll
      for (int k = 0; k < UNR; ++k) {
        v[k] = i0 + 256 * k < tot ? xb[(long)us[u] * ldx + j0 + j] : (T)0;
        j += dj;
        u += du;
        if (j >= w) {
          j -= w;
          ++u;
        }
      }
#pragma unroll
      for (int k = 0; k < UNR; ++k)
        if (i0 + 256 * k < tot) xs[i0 + 256 * k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = ra + wave + 4 * i;
      if (r >= rb) break;   // uniform per wave
      const int n = rlen[r];
      const int* lr = lidx + (long)r * ELL_WIDTH;
      const T* vr = eval + (long)r * ELL_WIDTH;
      T acc = 0;
      for (int k = 0; k < n; k += ELL_CHUNK) {
        T xv[ELL_CHUNK];
#pragma unroll
        for (int q = 0; q < ELL_CHUNK; ++q) xv[q] = xs[lr[k + q] * w + jc];
#pragma unroll
        for (int q = 0; q < ELL_CHUNK; ++q) acc = fma(vr[k + q], xv[q], acc);
      }
      if (lane < w) y[((long)c * ocs + r) * ldy + ycol0 + j0 + lane] = alpha * acc + beta * yo[i];
    }
  }
}

// ------------------------------------------------------------------ core ops
__global__ void k_core1_op(int kind, int n1, int r, const double* __restrict__ in, int ldi, double* __restrict__ out,
                           int ldo, int col0, double scale, const double* dscale) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= r) return;
  double sc = scale * (dscale ? *dscale : 1.0);
  if (kind == 0) {
    double prev = 0.0;
    for (int t = 0; t < n1; ++t) {
      double v = in[(long)t * ldi + a];
      out[(long)t * ldo + col0 + a] = sc * (v - prev);
      prev = v;
    }
  } else if (kind == 1) {
    for (int t = 0; t < n1; ++t) out[(long)t * ldo + col0 + a] = sc * in[(long)t * ldi + a];
  } else {
    double s = 0.0;
    for (int t = 0; t < n1; ++t) {
      s += in[(long)t * ldi + a];
      out[(long)t * ldo + col0 + a] = sc * s;
    }
  }
}

__global__ void k_core1_diag(int n1, int r, int k, const double* __restrict__ w, int ldw, const double* __restrict__ in,
                             int ldi, double* __restrict__ out, int ldo, int col0) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)n1 * k * r;
  if (e >= total) return;
  int al = e % r;
  long q = e / r;
  int a = q % k;
  int t = q / k;
  out[(long)t * ldo + col0 + a * r + al] = w[(long)t * ldw + a] * in[(long)t * ldi + al];
}

__global__ void k_core2_block(int r1, int n2, int r2, const double* __restrict__ in, const double* __restrict__ X,
                              int k1, int k2, double* __restrict__ out, int R1, int R2, int row0, int col0) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)k1 * k2 * r1 * n2 * r2;
  if (e >= total) return;
  int be = e % r2;
  long q = e / r2;
  int i = q % n2;
  q /= n2;
  int al = q % r1;
  q /= r1;
  int b = q % k2;
  int a = q / k2;
  double s;
  if (X == nullptr) {
    s = in[((long)al * n2 + i) * r2 + be];
  } else {
    const double* Xab = X + ((long)a * k2 + b) * n2 * n2 + (long)i * n2;
    s = 0.0;
    for (int j = 0; j < n2; ++j) s = fma(Xab[j], in[((long)al * n2 + j) * r2 + be], s);
  }
  out[((long)(row0 + a * r1 + al) * n2 + i) * R2 + col0 + b * r2 + be] = s;
}

// ------------------------------------------------------------------ truncation
constexpr int TE_THREADS = 1024;
constexpr int KSMALL = 96;     // max rank handled by the LDS eigen solver
constexpr int KLD = KSMALL + 1;   // LDS row stride of its matrices (odd: rows start on different banks)
constexpr int KCAP = 512;      // max rank of any truncation

// sum_t L[t*N + i] * coef[t*cs] for t < j (L column-major in global memory,
// coef in LDS): eight loads in flight, four partial sums.
__device__ inline double col_combo(const double* __restrict__ L, long N, int i, const double* coef, int cs, int j) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int t = 0;
  for (; t + 8 <= j; t += 8) {
    double l[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) l[q] = L[(long)(t + q) * N + i];
    a0 = fma(l[0], coef[(t + 0) * cs], a0);
    a1 = fma(l[1], coef[(t + 1) * cs], a1);
    a2 = fma(l[2], coef[(t + 2) * cs], a2);
    a3 = fma(l[3], coef[(t + 3) * cs], a3);
    a0 = fma(l[4], coef[(t + 4) * cs], a0);
    a1 = fma(l[5], coef[(t + 5) * cs], a1);
    a2 = fma(l[6], coef[(t + 6) * cs], a2);
    a3 = fma(l[7], coef[(t + 7) * cs], a3);
  }
  for (; t < j; ++t) a0 = fma(L[(long)t * N + i], coef[t * cs], a0);
  return (a0 + a1) + (a2 + a3);
}

// wave-wide dot product of two length-N vectors in global memory (result on
// every lane): eight loads per vector in flight
__device__ inline double wave_dot(const double* __restrict__ x, const double* __restrict__ y, int N) {
  const int ln = threadIdx.x % WAVE;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = ln;
  for (; i + 7 * WAVE < N; i += 8 * WAVE) {
    double xv[8], yv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      xv[q] = x[i + q * WAVE];
      yv[q] = y[i + q * WAVE];
    }
    a0 = fma(xv[0], yv[0], a0);
    a1 = fma(xv[1], yv[1], a1);
    a2 = fma(xv[2], yv[2], a2);
    a3 = fma(xv[3], yv[3], a3);
    a0 = fma(xv[4], yv[4], a0);
    a1 = fma(xv[5], yv[5], a1);
    a2 = fma(xv[6], yv[6], a2);
    a3 = fma(xv[7], yv[7], a3);
  }
  for (; i < N; i += WAVE) a0 = fma(x[i], y[i], a0);
  double s = (a0 + a1) + (a2 + a3);
  for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
  return s;
}

// Block-wide (max with smallest index on ties, sum) in one barrier: each wave
// posts its partials to buffer `par` (alternate two buffers between calls),
// then every thread combines all of them.
__device__ inline void block_argmax_sum(double v, int idx, double sm, double* shv, int* shi, double* shs, int par,
                                        double& bv, int& bi, double& bsum) {
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const double ov = __shfl_down(v, o, WAVE);
    const int oi = __shfl_down(idx, o, WAVE);
    sm += __shfl_down(sm, o, WAVE);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  if (threadIdx.x % WAVE == 0) {
    shv[par * 16 + w] = v;
    shi[par * 16 + w] = idx;
    shs[par * 16 + w] = sm;
  }
  __syncthreads();
  bv = shv[par * 16];
  bi = shi[par * 16];
  bsum = shs[par * 16];
  for (int q = 1; q < nw; ++q) {
    const double qv = shv[par * 16 + q];
    const int qi = shi[par * 16 + q];
    if (qv > bv || (qv == bv && qi < bi)) {
      bv = qv;
      bi = qi;
    }
    bsum += shs[par * 16 + q];
  }
}

// Two-pass classical Gram-Schmidt of the k columns of X (column-major, ld
// N, overwritten), one wave per coefficient; U (N x k, ld kmax) receives the
// orthonormal columns.  Whole workgroup; lp holds >= k doubles of LDS.
__device__ void gs2_block(int N, int k, double* __restrict__ X, double* __restrict__ U, int kmax, double* lp,
                          double* shv) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int wv = tid / WAVE, ln = tid % WAVE, nwv = nth / WAVE;
  for (int c = 0; c < k; ++c) {
    double* xc = X + (long)c * N;
    for (int pass = 0; pass < 2 && c > 0; ++pass) {
      for (int d = wv; d < c; d += nwv) {
        const double sv = wave_dot(X + (long)d * N, xc, N);
        if (ln == 0) lp[d] = sv;
      }
      __syncthreads();
      for (int i = tid; i < N; i += nth) xc[i] -= col_combo(X, N, i, lp, 1, c);
      __syncthreads();
    }
    double s = 0.0;
    for (int i = tid; i < N; i += nth) s = fma(xc[i], xc[i], s);
    s = block_sum(s, shv);
    double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int i = tid; i < N; i += nth) xc[i] *= inv;
    __syncthreads();
  }
  for (long e = tid; e < (long)N * k; e += nth) {
    int i = e / k, c = e % k;
    U[(long)i * kmax + c] = X[(long)c * N + i];
  }
}


// Symmetric truncation of a Gram matrix S (N x N), first stage, one
// workgroup.  Pivoted Cholesky S ~ L L^T (L column-major, ld N).  Outcomes:
// info = 2 (more than KSMALL pivots needed and large_ok: the caller runs the
// blocked path); a zero matrix (rank 1, U = e_1); mode 1 (more than KSMALL
// pivots, bond without a large path: U = orthonormal basis of the pivoted
// columns, by two-pass Gram-Schmidt here); or mode 0: *kp_out = kp > 0 and
// state = {trace, delta^2, zero threshold, residual trace} for the
// eigen-decomposition stage (k_trunc_jacobi), else *kp_out = 0.
__global__ __launch_bounds__(TE_THREADS) void k_trunc_pc(int N, double* __restrict__ S, double eps,
                                                         const double* normsq_in, double* normsq_out,
                                                         double* __restrict__ U, int kmax, double* __restrict__ L,
                                                         double* __restrict__ dwork, int* k_out, double* kept_out,
                                                         int* info, int rank_bound, int large_ok, int* kp_out,
                                                         double* state, int* piv_out) {
  __shared__ double shv[32];
  __shared__ int shi[32];
  __shared__ double shs[32];
  __shared__ double lp[KCAP];
  const int tid = threadIdx.x, nth = blockDim.x;
  if (kmax > KCAP) kmax = KCAP;
  // --- trace and tolerance
  double tr = 0.0;
  for (int i = tid; i < N; i += nth) {
    double d = S[(long)i * N + i];
    dwork[i] = d > 0.0 ? d : 0.0;
    tr += dwork[i];
  }
  tr = block_sum(tr, shv);
  double normsq = normsq_in ? *normsq_in : tr;
  if (normsq_out && tid == 0) *normsq_out = tr;
  const double delta2 = 0.5 * eps * eps * normsq;
  const double zero_thr = 64.0 * 2.220446049250313e-16 * (tr > 0.0 ? tr : 0.0);
  const double res_stop = delta2 * 0.0625;
  // --- pivoted Cholesky S ~ L L^T.  Stops at resid <= delta2/16 (then the
  // eigen-decomposition of the small factor decides the rank), or, when more
  // than KSMALL pivots would be needed, at resid <= delta2 (then the pivoted
  // Cholesky subspace itself is the truncation: mode 1).
  double resid = tr;
  int kp = 0, ka = -1, mode = 0;
  // largest remaining diagonal entry (bv at index bi) and the residual trace
  // are reduced together, once per pivot
  double bv, rsum;
  int bi;
  {
    double mv = -1.0;
    int mi = 0;
    for (int i = tid; i < N; i += nth)
      if (dwork[i] > mv) { mv = dwork[i]; mi = i; }
    block_argmax_sum(mv, mi, 0.0, shv, shi, shs, 0, bv, bi, rsum);
  }
  for (int j = 0; j < kmax; ++j) {
    if (delta2 > 0.0) {
      if (resid <= delta2 && ka < 0) ka = kp;
      if (mode == 0 && resid <= res_stop) break;
      if (mode == 0 && kp == KSMALL) {
        if (ka >= 0) break;
        mode = 1;
        if (large_ok) break;   // more than KSMALL pivots: the caller runs the blocked path
      }
      if (mode == 1 && resid <= delta2) break;
    }
    if (bv <= zero_thr || bv <= 0.0) break;
    const int p = bi;
    if (tid == 0 && j < KSMALL) piv_out[j] = p;
    for (int t = tid; t < j; t += nth) lp[t] = L[(long)t * N + p];
    __syncthreads();
    const double ljj = sqrt(bv);
    double mv = -1.0, rr = 0.0;
    int mi = 0;
    for (int i = tid; i < N; i += nth) {
      // S is symmetric: row p read coalesced
      const double sv = S[(long)p * N + i] - col_combo(L, N, i, lp, 1, j);
      const double lij = (i == p) ? ljj : sv / ljj;
      L[(long)j * N + i] = lij;
      const double d = dwork[i] - lij * lij;
      const double dn = (i == p || d < 0.0) ? 0.0 : d;
      dwork[i] = dn;
      rr += dn;
      if (dn > mv) { mv = dn; mi = i; }
    }
    block_argmax_sum(mv, mi, rr, shv, shi, shs, (j + 1) & 1, bv, bi, resid);
    kp = j + 1;
  }
  __syncthreads();
  if (tid == 0) {
    *kp_out = 0;
    // residual trace, target, zero threshold, trace: the layout of the
    // blocked path's state, which resumes from these pivots
    state[0] = resid;
    state[1] = delta2;
    state[2] = zero_thr;
    state[3] = tr;
  }
  if (mode == 1 && large_ok) {
    if (tid == 0) *info = 2;
    return;
  }
  if (kp == 0) {
    // zero (or numerically zero) matrix: rank-1 zero
    for (int i = tid; i < N; i += nth) U[(long)i * kmax] = (i == 0) ? 1.0 : 0.0;
    if (tid == 0) {
      *k_out = 1;
      *kept_out = 0.0;
      *info = 0;
    }
    return;
  }
  if (tid == 0) *info = (kp == kmax && kmax < rank_bound && resid > (mode ? delta2 : res_stop) && resid > zero_thr) ? 1 : 0;
  if (mode == 1) {
    // truncation = span of the pivoted Cholesky columns (rank kp); U is an
    // orthonormal basis of that span (Gram-Schmidt below)
    if (tid == 0) {
      shi[0] = kp;
      *k_out = kp;
      *kept_out = tr - resid;
    }
    __syncthreads();
  }
  if (mode == 0) {
    // columns kp .. min(KSMALL, kmax) - 1 of L are zero for the fixed-size
    // products of the next stages
    const int km = min(KSMALL, kmax);
    for (long e = tid; e < (long)N * (km - kp); e += nth) L[(long)kp * N + e] = 0.0;
    if (tid == 0) *kp_out = kp;
    return;
  }
  const int k = shi[0];
  __syncthreads();
  gs2_block(N, k, L, U, kmax, lp, shv);
}

// Second stage: eigen-decomposition of T = L^T L (kp x kp of a km x km
// product, ld KSMALL; kp read from the first stage, nothing to do when 0) by
// cyclic Jacobi in LDS, rank cut k (smallest k with discarded eigenvalues +
// residual trace <= delta^2, or every numerically nonzero direction when
// delta = 0), and W = V_k diag(lambda^-1/2) (km x km, zero outside kp x k,
// ld KSMALL) so that L W spans the kept subspace with orthonormal columns.
__global__ __launch_bounds__(TE_THREADS) void k_trunc_jacobi(int km, const int* __restrict__ kp_dev,
                                                             const double* __restrict__ Tg,
                                                             const double* __restrict__ state, double* __restrict__ W,
                                                             int* k_out, double* kept_out) {
  __shared__ double T[KSMALL * KLD];
  __shared__ double V[KSMALL * KLD];
  __shared__ int shi[32];
  __shared__ double rc[KSMALL / 2 + 1], rs[KSMALL / 2 + 1];
  __shared__ int rp[KSMALL / 2 + 1], rq[KSMALL / 2 + 1];
  __shared__ double lam[KSMALL];
  __shared__ int order[KSMALL];
  __shared__ int s_flag;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int n = *kp_dev;
  if (n <= 0) return;   // the first stage finished the truncation
  const double resid = state[0], delta2 = state[1], zero_thr = state[2];
  for (int e = tid; e < n * n; e += nth) {
    const int a = e / n, b = e - a * n;
    T[a * KLD + b] = 0.5 * (Tg[a * KSMALL + b] + Tg[b * KSMALL + a]);
    V[a * KLD + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  // --- cyclic Jacobi (round-robin pairs)
  double ttr = 0.0;
  for (int i = 0; i < n; ++i) ttr += fabs(T[i * KLD + i]);
  const int np2 = n + (n & 1);
  const int npairs = np2 / 2;
  static_assert(KSMALL <= 128, "item grids of the rotation updates");
  int tsh = 0, vsh = 0;   // log2 of the item grid widths (>= npairs, >= n)
  while ((1 << tsh) < npairs) ++tsh;
  while ((1 << vsh) < n) ++vsh;
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    // a sweep in which no pair would rotate changes nothing: test every
    // pair against the rotation threshold first and stop without it
    if (tid == 0) s_flag = 0;
    __syncthreads();
    for (int e = tid; e < n * n; e += nth) {
      const int a = e / n, b = e - a * n;
      if (a < b) {
        const double apq = T[a * KLD + b];
        if (fabs(apq) > fmax(1e-13 * sqrt(fabs(T[a * KLD + a] * T[b * KLD + b])), 1e-16 * ttr) && apq != 0.0)
          s_flag = 1;
      }
    }
    __syncthreads();
    if (!s_flag) break;   // uniform: every thread reads the flag after the barrier
    __syncthreads();
    if (tid == 0) s_flag = 0;
    __syncthreads();
    for (int rnd = 0; rnd < np2 - 1; ++rnd) {
      if (tid < npairs) {
        int a, b;
        if (tid == 0) {
          a = np2 - 1;
          b = rnd;
        } else {   // (rnd + tid) and (rnd - tid) modulo np2 - 1, both in range after one step
          a = rnd + tid;
          if (a >= np2 - 1) a -= np2 - 1;
          b = rnd - tid;
          if (b < 0) b += np2 - 1;
        }
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < n) {
          double apq = T[p * KLD + q], app = T[p * KLD + p], aqq = T[q * KLD + q];
          if (fabs(apq) > fmax(1e-13 * sqrt(fabs(app * aqq)), 1e-16 * ttr) && apq != 0.0) {
            double th = (aqq - app) / (2.0 * apq);
            double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            s_flag = 1;
          }
        } else {
          q = p;   // dummy pair
        }
        rp[tid] = p;
        rq[tid] = q;
        rc[tid] = c;
        rs[tid] = s;
      }
      __syncthreads();
      // T <- J^T T J in one pass: the pairs are disjoint, so every 2 x 2
      // block (rows of pair a, columns of pair b) is updated on its own by
      // the two rotations; V <- V J alongside
      // (item grids a power of two wide: no integer division by a count)
      for (int e = tid; e < (npairs << tsh); e += nth) {
        const int a = e >> tsh, b = e & ((1 << tsh) - 1);
        if (b >= npairs) continue;
        const double sa = rs[a], sb = rs[b];
        if (sa == 0.0 && sb == 0.0) continue;
        const double ca = rc[a], cb = rc[b];
        const int pa = rp[a], qa = rq[a], pb = rp[b], qb = rq[b];
        const bool ra = pa != qa, rb = pb != qb;   // a dummy pair is one index
        const double bpp = T[pa * KLD + pb];
        const double bpq = rb ? T[pa * KLD + qb] : 0.0;
        const double bqp = ra ? T[qa * KLD + pb] : 0.0;
        const double bqq = (ra && rb) ? T[qa * KLD + qb] : 0.0;
        const double xpp = ca * bpp - sa * bqp, xpq = ca * bpq - sa * bqq;
        const double xqp = sa * bpp + ca * bqp, xqq = sa * bpq + ca * bqq;
        T[pa * KLD + pb] = cb * xpp - sb * xpq;
        if (rb) T[pa * KLD + qb] = sb * xpp + cb * xpq;
        if (ra) T[qa * KLD + pb] = cb * xqp - sb * xqq;
        if (ra && rb) T[qa * KLD + qb] = sb * xqp + cb * xqq;
      }
      for (int e = tid; e < (npairs << vsh); e += nth) {
        const int pr = e >> vsh, i = e & ((1 << vsh) - 1);
        if (i >= n) continue;
        const int p = rp[pr], q = rq[pr];
        if (p == q || rs[pr] == 0.0) continue;
        const double c = rc[pr], s = rs[pr];
        const double vp = V[i * KLD + p], vq = V[i * KLD + q];
        V[i * KLD + p] = c * vp - s * vq;
        V[i * KLD + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    int f = s_flag;
    __syncthreads();
    if (!f) break;
  }
  // --- sort eigenvalues descending
  if (tid < n) lam[tid] = T[tid * KLD + tid] > 0.0 ? T[tid * KLD + tid] : 0.0;
  __syncthreads();
  if (tid < n) {
    double v = lam[tid];
    int rank = 0;
    for (int j = 0; j < n; ++j)
      if (lam[j] > v || (lam[j] == v && j < tid)) ++rank;
    order[rank] = tid;
  }
  __syncthreads();
  // --- rank cut: smallest k >= 1 with tail + resid <= delta2
  if (tid == 0) {
    int k = 0;
    double kept = 0.0;
    if (delta2 > 0.0) {
      double tail = resid;
      for (int j = 0; j < n; ++j) tail += lam[order[j]];
      k = n;
      for (int j = 0; j < n; ++j) {
        tail -= lam[order[j]];
        kept += lam[order[j]];
        if (tail <= delta2) { k = j + 1; break; }
      }
    } else {
      // exact mode: keep every numerically nonzero direction
      for (int j = 0; j < n; ++j)
        if (lam[order[j]] > zero_thr) { ++k; kept += lam[order[j]]; }
      if (k == 0) k = 1;
    }
    shi[0] = k;
    *k_out = k;
    *kept_out = kept;
  }
  __syncthreads();
  const int kc = shi[0];
  __syncthreads();
  // --- W = V_k diag(lambda^-1/2), zero outside kp x k (km x km written)
  for (int e = tid; e < km * km; e += nth) {
    const int a = e / km, c = e - a * km;
    double w = 0.0;
    if (a < n && c < kc) {
      const int oc = order[c];
      const double l = lam[oc];
      w = l > 0.0 ? V[a * KLD + oc] / sqrt(l) : 0.0;
    }
    W[a * KSMALL + c] = w;
  }
}

// R = C^-T (upper triangular, km x km, zero outside k x k, ld KSMALL) for
// the Cholesky factor C of the leading k x k block of the symmetric positive
// definite G (ld KSMALL), so that U R has orthonormal columns when
// G = U^T U (Cholesky QR); k read from the eigen stage, nothing to do when
// the first stage finished.  *info = 3 if G is not numerically positive
// definite.
__global__ __launch_bounds__(256) void k_chol_inv(int km, const int* __restrict__ kp_dev, const int* __restrict__ k_dev,
                                                  const double* __restrict__ G, double* __restrict__ R, int* info) {
  __shared__ double C[KSMALL * KLD];
  __shared__ double X[KSMALL * KLD];
  __shared__ int bad;
  const int tid = threadIdx.x, nth = blockDim.x;
  if (*kp_dev <= 0) return;   // the first stage finished the truncation
  const int k = *k_dev;
  for (int e = tid; e < km * km; e += nth) R[(e / km) * KSMALL + e % km] = 0.0;
  if (tid == 0) bad = 0;
  for (int e = tid; e < k * k; e += nth) {
    const int a = e / k, b = e - a * k;
    C[a * KLD + b] = a >= b ? 0.5 * (G[a * KSMALL + b] + G[b * KSMALL + a]) : 0.0;
  }
  __syncthreads();
  // right-looking Cholesky on the unscaled Schur complement: step j takes
  // d_j = S[j][j] and updates S[i][l] -= S[i][j] S[l][j] / d_j for
  // j < l <= i; column j is final after step j, so the scaling by sqrt(d_j)
  // waits until the end and each step needs one barrier
  __shared__ double rdiag[KSMALL];
  for (int j = 0; j < k; ++j) {
    __syncthreads();
    const double d = C[j * KLD + j];   // same value on every thread
    if (d <= 0.0) {
      if (tid == 0) bad = 1;
      break;
    }
    if (tid == 0) rdiag[j] = sqrt(d);
    const double inv_d = 1.0 / d;
    const int m = k - j - 1;
    for (int e = tid; e < m * (m + 1) / 2; e += nth) {
      // e -> (a, b), b <= a, row-major over the lower triangle
      int a = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while (a * (a + 1) / 2 > e) --a;
      while ((a + 1) * (a + 2) / 2 <= e) ++a;
      const int b = e - a * (a + 1) / 2;
      const int i = j + 1 + a, l = j + 1 + b;
      C[i * KLD + l] -= C[i * KLD + j] * C[l * KLD + j] * inv_d;
    }
  }
  __syncthreads();
  if (!bad) {
    for (int e = tid; e < k * k; e += nth) {
      const int i = e / k, j = e - i * k;
      if (i > j) C[i * KLD + j] /= rdiag[j];
    }
    for (int j = tid; j < k; j += nth) C[j * KLD + j] = rdiag[j];
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) *info = 3;
    return;
  }
  // X = C^-1 by columns (thread j owns column j), then R = X^T
  for (int j = tid; j < k; j += nth) {
    for (int i = 0; i < j; ++i) X[i * KLD + j] = 0.0;
    X[j * KLD + j] = 1.0 / C[j * KLD + j];
    for (int i = j + 1; i < k; ++i) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int l = j;
      for (; l + 4 <= i; l += 4) {
        s0 = fma(C[i * KLD + l], X[l * KLD + j], s0);
        s1 = fma(C[i * KLD + l + 1], X[(l + 1) * KLD + j], s1);
        s2 = fma(C[i * KLD + l + 2], X[(l + 2) * KLD + j], s2);
        s3 = fma(C[i * KLD + l + 3], X[(l + 3) * KLD + j], s3);
      }
      for (; l < i; ++l) s0 = fma(C[i * KLD + l], X[l * KLD + j], s0);
      X[i * KLD + j] = -((s0 + s1) + (s2 + s3)) / C[i * KLD + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += nth) {
    const int a = e / k, b = e - a * k;
    R[a * KSMALL + b] = X[b * KLD + a];
  }
}

// U[i][c] = X[i][c] (X row-major, ld ldx) for c < *k_dev, when the eigen
// stage ran (*kp_dev > 0)
__global__ void k_take_basis(const int* __restrict__ kp_dev, const int* __restrict__ k_dev, int N,
                             const double* __restrict__ X, int ldx, double* __restrict__ U, int kmax) {
  if (*kp_dev <= 0) return;
  const int k = *k_dev;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)N * k; e += (long)gridDim.x * blockDim.x) {
    const long i = e / k;
    const int c = (int)(e - i * k);
    U[i * kmax + c] = X[i * ldx + c];
  }
}

// ------------------------------------------------------------------ SG convection, full format
constexpr int SGC_NXI = 64;   // largest chaos dimension of the full-format convection

// One wave per (element, time step): out[t, i, c*ns + free(a)] += sign *
//   sum_g w_g phi_a(g) sum_{l,k} H_{ilk} (W_l(g) . grad) U_{k,c}(g) * (h/2),
// the stochastic Galerkin convection N(w) w of eq. 3.7 / eq. 4.12 with the
// wind w = free velocity (full tensor) + Dirichlet lift ramp(t) e_1 g.
__global__ __launch_bounds__(64) void k_sg_convection(int nxi, int n_u, int ns, int nall,
                                                      const int* __restrict__ conn, const int* __restrict__ free_id,
                                                      const double* __restrict__ ufree,
                                                      const double* __restrict__ ramp,
                                                      const double* __restrict__ gall, const int* __restrict__ hrow,
                                                      const int* __restrict__ hl, const int* __restrict__ hk,
                                                      const double* __restrict__ hv, const double* __restrict__ ref,
                                                      double hh, double sign, double* __restrict__ out) {
  __shared__ double wl[9 * 2 * SGC_NXI];        // nodal wind [a][c][l]; later reused for C[g][c][i]
  __shared__ double Wq[9 * 2 * SGC_NXI];        // wind at Gauss points [g][c][l]
  __shared__ double Gq[9 * 4 * SGC_NXI];        // reference gradients [g][c][d][k]
  __shared__ double rt[252];
  __shared__ int nodes[9], fids[9];
  const int e = blockIdx.x, t = blockIdx.y, tid = threadIdx.x;
  for (int q = tid; q < 252; q += 64) rt[q] = ref[q];
  if (tid < 9) {
    nodes[tid] = conn[(long)e * 9 + tid];
    fids[tid] = free_id[nodes[tid]];
  }
  __syncthreads();
  const double* W = rt;
  const double* PHI = rt + 9;
  const double* DX = rt + 90;
  const double* DY = rt + 171;
  const double rmp = ramp[t];
  for (int o = tid; o < 18 * nxi; o += 64) {
    const int a = o / (2 * nxi), c = (o / nxi) % 2, l = o % nxi;
    const int f = fids[a];
    double v;
    if (f >= 0) v = ufree[((long)t * nxi + l) * n_u + (long)c * ns + f];
    else v = (l == 0) ? rmp * gall[(long)c * nall + nodes[a]] : 0.0;
    wl[(a * 2 + c) * SGC_NXI + l] = v;
  }
  __syncthreads();
  for (int o = tid; o < 18 * nxi; o += 64) {
    const int g = o / (2 * nxi), c = (o / nxi) % 2, l = o % nxi;
    double sv = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const double v = wl[(a * 2 + c) * SGC_NXI + l];
      sv = fma(PHI[g * 9 + a], v, sv);
      sx = fma(DX[g * 9 + a], v, sx);
      sy = fma(DY[g * 9 + a], v, sy);
    }
    Wq[(g * 2 + c) * SGC_NXI + l] = sv;
    Gq[((g * 2 + c) * 2 + 0) * SGC_NXI + l] = sx;
    Gq[((g * 2 + c) * 2 + 1) * SGC_NXI + l] = sy;
  }
  __syncthreads();
  double* Cq = wl;
  for (int o = tid; o < 18 * nxi; o += 64) {
    const int g = o / (2 * nxi), c = (o / nxi) % 2, i = o % nxi;
    const double* w0 = Wq + (g * 2 + 0) * SGC_NXI;
    const double* w1 = Wq + (g * 2 + 1) * SGC_NXI;
    const double* gx = Gq + ((g * 2 + c) * 2 + 0) * SGC_NXI;
    const double* gy = Gq + ((g * 2 + c) * 2 + 1) * SGC_NXI;
    double s = 0.0;
    for (int q = hrow[i]; q < hrow[i + 1]; ++q) {
      const int l = hl[q], k = hk[q];
      s = fma(hv[q], fma(w0[l], gx[k], w1[l] * gy[k]), s);
    }
    Cq[(g * 2 + c) * SGC_NXI + i] = s;
  }
  __syncthreads();
  for (int o = tid; o < 18 * nxi; o += 64) {
    const int a = o / (2 * nxi), c = (o / nxi) % 2, i = o % nxi;
    const int f = fids[a];
    if (f < 0) continue;
    double s = 0.0;
#pragma unroll
    for (int g = 0; g < 9; ++g) s = fma(W[g] * PHI[g * 9 + a], Cq[(g * 2 + c) * SGC_NXI + i], s);
    atomicAdd(out + ((long)t * nxi + i) * n_u + (long)c * ns + f, sign * hh * s);
  }
}

// ------------------------------------------------------------------ block cyclic reduction
constexpr int BCR_MAXBS = 256;
static_assert(sizeof(BcrOpDesc) % 8 == 0, "descriptor layout");

// One pass of a block cyclic reduction solve.  Rows = scalar unknowns of one
// component; component z of a vector V with row stride ld starts at
// V + z*comp_rows*ld.  Each op (one output block, described by a BcrOpDesc
// so that a workgroup finds everything it needs in one load) computes
// out <- [B_out] + sum_t coef_t M_t V_t, where V_t is block t of B or of the
// solution X and the output goes to B (in place; no op of the pass reads a
// block the pass writes) or to X.  Every op spreads its row groups (rows
// [64 g, 64 g + 64), grid z) over workgroups and CB combined columns per
// workgroup (component-major: combined column j is column j % ncols of
// component j / ncols).  The products run on the FP64 matrix cores: wave w
// owns row tile 4g + w times CB/16 column tiles (v_mfma_f64_16x16x4: lane l
// supplies M[row l%16][k l/16] and V[k l/16][col l%16]; accumulator item v
// is row 4v + l/16); input tiles are staged in LDS.  Each block M_t is stored
// in that fragment order: row tile g, k-step q at off + (g*nq + q)*64 + l
// (nq = ceil(cols/4), zero-padded), so a wave reads one contiguous 512-byte
// run per k-step; the data array ends with BCR_DATA_PAD doubles of padding.
//
// Streaming variant, any block up to BCR_MAXBS rows: the M fragments of the
// next PF k-steps are in flight while the current ones are multiplied.
template <int CB, int PF>
__global__ __launch_bounds__(256) void k_bcr_stream(const BcrOpDesc* __restrict__ ops, int op0, int nops,
                                                    const double* __restrict__ data, double* __restrict__ B, long ldb,
                                                    double* __restrict__ X, long ldx, int ncols, int ncomp,
                                                    long comp_rows) {
  __shared__ double xs[BCR_MAXBS + 4][CB + 1];
  if ((int)blockIdx.x >= nops) return;   // grid padding (uniform per workgroup)
  const BcrOpDesc& d = ops[op0 + blockIdx.x];
  const int j0 = blockIdx.y * CB;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int lr = lane % 16, lk = lane / 16;
  const int r0 = d.r0, bo = d.bo;
  if ((int)blockIdx.z * 64 >= bo) return;   // uniform per workgroup
  const int rt = blockIdx.z * 4 + wave;
  const bool active = rt * 16 < bo;
  const int ctot = ncomp * ncols;
  auto addr = [&](int row, int j, long ld) -> long {
    const int comp = j / ncols, c = j - comp * ncols;
    return ((long)comp * comp_rows + row) * ld + c;
  };
  const bool to_x = d.flags & 2;
  double* out = to_x ? X : B;
  const long ldo = to_x ? ldx : ldb;
  constexpr int NCT = CB / 16;
  dbl4 acc[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) acc[ct] = dbl4{0.0, 0.0, 0.0, 0.0};
  if (active && (d.flags & 1)) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rt * 16 + 4 * v + lk, j = j0 + ct * 16 + lr;
        if (r < bo && j < ctot) acc[ct][v] = B[addr(r0 + r, j, ldb)];
      }
  }
  const int nterm = d.nterm;
  const int rtc = min(rt, (bo - 1) / 16);   // idle waves read a valid tile
  for (int t = 0; t < nterm; ++t) {
    const int i0 = d.in_r0[t], bi = d.in_bi[t];
    const int bi4 = (bi + 3) & ~3;
    const double* M = data + d.off[t] + (long)rtc * (bi4 / 4) * 64 + lane;   // fragment order
    const double coef = d.coef[t];
    const bool from_x = (d.in_x >> t) & 1;
    const double* src = from_x ? X : B;
    const long lds = from_x ? ldx : ldb;
    __syncthreads();
    for (int e = tid; e < bi4 * CB; e += blockDim.x) {
      const int k = e / CB, jj = e % CB, j = j0 + jj;
      xs[k][jj] = (k < bi && j < ctot) ? src[addr(i0 + k, j, lds)] : 0.0;
    }
    __syncthreads();
    if (!active) continue;
    // fragments past the block's end read the padding behind the data
    // array or the next block: in bounds, never multiplied
    double an[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) an[q] = M[q * 64];
    for (int k = 0; k < bi4; k += 4 * PF) {
      double a[PF];
#pragma unroll
      for (int q = 0; q < PF; ++q) a[q] = coef * an[q];
#pragma unroll
      for (int q = 0; q < PF; ++q) an[q] = M[(k / 4 + PF + q) * 64];
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int kr = k + 4 * q;
        if (kr >= bi4) break;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], xs[kr + lk][ct * 16 + lr], acc[ct], 0, 0, 0);
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rt * 16 + 4 * v + lk, j = j0 + ct * 16 + lr;
      if (r < bo && j < ctot) out[addr(r0 + r, j, ldo)] = acc[ct][v];
    }
}

// A term's matrix-core fragments: k-step q of the wave's row tile is 64
// contiguous doubles (fragment order); k-steps past the block's end read the
// padding behind the data array or the next block (in bounds, never
// multiplied).  Inlined by force, with the arrays by reference, so that they
// stay in registers.
template <int KM>
__device__ __forceinline__ void bcr_load_frag(const double* __restrict__ M, double (&m)[KM]) {
#pragma unroll
  for (int q = 0; q < KM; ++q) m[q] = M[q * 64];
}

// A term's input tile (rows of its block x CB combined columns) into
// registers, XPT values per thread, from X or B per the op's bits.
template <int CB, int XPT, int PER>
__device__ __forceinline__ void bcr_load_tile(const BcrOpDesc& d, int t, const double* B, long ldb, const double* X,
                                              long ldx, long comp_rows, int tid, const int (&xcomp)[PER],
                                              const int (&xcol)[PER], double (&xr)[XPT]) {
  const int i0 = d.in_r0[t], bi = d.in_bi[t];
  const bool from_x = (d.in_x >> t) & 1;
  const double* src = from_x ? X : B;
  const long lds = from_x ? ldx : ldb;
#pragma unroll
  for (int q = 0; q < XPT; ++q) {
    const int k = (tid + 256 * q) / CB, qc = q % PER;
    xr[q] = (k < bi && xcomp[qc] >= 0) ? src[((long)xcomp[qc] * comp_rows + i0 + k) * lds + xcol[qc]] : 0.0;
  }
}

// Latency variant for blocks of at most 4*KM rows: a term's whole M fragment
// (KM k-steps) and its input tile are loaded in one round trip.  With DB the
// next term's loads are in flight while the current term runs on the matrix
// cores (input tiles double-buffered in LDS, twice the registers); without,
// the registers are halved for occupancy on passes with many ops.
template <int CB, int KM, bool DB>
__global__ __launch_bounds__(256) void k_bcr_tile(const BcrOpDesc* __restrict__ ops, int op0, int nops,
                                                  const double* __restrict__ data, double* __restrict__ B, long ldb,
                                                  double* __restrict__ X, long ldx, int ncols, int ncomp,
                                                  long comp_rows) {
  constexpr int KR = 4 * KM;              // rows of the largest input block
  constexpr int XPT = KR * CB / 256;      // staged input values per thread
  constexpr int NCT = CB / 16;
  constexpr int NBUF = DB ? 2 : 1;
  // the column a thread stages repeats with period CB / gcd(256, CB) in q
  constexpr int PER = CB / (CB % 256 == 0 ? 256 : (CB & -CB) < 256 ? (CB & -CB) : 256);
  static_assert(KR * CB % 256 == 0, "tile must split evenly over the workgroup");
  static_assert(CB % 16 == 0 && (256 * PER) % CB == 0, "column period");
  __shared__ double xs[NBUF][KR][CB + 1];
  if ((int)blockIdx.x >= nops) return;   // grid padding (uniform per workgroup)
  const BcrOpDesc& d = ops[op0 + blockIdx.x];
  const int j0 = blockIdx.y * CB;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int lr = lane % 16, lk = lane / 16;
  const int r0 = d.r0, bo = d.bo;
  if ((int)blockIdx.z * 64 >= bo) return;   // uniform per workgroup
  const int rt = blockIdx.z * 4 + wave;
  const bool active = rt * 16 < bo;
  const int ctot = ncomp * ncols;
  const int rtc = min(rt, (bo - 1) / 16);   // idle waves read a valid tile
  // the combined columns this thread stages: component offset and column
  int xcomp[PER], xcol[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = j0 + (tid + 256 * q) % CB;
    xcomp[q] = j < ctot ? j / ncols : -1;
    xcol[q] = j < ctot ? j - xcomp[q] * ncols : 0;
  }
  const bool to_x = d.flags & 2;
  double* out = to_x ? X : B;
  const long ldo = to_x ? ldx : ldb;
  const int nterm = d.nterm;
  double mf[KM], xr[XPT];
  double mn[DB ? KM : 1];
  if (nterm > 0) {
    bcr_load_frag<KM>(data + d.off[0] + (long)rtc * ((d.in_bi[0] + 3) / 4) * 64 + lane, mf);
    bcr_load_tile<CB, XPT, PER>(d, 0, B, ldb, X, ldx, comp_rows, tid, xcomp, xcol, xr);
  }
  dbl4 acc[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) acc[ct] = dbl4{0.0, 0.0, 0.0, 0.0};
  if (active && (d.flags & 1)) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rt * 16 + 4 * v + lk, j = j0 + ct * 16 + lr;
        if (r < bo && j < ctot) {
          const int comp = j / ncols;
          acc[ct][v] = B[((long)comp * comp_rows + r0 + r) * ldb + (j - comp * ncols)];
        }
      }
  }
  for (int t = 0; t < nterm; ++t) {
    double(*xb)[CB + 1] = xs[DB ? (t & 1) : 0];
    if (!DB && t > 0) __syncthreads();   // the single buffer is free again
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int e = tid + 256 * q;
      xb[e / CB][e % CB] = xr[q];
    }
    __syncthreads();
    const int bi4 = (d.in_bi[t] + 3) & ~3;
    const double coef = d.coef[t];
    if (DB && t + 1 < nterm) {
      bcr_load_frag<DB ? KM : 1>(data + d.off[t + 1] + (long)rtc * ((d.in_bi[t + 1] + 3) / 4) * 64 + lane, mn);
      bcr_load_tile<CB, XPT, PER>(d, t + 1, B, ldb, X, ldx, comp_rows, tid, xcomp, xcol, xr);
    }
    if (active) {
#pragma unroll
      for (int q = 0; q < KM; ++q) {
        if (4 * q >= bi4) break;
        const double a = coef * mf[q];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xb[4 * q + lk][ct * 16 + lr], acc[ct], 0, 0, 0);
      }
    }
    if (DB) {
#pragma unroll
      for (int q = 0; q < KM; ++q) mf[q] = mn[DB ? q : 0];
    } else if (t + 1 < nterm) {
      bcr_load_frag<KM>(data + d.off[t + 1] + (long)rtc * ((d.in_bi[t + 1] + 3) / 4) * 64 + lane, mf);
      bcr_load_tile<CB, XPT, PER>(d, t + 1, B, ldb, X, ldx, comp_rows, tid, xcomp, xcol, xr);
    }
  }
  if (!active) return;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rt * 16 + 4 * v + lk, j = j0 + ct * 16 + lr;
      if (r < bo && j < ctot) {
        const int comp = j / ncols;
        out[((long)comp * comp_rows + r0 + r) * ldo + (j - comp * ncols)] = acc[ct][v];
      }
    }
}

// Operands of term t for one wave of the split-k variant: k-step q = wave +
// 4 s (s < KQ) of row tile rt, the M fragment (fragment order; k-steps past
// the term's end read the padding behind the data array or the next block, in
// bounds, never multiplied) and the input rows 4 q + lane / 16 in the B
// layout (rows past the block's end read its last row).
template <int KQ, int NCT>
__device__ __forceinline__ void bcr_split_load(const BcrOpDesc& d, int t, const double* __restrict__ data, int rt,
                                               int wave, int lk, int lane, const double* B, long ldb, const double* X,
                                               long ldx, const long (&cb_off)[NCT], const int (&cb_col)[NCT],
                                               double (&fa)[KQ], double (&fx)[KQ][NCT]) {
  const int i0 = d.in_r0[t], bi = d.in_bi[t];
  const int nq = (bi + 3) / 4;
  const double* M = data + d.off[t] + ((long)rt * nq + wave) * 64 + lane;
  const bool from_x = (d.in_x >> t) & 1;
  const double* src = from_x ? X : B;
  const long ld = from_x ? ldx : ldb;
#pragma unroll
  for (int s = 0; s < KQ; ++s) {
    fa[s] = M[(long)s * 256];
    const int k = min(4 * (wave + 4 * s) + lk, bi - 1);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) fx[s][ct] = src[(cb_off[ct] + i0 + k) * ld + cb_col[ct]];
  }
}

// Split-k variant (the default for blocks of up to 16 KQ rows): a workgroup
// computes one 16-row tile of an op (grid z) for CB combined columns, and its
// four waves share the k-steps of every term (wave w takes k-steps w, w + 4,
// ..., at most KQ per term).  Each wave loads its operands straight from
// memory (M fragments, input rows in the matrix-core B layout), TP terms per
// round trip, and the four partial products are added in LDS.  A wave's
// chain of dependent products is a quarter of the row-tile variants', and a
// small workgroup keeps many of them in flight per compute unit.  Input rows
// past a block's end are read at its last row (finite, multiplied by the zero
// padding of the fragment); k-steps past a term's end, and the last term
// loaded again where the last round of terms runs short, are multiplied by
// an exact zero.
template <int CB, int KQ, int TP>
__global__ __launch_bounds__(256) void k_bcr_split(const BcrOpDesc* __restrict__ ops, int op0, int nops,
                                                   const double* __restrict__ data, double* __restrict__ B, long ldb,
                                                   double* __restrict__ X, long ldx, int ncols, int ncomp,
                                                   long comp_rows) {
  constexpr int NCT = CB / 16;
  static_assert(CB % 16 == 0, "column tiles of 16");
  __shared__ double red[4][NCT * 256];
  if ((int)blockIdx.x >= nops) return;   // grid padding (uniform per workgroup)
  const BcrOpDesc& d = ops[op0 + blockIdx.x];
  const int rt = blockIdx.z;
  const int r0 = d.r0, bo = d.bo;
  if (rt * 16 >= bo) return;   // uniform per workgroup
  const int j0 = blockIdx.y * CB;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int lr = lane % 16, lk = lane / 16;
  const int ctot = ncomp * ncols;
  // this lane's B-operand columns, clamped to a valid one
  long cb_off[NCT];
  int cb_col[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int j = min(j0 + ct * 16 + lr, ctot - 1);
    const int comp = j / ncols;
    cb_off[ct] = (long)comp * comp_rows;
    cb_col[ct] = j - comp * ncols;
  }
  const int nterm = d.nterm;
  double a[TP][KQ], x[TP][KQ][NCT];
  dbl4 acc[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) acc[ct] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int t0 = 0; t0 < nterm; t0 += TP) {
#pragma unroll
    for (int u = 0; u < TP; ++u)
      bcr_split_load<KQ, NCT>(d, min(t0 + u, nterm - 1), data, rt, wave, lk, lane, B, ldb, X, ldx, cb_off, cb_col,
                              a[u], x[u]);
    __builtin_amdgcn_sched_barrier(0);   // keeps the round's loads ahead of its products
    // no branches between the loads and their use, so that every load of
    // the round is issued before the first product waits: k-steps past a
    // term's end and terms past the last one multiply an exact zero
#pragma unroll
    for (int u = 0; u < TP; ++u) {
      const int t = min(t0 + u, nterm - 1);
      const int nq = (d.in_bi[t] + 3) / 4;
      const double coef = (t0 + u < nterm) ? d.coef[t] : 0.0;
#pragma unroll
      for (int s = 0; s < KQ; ++s) {
        const double av = (wave + 4 * s < nq) ? coef * a[u][s] : 0.0;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, x[u][s][ct], acc[ct], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][(ct * 4 + v) * 64 + lane] = acc[ct][v];
  __syncthreads();
  const bool to_x = d.flags & 2;
  double* out = to_x ? X : B;
  const long ldo = to_x ? ldx : ldb;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    // thread tid sums accumulator item (ct, v = tid / 64, lane tid % 64)
    const int e = ct * 256 + tid, v = tid / 64, l = tid % 64;
    const int r = rt * 16 + 4 * v + l / 16, j = j0 + ct * 16 + l % 16;
    if (r < bo && j < ctot) {
      double sum = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
      const int comp = j / ncols, c = j - comp * ncols;
      if (d.flags & 1) sum += B[((long)comp * comp_rows + r0 + r) * ldb + c];
      out[((long)comp * comp_rows + r0 + r) * ldo + c] = sum;
    }
  }
}


// FP32 form of the split-k pass for the reduced-precision mean solve: blocks
// in the same fragment order as FP32 values, right-hand sides and solutions
// in FP32, products on v_mfma_f32_16x16x4f32 with FP32 accumulation (lane l
// supplies M[l%16][l/16] and V[l/16][l%16] as in FP64; accumulator item v is
// D[4(l/16) + v][l%16]).
template <int KQ, int NCT>
__device__ __forceinline__ void bcr_split_load32(const BcrOpDesc& d, int t, const float* __restrict__ data, int rt,
                                                 int wave, int lk, int lane, const float* B, long ldb, const float* X,
                                                 long ldx, const long (&cb_off)[NCT], const int (&cb_col)[NCT],
                                                 float (&fa)[KQ], float (&fx)[KQ][NCT]) {
  const int i0 = d.in_r0[t], bi = d.in_bi[t];
  const int nq = (bi + 3) / 4;
  const float* M = data + d.off[t] + ((long)rt * nq + wave) * 64 + lane;
  const bool from_x = (d.in_x >> t) & 1;
  const float* src = from_x ? X : B;
  const long ld = from_x ? ldx : ldb;
#pragma unroll
  for (int s = 0; s < KQ; ++s) {
    fa[s] = M[(long)s * 256];
    const int k = min(4 * (wave + 4 * s) + lk, bi - 1);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) fx[s][ct] = src[(cb_off[ct] + i0 + k) * ld + cb_col[ct]];
  }
}

template <int CB, int KQ, int TP>
__global__ __launch_bounds__(256) void k_bcr_split32(const BcrOpDesc* __restrict__ ops, int op0, int nops,
                                                     const float* __restrict__ data, float* __restrict__ B, long ldb,
                                                     float* __restrict__ X, long ldx, int ncols, int ncomp,
                                                     long comp_rows) {
  constexpr int NCT = CB / 16;
  static_assert(CB % 16 == 0, "column tiles of 16");
  __shared__ float red[4][NCT * 256];
  if ((int)blockIdx.x >= nops) return;   // grid padding (uniform per workgroup)
  const BcrOpDesc& d = ops[op0 + blockIdx.x];
  const int rt = blockIdx.z;
  const int r0 = d.r0, bo = d.bo;
  if (rt * 16 >= bo) return;   // uniform per workgroup
  const int j0 = blockIdx.y * CB;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int lr = lane % 16, lk = lane / 16;
  const int ctot = ncomp * ncols;
  long cb_off[NCT];
  int cb_col[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int j = min(j0 + ct * 16 + lr, ctot - 1);
    const int comp = j / ncols;
    cb_off[ct] = (long)comp * comp_rows;
    cb_col[ct] = j - comp * ncols;
  }
  const int nterm = d.nterm;
  float a[TP][KQ], x[TP][KQ][NCT];
  flt4 acc[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) acc[ct] = flt4{0.f, 0.f, 0.f, 0.f};
  for (int t0 = 0; t0 < nterm; t0 += TP) {
#pragma unroll
    for (int u = 0; u < TP; ++u)
      bcr_split_load32<KQ, NCT>(d, min(t0 + u, nterm - 1), data, rt, wave, lk, lane, B, ldb, X, ldx, cb_off, cb_col,
                                a[u], x[u]);
    __builtin_amdgcn_sched_barrier(0);   // keeps the round's loads ahead of its products
#pragma unroll
    for (int u = 0; u < TP; ++u) {
      const int t = min(t0 + u, nterm - 1);
      const int nq = (d.in_bi[t] + 3) / 4;
      const float coef = (t0 + u < nterm) ? (float)d.coef[t] : 0.f;
#pragma unroll
      for (int s = 0; s < KQ; ++s) {
        const float av = (wave + 4 * s < nq) ? coef * a[u][s] : 0.f;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, x[u][s][ct], acc[ct], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][(ct * 4 + v) * 64 + lane] = acc[ct][v];
  __syncthreads();
  const bool to_x = d.flags & 2;
  float* out = to_x ? X : B;
  const long ldo = to_x ? ldx : ldb;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    // thread tid sums accumulator item (ct, v = tid / 64, lane tid % 64)
    const int e = ct * 256 + tid, v = tid / 64, l = tid % 64;
    const int r = rt * 16 + 4 * (l / 16) + v, j = j0 + ct * 16 + l % 16;
    if (r < bo && j < ctot) {
      float sum = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
      const int comp = j / ncols, c = j - comp * ncols;
      if (d.flags & 1) sum += B[((long)comp * comp_rows + r0 + r) * ldb + c];
      out[((long)comp * comp_rows + r0 + r) * ldo + c] = sum;
    }
  }
}

// ------------------------------------------------------------------ blocked pivoted Cholesky
// state[0] = residual trace, [1] = target (delta^2), [2] = zero threshold,
// [3] = trace
__global__ __launch_bounds__(1024) void k_pc_init(int N, const double* __restrict__ S, double eps,
                                                  const double* normsq_in, double* normsq_out,
                                                  double* __restrict__ d, double* state) {
  __shared__ double sh[32];
  double tr = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double v = S[(long)i * N + i];
    v = v > 0.0 ? v : 0.0;
    d[i] = v;
    tr += v;
  }
  tr = block_sum(tr, sh);
  if (threadIdx.x == 0) {
    double nrm = normsq_in ? *normsq_in : tr;
    if (normsq_out) *normsq_out = tr;
    state[0] = tr;
    state[1] = 0.5 * eps * eps * nrm;
    state[2] = 64.0 * 2.220446049250313e-16 * tr;
    state[3] = tr;
  }
}

// Up to nsteps pivots on the current Schur complement S (earlier panels
// already subtracted): column t of the panel Lp (N x nsteps, column-major,
// ld N) = (S[:, p] - Lp[:, :t] Lp[p, :t]^T) / sqrt(d[p]).  Stops when the
// residual trace reaches the target or the largest pivot is numerically 0.
// out[0] = pivots taken, out[1] = 1 if finished.  Each thread keeps the
// Schur diagonal of its rows (i = tid + q * blockDim, q < PC_Q) in
// registers; one combined reduction per pivot yields both the next pivot
// and the residual trace (three workgroup barriers per pivot).
constexpr int PC_Q = 8;
__global__ __launch_bounds__(1024) void k_pc_panel(int N, const double* __restrict__ S, double* __restrict__ d,
                                                   double* __restrict__ Lp, int* __restrict__ piv, int nsteps,
                                                   double* state, int* out, double* kept) {
  __shared__ double shv[16], shs[16];
  __shared__ int shi[16];
  __shared__ double lp[64];
  __shared__ double s_bv, s_res;
  __shared__ int s_p;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int wv = tid / WAVE, ln = tid % WAVE, nwv = nth / WAVE;
  double dl[PC_Q];
#pragma unroll
  for (int q = 0; q < PC_Q; ++q) {
    const int i = tid + q * nth;
    dl[q] = (i < N) ? d[i] : 0.0;
  }
  const double target = state[1], zero_thr = state[2];
  double resid = state[0];
  int t = 0, done = 0;
  for (;; ++t) {
    // combined block reduction: argmax of the Schur diagonal and its sum
    double mv = -1.0, sm = 0.0;
    int mi = 0;
#pragma unroll
    for (int q = 0; q < PC_Q; ++q) {
      const int i = tid + q * nth;
      if (i < N) {
        sm += dl[q];
        if (dl[q] > mv) { mv = dl[q]; mi = i; }
      }
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const double ov = __shfl_down(mv, o, WAVE);
      const int oi = __shfl_down(mi, o, WAVE);
      sm += __shfl_down(sm, o, WAVE);
      if (ov > mv || (ov == mv && oi < mi)) { mv = ov; mi = oi; }
    }
    if (ln == 0) {
      shv[wv] = mv;
      shi[wv] = mi;
      shs[wv] = sm;
    }
    __syncthreads();
    if (tid == 0) {
      double bv = shv[0], tot = shs[0];
      int bi = shi[0];
      for (int q = 1; q < nwv; ++q) {
        tot += shs[q];
        if (shv[q] > bv || (shv[q] == bv && shi[q] < bi)) { bv = shv[q]; bi = shi[q]; }
      }
      s_bv = bv;
      s_p = bi;
      s_res = tot;
    }
    __syncthreads();
    const double bv = s_bv;
    const int p = s_p;
    if (t > 0) resid = s_res;   // the first pass keeps the trace handed in
    if (resid <= target) { done = 1; break; }
    if (t == nsteps) break;
    if (bv <= zero_thr || bv <= 0.0) { done = 1; break; }
    if (tid < t) lp[tid] = Lp[(long)tid * N + p];
    if (tid == 0) piv[t] = p;
    __syncthreads();
    const double l = sqrt(bv);
#pragma unroll
    for (int q = 0; q < PC_Q; ++q) {
      const int i = tid + q * nth;
      if (i >= N) continue;
      // S is symmetric: row p read coalesced
      const double v = S[(long)p * N + i] - col_combo(Lp, N, i, lp, 1, t);
      // rows already eliminated (zero Schur diagonal) have a zero Schur row
      const double li = (i == p) ? l : (dl[q] > 0.0 ? v / l : 0.0);
      Lp[(long)t * N + i] = li;
      const double dd = dl[q] - li * li;
      dl[q] = (i == p || dd < 0.0) ? 0.0 : dd;
    }
  }
#pragma unroll
  for (int q = 0; q < PC_Q; ++q) {
    const int i = tid + q * nth;
    if (i < N) d[i] = dl[q];
  }
  if (tid == 0) {
    state[0] = resid;
    out[0] = t;
    out[1] = done;
    if (kept) *kept = state[3] - resid;
  }
}

// (argmax of the Schur diagonal with the smallest index on ties, its sum)
// over a 1024-thread workgroup whose threads hold RQ diagonal entries each;
// two barriers, the result broadcast to every thread.
template <int RQ>
__device__ __forceinline__ void pc_reg_reduce(int N, const double (&dl)[RQ], double* shv, int* shi, double* shs,
                                              double* s_bv, int* s_p, double* s_res, double& bv, int& p,
                                              double& sum) {
  const int tid = threadIdx.x, wv = tid / WAVE, ln = tid % WAVE, nwv = blockDim.x / WAVE;
  double mv = -1.0, sm = 0.0;
  int mi = 0;
#pragma unroll
  for (int q = 0; q < RQ; ++q) {
    const int i = tid + q * 1024;
    if (i < N) {
      sm += dl[q];
      if (dl[q] > mv) {
        mv = dl[q];
        mi = i;
      }
    }
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const double ov = __shfl_down(mv, o, WAVE);
    const int oi = __shfl_down(mi, o, WAVE);
    sm += __shfl_down(sm, o, WAVE);
    if (ov > mv || (ov == mv && oi < mi)) {
      mv = ov;
      mi = oi;
    }
  }
  if (ln == 0) {
    shv[wv] = mv;
    shi[wv] = mi;
    shs[wv] = sm;
  }
  __syncthreads();
  if (tid == 0) {
    double b = shv[0], tot = shs[0];
    int bi = shi[0];
    for (int q = 1; q < nwv; ++q) {
      tot += shs[q];
      if (shv[q] > b || (shv[q] == b && shi[q] < bi)) {
        b = shv[q];
        bi = shi[q];
      }
    }
    *s_bv = b;
    *s_p = bi;
    *s_res = tot;
  }
  __syncthreads();
  bv = *s_bv;
  p = *s_p;
  sum = *s_res;
}

// Register-resident form of k_pc_panel (same contract, panels of at most PW
// pivots, N <= 1024 RQ): thread tid owns rows i = tid + 1024 q (q < RQ) and
// keeps their Schur diagonal and panel entries in registers, so a pivot
// column is its S row minus register dot products with the pivot row's
// panel entries, which the owner publishes in LDS.  The pivot loop is
// unrolled so that every register index is static.
template <int RQ, int PW>
__global__ __launch_bounds__(1024) void k_pc_panel_reg(int N, const double* __restrict__ S, double* __restrict__ d,
                                                       double* __restrict__ Lp, int* __restrict__ piv, int nsteps,
                                                       double* state, int* out, double* kept) {
  __shared__ double shv[16], shs[16];
  __shared__ int shi[16];
  __shared__ double lp[PW];
  __shared__ double s_bv, s_res;
  __shared__ int s_p;
  const int tid = threadIdx.x;
  double dl[RQ], lr[RQ][PW];
#pragma unroll
  for (int q = 0; q < RQ; ++q) {
    const int i = tid + q * 1024;
    dl[q] = (i < N) ? d[i] : 0.0;
#pragma unroll
    for (int c = 0; c < PW; ++c) lr[q][c] = 0.0;
  }
  const double target = state[1], zero_thr = state[2];
  double resid = state[0];
  int t_end = PW, done = 0;
  bool stopped = false;
#pragma unroll
  for (int t = 0; t < PW; ++t) {
    double bv, sum;
    int p;
    pc_reg_reduce<RQ>(N, dl, shv, shi, shs, &s_bv, &s_p, &s_res, bv, p, sum);
    if (t > 0) resid = sum;   // the first pass keeps the trace handed in
    if (resid <= target || t == nsteps || bv <= zero_thr || bv <= 0.0) {
      done = (t != nsteps || resid <= target) ? 1 : 0;
      t_end = t;
      stopped = true;
      break;
    }
    // the owner of row p publishes that row's panel entries
    if ((p & 1023) == tid) {
#pragma unroll
      for (int q = 0; q < RQ; ++q)
        if (q == (p >> 10)) {
#pragma unroll
          for (int c = 0; c < t; ++c) lp[c] = lr[q][c];
        }
    }
    if (tid == 0) piv[t] = p;
    __syncthreads();
    const double l = sqrt(bv);
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int i = tid + q * 1024;
      if (i < N) {
        // S is symmetric: row p read coalesced
        double v = S[(long)p * N + i];
#pragma unroll
        for (int c = 0; c < t; ++c) v = fma(-lr[q][c], lp[c], v);
        // rows already eliminated (zero Schur diagonal) have a zero Schur row
        const double li = (i == p) ? l : (dl[q] > 0.0 ? v / l : 0.0);
        lr[q][t] = li;
        const double dd = dl[q] - li * li;
        dl[q] = (i == p || dd < 0.0) ? 0.0 : dd;
      }
    }
  }
  if (!stopped) {
    // all PW pivots taken: the residual trace after the last one
    double bv, sum;
    int p;
    pc_reg_reduce<RQ>(N, dl, shv, shi, shs, &s_bv, &s_p, &s_res, bv, p, sum);
    resid = sum;
    done = resid <= target ? 1 : 0;
  }
#pragma unroll
  for (int q = 0; q < RQ; ++q) {
    const int i = tid + q * 1024;
    if (i < N) {
      d[i] = dl[q];
#pragma unroll
      for (int c = 0; c < PW; ++c)
        if (c < t_end) Lp[(long)c * N + i] = lr[q][c];
    }
  }
  if (tid == 0) {
    state[0] = resid;
    out[0] = t_end;
    out[1] = done;
    if (kept) *kept = state[3] - resid;
  }
}

// LP[a*k + c] = L[c*N + piv[a]]: the pivot rows of L (row-major k x k,
// lower triangular up to rounding)
__global__ void k_gather_pivot_rows(int N, int k, const double* __restrict__ L, const int* __restrict__ piv,
                                    double* __restrict__ LP) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)k * k) return;
  int a = e / k, c = e % k;
  LP[e] = (c <= a) ? L[(long)c * N + piv[a]] : 0.0;
}

// In place, per row i of F (column-major, ld N, nb <= 64 columns):
// F[i, :] <- F[i, :] T^{-1}, T = LP block (lower triangular, row-major ld).
__global__ __launch_bounds__(256) void k_skel_tri(int N, int nb, const double* __restrict__ T, int ldt,
                                                  double* __restrict__ F) {
  __shared__ double t[64 * 64];
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    int a = e / 64, c = e % 64;
    double v = 0.0;
    if (a < nb && c < nb) v = (c <= a) ? T[(long)a * ldt + c] : 0.0;
    else if (a == c) v = 1.0;
    t[e] = v;
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double f[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) f[c] = (c < nb) ? F[(long)c * N + i] : 0.0;
#pragma unroll
  for (int c = 63; c >= 0; --c) {
    double v = f[c];
#pragma unroll
    for (int a = c + 1; a < 64; ++a) v -= f[a] * t[a * 64 + c];
    f[c] = v / t[c * 64 + c];
  }
#pragma unroll
  for (int c = 0; c < 64; ++c)
    if (c < nb) F[(long)c * N + i] = f[c];
}

// out[a*ld + j] = in[piv[a]*ld_in + j]
__global__ void k_gather_rows(int k, int cols, const double* __restrict__ in, long ld_in, const int* __restrict__ piv,
                              double* __restrict__ out, long ld_out) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)k * cols) return;
  int a = e / cols, j = e % cols;
  out[(long)a * ld_out + j] = in[(long)piv[a] * ld_in + j];
}

// ------------------------------------------------------------------ small sequential kernels
__global__ void k_hessenberg_lsq(const double* H, int ld, int k, const double* beta, double* y, double* resid) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  extern __shared__ double sm[];
  double* Rm = sm;                 // (k+1) x k column-major, ld k+1
  double* g = sm + (k + 1) * k;    // k+1
  double* cs = g + (k + 1);        // k
  double* sn = cs + k;             // k
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= k; ++i) Rm[j * (k + 1) + i] = (i <= j + 1) ? H[(long)j * ld + i] : 0.0;
  for (int i = 0; i <= k; ++i) g[i] = 0.0;
  g[0] = *beta;
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < j; ++i) {
      double a = Rm[j * (k + 1) + i], b = Rm[j * (k + 1) + i + 1];
      Rm[j * (k + 1) + i] = cs[i] * a + sn[i] * b;
      Rm[j * (k + 1) + i + 1] = -sn[i] * a + cs[i] * b;
    }
    double a = Rm[j * (k + 1) + j], b = Rm[j * (k + 1) + j + 1];
    double r = hypot(a, b);
    double c = (r == 0.0) ? 1.0 : a / r, s = (r == 0.0) ? 0.0 : b / r;
    cs[j] = c;
    sn[j] = s;
    Rm[j * (k + 1) + j] = r;
    Rm[j * (k + 1) + j + 1] = 0.0;
    double ga = g[j], gb = g[j + 1];
    g[j] = c * ga + s * gb;
    g[j + 1] = -s * ga + c * gb;
  }
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= Rm[j * (k + 1) + i] * y[j];
    double d = Rm[i * (k + 1) + i];
    y[i] = (d != 0.0) ? s / d : 0.0;
  }
  if (resid) *resid = fabs(g[k]);
}

__global__ void k_mgs_coef(int k, const double* d, const double* GV, int ldg, double* Hcol, double* coef) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  coef[0] = 1.0;
  for (int i = 0; i < k; ++i) {
    double h = d[i];
    for (int j = 0; j < i; ++j) h -= Hcol[j] * GV[(long)j * ldg + i];
    Hcol[i] = h;
    coef[1 + i] = -h;
  }
}

}  // namespace

// ====================================================================== launchers
namespace {
// library-internal workspace for split-K partial sums, one per stream (work
// on one stream is ordered, so the buffer is reused safely); grown on demand
std::mutex g_splitk_mu;
std::unordered_map<hipStream_t, std::pair<double*, size_t>> g_splitk;
std::atomic<long> g_kernel_allocs{0};   // hipMalloc calls made here (workspaces, tuning copies)
double* splitk_ws(hipStream_t s, size_t n) {
  std::lock_guard<std::mutex> lk(g_splitk_mu);
  auto& e = g_splitk[s];
  if (n > e.second) {
    if (e.first) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(e.first);
    }
    e.first = nullptr;
    e.second = 0;
    ++g_kernel_allocs;
    if (hipMalloc(&e.first, n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      e.first = nullptr;
      return nullptr;
    }
    e.second = n;
  }
  return e.first;
}

__global__ void k_reduce_scaled(int nb, int m, int n, const double* __restrict__ ws, double alpha, double beta,
                                double* __restrict__ C, long sCi, long sCj) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long ne = (long)m * n;
  if (e >= ne) return;
  double sum = 0.0;
  for (int b = 0; b < nb; ++b) sum += ws[(long)b * ne + e];
  long i = e / n, j = e % n;
  double* cp = C + i * sCi + j * sCj;
  double v = alpha * sum;
  if (beta != 0.0) v += beta * (*cp);
  *cp = v;
}
}  // namespace

namespace {
thread_local int g_gemm_tag = GEMM_PLAIN;   // what gemm() is running, see GemmTagScope
using GemmKernel = void (*)(int, int, int, double, const double*, long, long, long, const double*, long, long, long,
                            double, double*, long, long, long, int, long);
GemmKernel gemm_kernel() {
  if (g_gemm_prec == GP_F64 && g_gemm_tag == GEMM_GRAM) return k_gemm<GP_F64, GEMM_GRAM>;
  if (g_gemm_prec == GP_F64 && g_gemm_tag == GEMM_PROJ) return k_gemm<GP_F64, GEMM_PROJ>;
  return g_gemm_prec == GP_F32 ? k_gemm<GP_F32> : (g_gemm_prec == GP_BF16 ? k_gemm<GP_BF16> : k_gemm<GP_F64>);
}
int gemm_class() {
  if (g_gemm_prec != GP_F64) return KC_GEMM_LOWP;
  return g_gemm_tag == GEMM_GRAM ? KC_GRAM : (g_gemm_tag == GEMM_PROJ ? KC_PROJ : KC_GEMM);
}
}  // namespace

long kernel_device_allocs() { return g_kernel_allocs.load(); }

// the split-K partial sums of one launch never exceed 256 chunks of at
// most 256 / chunks output tiles of 64 x 64
void splitk_reserve(hipStream_t s) {
  if (!splitk_ws(s, (size_t)256 * 64 * 64)) throw std::runtime_error("split-K workspace: device allocation failed");
}

void splitk_release(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_splitk_mu);
  auto it = g_splitk.find(s);
  if (it == g_splitk.end()) return;
  if (it->second.first) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(it->second.first);
  }
  g_splitk.erase(it);
}

GemmTagScope::GemmTagScope(int tag) : old(g_gemm_tag) { g_gemm_tag = tag; }
GemmTagScope::~GemmTagScope() { g_gemm_tag = old; }

void gemm(hipStream_t s, int batch, int m, int n, int k, double alpha, const double* A, long sAb, long sAi, long sAk,
          const double* B, long sBb, long sBk, long sBj, double beta, double* C, long sCb, long sCi, long sCj,
          int kstep, long klimit) {
  if (m <= 0 || n <= 0 || batch <= 0) return;
  const long tiles = (long)cdiv(m, TM) * cdiv(n, TN);
  if (batch == 1 && klimit == 0 && tiles <= 16 && k >= 384) {
    // small output, long reduction: split K over workgroups (chunks of at
    // least 128), then reduce
    long nch = std::min<long>(k / 128, 256 / tiles);
    long ne = (long)m * n;
    double* ws = nch > 1 ? splitk_ws(s, (size_t)(nch * ne)) : nullptr;
    if (ws) {
      long chunk = (k + nch - 1) / nch;
      nch = (k + chunk - 1) / chunk;
      dim3 grid(cdiv(n, TN), cdiv(m, TM), (unsigned)nch);
      {
        ProfScope ps(gemm_class(), s, 8.0 * ((double)k * (m + n) + (double)ne * nch), 2.0 * m * n * (double)k);
        auto kern = gemm_kernel();
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, m, n, (int)chunk, 1.0, A, chunk * sAk, sAi, sAk, B,
                           chunk * sBk, sBk, sBj, 0.0, ws, ne, (long)n, 1L, (int)chunk, (long)k);
      }
      hipLaunchKernelGGL(k_reduce_scaled, dim3(cdiv(ne, 256)), dim3(256), 0, s, (int)nch, m, n, ws, alpha, beta, C,
                         sCi, sCj);
      return;
    }
  }
  dim3 grid(cdiv(n, TN), cdiv(m, TM), batch);
  double kk = klimit > 0 ? (double)klimit : (double)k * batch;   // total reduction length
  double by = klimit > 0 ? 8.0 * (kk * (m + n) + (double)m * n * batch)
                         : 8.0 * batch * ((double)m * k + (double)k * n + (double)m * n * (beta != 0.0 ? 2 : 1));
  ProfScope ps(gemm_class(), s, by, 2.0 * m * n * kk);
  auto kern = gemm_kernel();
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, m, n, k, alpha, A, sAb, sAi, sAk, B, sBb, sBk, sBj, beta, C, sCb,
                     sCi, sCj, kstep, klimit);
}

void gemm_batched(hipStream_t s, int nb, const GemmDesc* d_desc, int max_m, int max_n) {
  if (nb <= 0 || max_m <= 0 || max_n <= 0) return;
  for (int b0 = 0; b0 < nb; b0 += 65535) {
    int n = std::min(65535, nb - b0);
    dim3 grid(cdiv(max_n, TN), cdiv(max_m, TM), n);
    ProfScope ps(KC_GEMM_PTR, s, 0.0, 0.0);
    auto kern = g_gemm_prec == GP_F32 ? k_gemm_ptr<GP_F32>
                                      : (g_gemm_prec == GP_BF16 ? k_gemm_ptr<GP_BF16> : k_gemm_ptr<GP_F64>);
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, d_desc + b0);
  }
}

void gemm_f32out(hipStream_t s, int m, int n, int k, const double* A, long sAi, long sAk, const double* B, long sBk,
                 long sBj, float* C, long sCi, long sCj) {
  if (m <= 0 || n <= 0) return;
  ProfScope ps(KC_GEMM, s, 8.0 * ((double)m * k + (double)k * n) + 4.0 * m * (double)n, 2.0 * m * n * (double)k);
  hipLaunchKernelGGL(k_gemm_f32out, dim3(cdiv(n, TN), cdiv(m, TM)), dim3(256), 0, s, m, n, k, A, sAi, sAk, B, sBk, sBj,
                     C, sCi, sCj);
}

void gemm_csplit(hipStream_t s, int m, int n, int k, const double* A, long sAi, long sAk, const double* B, long sBk,
                 long sBj, double* C, long sCi, int csplit, long sCt) {
  if (m <= 0 || n <= 0) return;
  if (csplit <= 0) throw std::runtime_error("gemm_csplit: column block must be positive");
  ProfScope ps(gemm_class(), s, 8.0 * ((double)m * k + (double)k * n + (double)m * n), 2.0 * m * n * (double)k);
  auto kern = g_gemm_prec == GP_F32 ? k_gemm_csplit<GP_F32, double>
                                    : (g_gemm_prec == GP_BF16 ? k_gemm_csplit<GP_BF16, double>
                                                              : k_gemm_csplit<GP_F64, double>);
  hipLaunchKernelGGL(kern, dim3(cdiv(n, TN), cdiv(m, TM)), dim3(256), 0, s, m, n, k, A, sAi, sAk, B, sBk, sBj, C, sCi,
                     csplit, sCt);
}

void gemm_csplit_f32out(hipStream_t s, int m, int n, int k, const double* A, long sAi, long sAk, const double* B,
                        long sBk, long sBj, float* C, long sCi, int csplit, long sCt) {
  if (m <= 0 || n <= 0) return;
  if (csplit <= 0) throw std::runtime_error("gemm_csplit: column block must be positive");
  ProfScope ps(KC_GEMM, s, 8.0 * ((double)m * k + (double)k * n) + 4.0 * m * (double)n, 2.0 * m * n * (double)k);
  hipLaunchKernelGGL((k_gemm_csplit<GP_F64, float>), dim3(cdiv(n, TN), cdiv(m, TM)), dim3(256), 0, s, m, n, k, A, sAi,
                     sAk, B, sBk, sBj, C, sCi, csplit, sCt);
}

void gram(hipStream_t s, long rows, int nx, int ny, const double* X, long sXr, long sXc, const double* Y, long sYr,
          long sYc, double* out, double* ws, size_t ws_doubles) {
  GemmPrecisionScope f64(GP_F64);   // Grams decide truncations: always FP64
  GemmTagScope tag(GEMM_GRAM);
  const long ne = (long)nx * ny;
  if (rows <= 0) {
    fill(s, out, ne, 0.0);
    return;
  }
  const long tiles = (long)cdiv(nx, TM) * cdiv(ny, TN);
  long nch = std::min<long>(rows / 128, 1024 / tiles);
  nch = std::min<long>(nch, (long)(ws_doubles / std::max<long>(ne, 1)));
  if (nch <= 1) {
    gemm(s, 1, nx, ny, (int)std::min<long>(rows, INT_MAX), 1.0, X, 0, sXc, sXr, Y, 0, sYr, sYc, 0.0, out, 0, ny, 1);
    return;
  }
  long chunk = (rows + nch - 1) / nch;
  nch = (rows + chunk - 1) / chunk;
  gemm(s, (int)nch, nx, ny, (int)chunk, 1.0, X, chunk * sXr, sXc, sXr, Y, chunk * sYr, sYr, sYc, 0.0, ws, ne, ny, 1,
       (int)chunk, rows);
  ProfScope ps(KC_REDUCE, s, 8.0 * (double)ne * (nch + 1), (double)ne * nch);
  hipLaunchKernelGGL(k_reduce_partials, dim3(cdiv(ne, 64)), dim3(256), 0, s, (int)nch, ne, ws, out);
}

void sumsq(hipStream_t s, const double* x, long n, double* out, double* ws, size_t ws_doubles) {
  int nb = (int)std::min<long>(std::min<long>(1024, (long)ws_doubles), std::max<long>(1, cdiv(n, 256)));
  hipLaunchKernelGGL(k_sumsq_stage1, dim3(nb), dim3(256), 0, s, x, n, ws);
  hipLaunchKernelGGL(k_sum_stage2, dim3(1), dim3(1024), 0, s, ws, nb, out);
}

void store_ranks(hipStream_t s, int* d, int r1, int r2) {
  hipLaunchKernelGGL(k_store_ranks, dim3(1), dim3(64), 0, s, d, r1, r2);
}

void fill(hipStream_t s, double* p, long n, double v) {
  if (n <= 0) return;
  unsigned nb = std::min<unsigned>(cdiv(n, 256), 8192);
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, p, n, v);
}

void copy2d(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst, long ldd, double alpha,
            const double* dscale, int inv) {
  long total = (long)rows * cols;
  if (total <= 0) return;
  unsigned nb = std::min<unsigned>(cdiv(total, 256), 8192);
  hipLaunchKernelGGL(k_copy2d, dim3(nb), dim3(256), 0, s, rows, cols, src, lds, dst, ldd, alpha, dscale, inv);
}

void transpose_copy_batched(hipStream_t s, int batch, int rows, int cols, const double* src, long sbatch, long lds,
                            double* dst, long dbatch, long ldd) {
  if (batch <= 0 || rows <= 0 || cols <= 0) return;
  if (batch > 65535) throw std::runtime_error("transpose_copy_batched: batch too large");
  const unsigned gx = (unsigned)cdiv(cols, 32);
  const unsigned gy = (unsigned)std::min<long>(cdiv(rows, 32), std::max<long>(1, 65536 / ((long)gx * batch)));
  hipLaunchKernelGGL((k_transpose_copy<double, double>), dim3(gx, std::max(1u, std::min(gy, 65535u)), batch), dim3(32, 8), 0, s, rows,
                     cols, src, lds, sbatch, dst, ldd, dbatch);
}

void block_copy_batched(hipStream_t s, const BlockCopy* d_descs, int n, int max_rows, int max_cols) {
  if (n <= 0 || max_rows <= 0 || max_cols <= 0) return;
  if (n > 65535 || cdiv(max_rows, 32) > 65535) throw std::runtime_error("block_copy_batched: grid too large");
  hipLaunchKernelGGL(k_block_copy, dim3((unsigned)cdiv(max_cols, 32), (unsigned)cdiv(max_rows, 32), n), dim3(32, 8), 0,
                     s, d_descs);
}

void transpose_copy(hipStream_t s, int rows, int cols, const double* src, long lds, double* dst, long ldd) {
  transpose_copy_batched(s, 1, rows, cols, src, 0, lds, dst, 0, ldd);
}

void transpose_widen_batched(hipStream_t s, int batch, int rows, int cols, const float* src, long sbatch, long lds,
                             double* dst, long dbatch, long ldd) {
  if (batch <= 0 || rows <= 0 || cols <= 0) return;
  if (batch > 65535) throw std::runtime_error("transpose_widen_batched: batch too large");
  const unsigned gx = (unsigned)cdiv(cols, 32);
  const unsigned gy = (unsigned)std::min<long>(cdiv(rows, 32), std::max<long>(1, 65536 / ((long)gx * batch)));
  hipLaunchKernelGGL((k_transpose_copy<float, double>), dim3(gx, std::max(1u, std::min(gy, 65535u)), batch),
                     dim3(32, 8), 0, s, rows, cols, src, lds, sbatch, dst, ldd, dbatch);
}

void transpose_widen(hipStream_t s, int rows, int cols, const float* src, long lds, double* dst, long ldd) {
  transpose_widen_batched(s, 1, rows, cols, src, 0, lds, dst, 0, ldd);
}

void ell_groups_build(int nrows, const int* rowptr, const int* col, std::vector<int>& row0, std::vector<int>& uptr,
                      std::vector<int>& ucols, std::vector<int>& lidx, std::vector<int>& rlen, int& umax) {
  row0.assign(1, 0);
  uptr.assign(1, 0);
  ucols.clear();
  lidx.assign((size_t)nrows * ELL_WIDTH, 0);
  rlen.assign(nrows, 0);
  umax = 0;
  std::vector<int> cur, next;
  int r = 0;
  while (r < nrows) {
    const int g0 = r;
    cur.clear();
    while (r < nrows && r - g0 < ELL_GROUP_ROWS) {
      if (rowptr[r + 1] - rowptr[r] > ELL_WIDTH) throw std::runtime_error("row longer than the padded width");
      next = cur;
      next.insert(next.end(), col + rowptr[r], col + rowptr[r + 1]);
      std::sort(next.begin(), next.end());
      next.erase(std::unique(next.begin(), next.end()), next.end());
      if ((int)next.size() > ELL_GROUP_UMAX) break;   // a new group starts at r
      cur.swap(next);
      ++r;
    }
    for (int q = g0; q < r; ++q) {
      const int n = rowptr[q + 1] - rowptr[q];
      rlen[q] = (n + ELL_CHUNK - 1) / ELL_CHUNK * ELL_CHUNK;
      for (int t = 0; t < n; ++t)
        lidx[(size_t)q * ELL_WIDTH + t] =
            (int)(std::lower_bound(cur.begin(), cur.end(), col[rowptr[q] + t]) - cur.begin());
    }
    ucols.insert(ucols.end(), cur.begin(), cur.end());
    row0.push_back(r);
    uptr.push_back((int)ucols.size());
    umax = std::max(umax, (int)cur.size());
  }
}

namespace {
template <typename T>
void ell_launch(hipStream_t s, int ncomp, int ics, int ocs, const EllGroups& G, const T* eval, const T* x, int ldx,
                int xcol0, int ncols, T* y, int ldy, int ycol0, T alpha, T beta) {
  // the chunk width keeps the staged rows within 64 KB of LDS
  const int cw = std::max(1, std::min(WAVE, (int)(65536 / (sizeof(T) * std::max(1, G.umax)))));
  const size_t lds = sizeof(T) * (size_t)std::max(1, G.umax) * std::min(cw, ncols);
  const unsigned nb = 8 * cdiv(G.ngroups, 8);
  hipLaunchKernelGGL((k_ell_grouped<T>), dim3(nb, ncomp), dim3(256), lds, s, G.ngroups, ics, ocs, G.row0, G.uptr,
                     G.ucols, G.lidx, G.rlen, eval, x, ldx, xcol0, ncols, cw, y, ldy, ycol0, alpha, beta);
}
}  // namespace

void ell_spmm(hipStream_t s, int nrows, int ncomp, int ics, int ocs, const EllGroups& G, const double* eval, long nnz,
              const double* x, int ldx, int xcol0, int ncols, double* y, int ldy, int ycol0, double alpha,
              double beta) {
  if (nrows <= 0 || ncols <= 0 || ncomp <= 0 || G.ngroups <= 0) return;
  // algorithmic: the matrix's nonzeros (column index and value) once, the
  // inputs once, the outputs written (and read when accumulated)
  const double by = 12.0 * nnz + 8.0 * ncomp * ((double)nrows * ncols) +
                    8.0 * ncomp * (double)nrows * ncols * (beta != 0.0 ? 2.0 : 1.0);
  ProfScope ps(KC_ELL, s, by, 2.0 * (double)nnz * ncomp * ncols);
  ell_launch<double>(s, ncomp, ics, ocs, G, eval, x, ldx, xcol0, ncols, y, ldy, ycol0, alpha, beta);
}

void ell_spmm32(hipStream_t s, int nrows, int ncomp, int ics, int ocs, const EllGroups& G, const float* eval,
                long nnz, const float* x, int ldx, int xcol0, int ncols, float* y, int ldy, int ycol0, float alpha,
                float beta) {
  if (nrows <= 0 || ncols <= 0 || ncomp <= 0 || G.ngroups <= 0) return;
  const double by = 8.0 * nnz + 4.0 * ncomp * ((double)nrows * ncols) +
                    4.0 * ncomp * (double)nrows * ncols * (beta != 0.0f ? 2.0 : 1.0);
  ProfScope ps(KC_ELL, s, by, 2.0 * (double)nnz * ncomp * ncols);
  ell_launch<float>(s, ncomp, ics, ocs, G, eval, x, ldx, xcol0, ncols, y, ldy, ycol0, alpha, beta);
}

void spmm(hipStream_t s, int nrows, int ncomp, int ics, int ocs, const int* rowptr, const int* col, const double* vals,
          int nv, long vstride, const double* x, int ldx, int xcol0, int ncols, double* y, int ldy, int ycol0,
          int yvstep, double alpha, double beta, int max_row_nnz) {
  if (nrows <= 0 || ncols <= 0 || nv <= 0) return;
  if (nv == 1 && max_row_nnz > 0 && max_row_nnz <= 32) {
    const double nnz = (double)vstride > 0 ? (double)vstride : 0.0;
    const double by = 4.0 * (nrows + 1) + nnz * 12.0 + 8.0 * ncomp * ((double)std::max(ics, nrows) * ncols) +
                      8.0 * ncomp * (double)nrows * ncols * (beta != 0.0 ? 2.0 : 1.0);
    ProfScope ps(KC_SPMM, s, by, 2.0 * nnz * ncomp * ncols);
    hipLaunchKernelGGL(k_spmm_short<32>, dim3(cdiv(nrows, 4), ncomp), dim3(256), 0, s, nrows, ics, ocs, rowptr, col,
                       vals, x, ldx, xcol0, ncols, y, ldy, ycol0, alpha, beta);
    return;
  }
  for (int v0 = 0; v0 < nv; v0 += NVMAX) {
    int nvb = std::min(NVMAX, nv - v0);
    dim3 grid(cdiv(nrows, 4), ncomp);
    // algorithmic bytes: pattern + values once, each input row once, each output once
    double nnz = (double)vstride > 0 ? (double)vstride : 0.0;
    double by = 4.0 * (nrows + 1) + nnz * (4.0 + 8.0 * nvb) + 8.0 * ncomp * ((double)std::max(ics, nrows) * ncols) +
                8.0 * ncomp * (double)nrows * nvb * ncols;
    ProfScope ps(KC_SPMM, s, by, 2.0 * nnz * ncomp * nvb * ncols);
    hipLaunchKernelGGL(k_spmm, grid, dim3(256), 0, s, nrows, ics, ocs, rowptr, col, vals + v0 * vstride, nvb, vstride,
                       x, ldx, xcol0, ncols, y, ldy, ycol0 + v0 * yvstep, yvstep, alpha, beta);
  }
}

void core1_op(hipStream_t s, int kind, int n1, int r, const double* in, int ldi, double* out, int ldo, int col0,
              double scale, const double* dscale) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_core1_op, dim3(cdiv(r, 64)), dim3(64), 0, s, kind, n1, r, in, ldi, out, ldo, col0, scale,
                     dscale);
}

void core1_diag(hipStream_t s, int n1, int r, int k, const double* w, int ldw, const double* in, int ldi, double* out,
                int ldo, int col0) {
  long total = (long)n1 * k * r;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_core1_diag, dim3(cdiv(total, 256)), dim3(256), 0, s, n1, r, k, w, ldw, in, ldi, out, ldo, col0);
}

void core2_block(hipStream_t s, int r1, int n2, int r2, const double* in, const double* X, int k1, int k2, double* out,
                 int R1, int R2, int row0, int col0) {
  long total = (long)k1 * k2 * r1 * n2 * r2;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_core2_block, dim3(cdiv(total, 256)), dim3(256), 0, s, r1, n2, r2, in, X, k1, k2, out, R1, R2,
                     row0, col0);
}

void trunc_pc(hipStream_t s, int N, double* S, double eps, const double* normsq_in, double* normsq_out, double* U,
              int kmax, double* L, int* k_out, double* kept_out, int* info, int rank_bound, int large_ok,
              int* kp_out, double* state, int* piv_out) {
  static_assert(TRUNC_KSMALL == KSMALL, "truncation stage sizes");
  // dwork: N doubles placed after L (caller sizes L as N*kmax + N)
  double* dwork = L + (long)N * kmax;
  ProfScope ps(KC_TRUNC, s, 8.0 * (double)N * N, 0.0);
  hipLaunchKernelGGL(k_trunc_pc, dim3(1), dim3(TE_THREADS), 0, s, N, S, eps, normsq_in, normsq_out, U, kmax, L, dwork,
                     k_out, kept_out, info, rank_bound, large_ok, kp_out, state, piv_out);
}

void trunc_jacobi(hipStream_t s, int km, const int* kp_dev, const double* T, const double* state, double* W,
                  int* k_out, double* kept_out) {
  if (km < 1 || km > KSMALL) throw std::runtime_error("trunc_jacobi: size out of range");
  ProfScope ps(KC_TRUNC, s, 8.0 * 2.0 * km * km, 0.0);
  hipLaunchKernelGGL(k_trunc_jacobi, dim3(1), dim3(TE_THREADS), 0, s, km, kp_dev, T, state, W, k_out, kept_out);
}

void chol_inv_upper(hipStream_t s, int km, const int* kp_dev, const int* k_dev, const double* G, double* R,
                    int* info) {
  if (km < 1 || km > KSMALL) throw std::runtime_error("chol_inv_upper: size out of range");
  ProfScope ps(KC_TRUNC, s, 8.0 * 2.0 * km * km, (double)km * km * km / 2.0);
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, s, km, kp_dev, k_dev, G, R, info);
}

void take_basis(hipStream_t s, const int* kp_dev, const int* k_dev, int N, const double* X, int ldx, double* U,
                int kmax) {
  const unsigned nb = std::min<unsigned>(cdiv((long)N * ldx, 256), 1024);
  hipLaunchKernelGGL(k_take_basis, dim3(std::max(1u, nb)), dim3(256), 0, s, kp_dev, k_dev, N, X, ldx, U, kmax);
}



void pc_init(hipStream_t s, int N, const double* S, double eps, const double* normsq_in, double* normsq_out, double* d,
             double* state) {
  hipLaunchKernelGGL(k_pc_init, dim3(1), dim3(1024), 0, s, N, S, eps, normsq_in, normsq_out, d, state);
}

int pc_panel_width(int N) { return N <= 1024 ? 24 : N <= 2048 ? 16 : N <= 4096 ? 8 : 32; }

void pc_panel(hipStream_t s, int N, const double* S, double* d, double* Lp, int* piv, int nsteps, double* state,
              int* out, double* kept) {
  if (N > PC_Q * 1024 || nsteps > 64) throw std::runtime_error("pivoted Cholesky panel: size out of range");
  ProfScope ps(KC_TRUNC, s, 8.0 * (double)N * nsteps * 2, (double)N * nsteps * nsteps);
  if (N <= 4096 && nsteps <= pc_panel_width(N)) {
    // register-resident panel
    auto kern = N <= 1024 ? k_pc_panel_reg<1, 24> : N <= 2048 ? k_pc_panel_reg<2, 16> : k_pc_panel_reg<4, 8>;
    hipLaunchKernelGGL(kern, dim3(1), dim3(1024), 0, s, N, S, d, Lp, piv, nsteps, state, out, kept);
    return;
  }
  hipLaunchKernelGGL(k_pc_panel, dim3(1), dim3(1024), 0, s, N, S, d, Lp, piv, nsteps, state, out, kept);
}

void skeleton_factor(hipStream_t s, int N, int k, const double* L, const int* piv, double* LP, double* F) {
  if (k <= 0) return;
  ProfScope ps(KC_TRUNC, s, 8.0 * (3.0 * N * (double)k + (double)k * k), (double)N * k * k);
  long kk = (long)k * k;
  hipLaunchKernelGGL(k_gather_pivot_rows, dim3(cdiv(kk, 256)), dim3(256), 0, s, N, k, L, piv, LP);
  copy2d(s, k, N, L, N, F, N, 1.0, nullptr, 0);
  // column blocks of 64 from the right: F_J = (L_J - F_{>J} LP_{>J,J}) LP_JJ^{-1}
  const int nblk = cdiv(k, 64);
  for (int jb = nblk - 1; jb >= 0; --jb) {
    const int j0 = jb * 64, j1 = std::min(k, j0 + 64), nb = j1 - j0;
    if (j1 < k)
      gemm(s, 1, N, nb, k - j1, -1.0, F + (long)j1 * N, 0, 1, N, LP + (long)j1 * k + j0, 0, k, 1, 1.0,
           F + (long)j0 * N, 0, 1, N);
    hipLaunchKernelGGL(k_skel_tri, dim3(cdiv(N, 256)), dim3(256), 0, s, N, nb, LP + (long)j0 * k + j0, k,
                       F + (long)j0 * N);
  }
}

void gather_rows(hipStream_t s, int k, int cols, const double* in, long ld_in, const int* piv, double* out,
                 long ld_out) {
  long total = (long)k * cols;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(cdiv(total, 256)), dim3(256), 0, s, k, cols, in, ld_in, piv, out, ld_out);
}

void sg_convection_full(hipStream_t s, int nt, int nxi, int n_u, int ns, int nall, int nelem, const int* conn,
                        const int* free_id, const double* ufree, const double* ramp, const double* gall,
                        const int* hrow, const int* hl, const int* hk, const double* hv, const double* ref, double hh,
                        double sign, double* out) {
  if (nt <= 0 || nelem <= 0) return;
  ProfScope ps(KC_OTHER, s, 8.0 * 2.0 * nt * nxi * (double)n_u, 0.0);
  hipLaunchKernelGGL(k_sg_convection, dim3(nelem, nt), dim3(64), 0, s, nxi, n_u, ns, nall, conn, free_id, ufree,
                     ramp, gall, hrow, hl, hk, hv, ref, hh, sign, out);
}

namespace {
// the (CB, PF) variants of k_bcr_pass that the tuner chooses from
struct BcrVariant {
  int cb;
  int max_rows;   // largest block the variant takes
  int wg_rows;    // output rows per workgroup (grid z covers the largest block)
  decltype(&k_bcr_stream<32, 8>) fn;
};
const BcrVariant kBcrVariants[] = {
    {32, BCR_MAXBS, 64, k_bcr_stream<32, 8>},  {16, BCR_MAXBS, 64, k_bcr_stream<16, 8>},
    {32, BCR_MAXBS, 64, k_bcr_stream<32, 16>}, {16, 128, 64, k_bcr_tile<16, 32, true>},
    {32, 128, 64, k_bcr_tile<32, 32, true>},   {16, 128, 64, k_bcr_tile<16, 32, false>},
    {32, 128, 64, k_bcr_tile<32, 32, false>},  {16, 64, 64, k_bcr_tile<16, 16, true>},
    {32, 64, 64, k_bcr_tile<32, 16, true>},    {48, 128, 64, k_bcr_tile<48, 32, true>},
    {48, 128, 64, k_bcr_tile<48, 32, false>},  {80, 128, 64, k_bcr_tile<80, 32, false>},
    {16, 128, 16, k_bcr_split<16, 8, 1>},      {16, 128, 16, k_bcr_split<16, 8, 2>},
    {16, 128, 16, k_bcr_split<16, 8, 4>},      {32, 128, 16, k_bcr_split<32, 8, 1>},
    {32, 128, 16, k_bcr_split<32, 8, 2>},      {16, 256, 16, k_bcr_split<16, 16, 1>}};
constexpr int kNumBcrVariants = sizeof(kBcrVariants) / sizeof(kBcrVariants[0]);

// ev (npass + 1 events, optional) brackets every pass.  The profiler sees
// one scope per solve that counts every pass as a launch (algorithmic bytes
// of a pass: its block data once, the right-hand side rows it reads and
// writes).
void bcr_run(hipStream_t s, const BcrDev& f, const std::vector<int>& vars, int ncomp, double* B, long ldb, double* X,
             long ldx, int ncols, hipEvent_t* ev = nullptr) {
  // every pass needs a variant that takes the factor's largest block
  if ((int)vars.size() != f.npass) throw std::runtime_error("block cyclic reduction: variant list does not match");
  for (int v : vars)
    if (v < 0 || v >= kNumBcrVariants || f.maxbs > kBcrVariants[v].max_rows)
      throw std::runtime_error("block cyclic reduction: variant does not take the factor's blocks");
  const double cols = (double)ncomp * ncols;
  ProfScope ps(KC_BCR, s, 0.0, 0.0, 0);
  for (int p = 0; p < f.npass; ++p) {
    if (ev) (void)hipEventRecord(ev[p], s);
    const int o0 = f.pass_begin[p], no = f.pass_begin[p + 1] - o0;
    if (no <= 0) continue;
    const BcrVariant& v = kBcrVariants[vars[p]];
    ps.add(8.0 * (f.pass_data[p] + f.pass_rows[p] * cols), 2.0 * f.pass_mk[p] * cols, 1);
    // workgroup ids are dealt round-robin over the 8 XCDs; with the op index
    // padded to a multiple of 8, every column chunk and row group of an op
    // runs on the same XCD and shares its blocks through that XCD's L2
    const unsigned gx = 8 * cdiv(no, 8);
    hipLaunchKernelGGL(v.fn, dim3(gx, cdiv((long)ncomp * ncols, v.cb), cdiv(f.maxbs, v.wg_rows)), dim3(256), 0, s,
                       f.ops, o0, no, f.data, B, ldb, X, ldx, ncols, ncomp, (long)f.n);
  }
  if (ev) (void)hipEventRecord(ev[f.npass], s);
}

// time every variant on scratch copies of the right-hand side, pass by pass;
// keep the fastest variant of each pass
std::vector<int> bcr_tune(hipStream_t s, const BcrDev& f, int ncomp, const double* B, long ldb, int ncols) {
  const int np = f.npass;
  std::vector<int> best(np, 0);
  const long rows = (long)ncomp * f.n;
  double *b0 = nullptr, *bw = nullptr, *xw = nullptr;
  g_kernel_allocs += 3;
  if (hipMalloc(&b0, sizeof(double) * rows * ncols) != hipSuccess ||
      hipMalloc(&bw, sizeof(double) * rows * ncols) != hipSuccess ||
      hipMalloc(&xw, sizeof(double) * rows * ncols) != hipSuccess) {
    (void)hipGetLastError();
    for (double* p : {b0, bw, xw})
      if (p) (void)hipFree(p);
    return best;
  }
  copy2d(s, (int)rows, ncols, B, ldb, b0, ncols, 1.0, nullptr, 0);
  copy2d(s, (int)rows, ncols, b0, ncols, xw, ncols, 1.0, nullptr, 0);   // finite inputs for product passes
  std::vector<hipEvent_t> ev(np + 1);
  for (auto& e : ev) (void)hipEventCreate(&e);
  std::vector<float> best_ms(np, 1e30f);
  for (int v = 0; v < kNumBcrVariants; ++v) {
    if (f.maxbs > kBcrVariants[v].max_rows) continue;
    const std::vector<int> vv(np, v);
    std::vector<float> tot(np, 0.f);
    for (int rep = 0; rep < 3; ++rep) {
      copy2d(s, (int)rows, ncols, b0, ncols, bw, ncols, 1.0, nullptr, 0);
      bcr_run(s, f, vv, ncomp, bw, ncols, xw, ncols, ncols, ev.data());
      (void)hipEventSynchronize(ev[np]);
      if (rep == 0) continue;   // the first run warms the caches
      for (int p = 0; p < np; ++p) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[p], ev[p + 1]);
        tot[p] += ms;
      }
    }
    for (int p = 0; p < np; ++p)
      if (tot[p] < best_ms[p]) {
        best_ms[p] = tot[p];
        best[p] = v;
      }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  (void)hipStreamSynchronize(s);
  for (double* p : {b0, bw, xw}) (void)hipFree(p);
  if (std::getenv("SGTT_BCR_TUNE_LOG")) {
    // per pass: ops, terms, block data, the chosen variant and its time
    for (int p = 0; p < np; ++p)
      std::fprintf(stderr, "[bcr tune] n=%d cols=%d pass %d: ops %d, mk %.3g, data %.3g MB, rows %.3g -> variant %d "
                           "%.2f us\n",
                   f.n, ncomp * ncols, p, f.pass_begin[p + 1] - f.pass_begin[p], f.pass_mk[p], 8e-6 * f.pass_data[p],
                   f.pass_rows[p], best[p], best_ms[p] * 1e3 / 2);
  }
  return best;
}
}  // namespace

namespace {
// column counts share a choice per power-of-two bucket (ranks vary from call
// to call; the variants' ranking follows the column count slowly)
std::pair<int, int> bcr_choice_key(int ncomp, int ncols) {
  int bucket = 16;
  while (bucket < ncols) bucket *= 2;
  return std::make_pair(bucket, ncomp);
}
}  // namespace

void bcr_solve(hipStream_t s, const BcrDev& f, int ncomp, double* B, long ldb, double* X, long ldx, int ncols) {
  if (ncols <= 0 || f.npass == 0) return;
  if (f.maxbs > BCR_MAXBS) throw std::runtime_error("block cyclic reduction: block larger than 256");
  std::vector<int> vars;
  {
    if (!f.choices) throw std::runtime_error("block cyclic reduction: factor without a choice table");
    BcrChoices& ch = *f.choices;
    const auto key = bcr_choice_key(ncomp, ncols);
    std::unique_lock<std::mutex> lk(ch.mu);
    auto it = ch.by_key.find(key);
    if (it != ch.by_key.end()) {
      vars = it->second;
    } else {
      lk.unlock();
      const unsigned was = prof_mask();   // tuning runs are not profiled
      prof_enable_mask(0u);
      vars = bcr_tune(s, f, ncomp, B, ldb, ncols);
      prof_enable_mask(was);
      lk.lock();
      ch.by_key[key] = vars;
    }
  }
  bcr_run(s, f, vars, ncomp, B, ldb, X, ldx, ncols);
}

void bcr_solve_untuned(hipStream_t s, const BcrDev& f, int ncomp, double* B, long ldb, double* X, long ldx, int ncols,
                       int variant) {
  if (ncols <= 0 || f.npass == 0) return;
  if (f.maxbs > BCR_MAXBS) throw std::runtime_error("block cyclic reduction: block larger than 256");
  std::vector<int> vars;
  if (variant >= 0) {
    if (!bcr_variant_takes(f, variant))
      throw std::runtime_error("block cyclic reduction: blocks too large for the variant");
    vars.assign(f.npass, variant);
  } else {
    if (f.choices) {
      std::lock_guard<std::mutex> lk(f.choices->mu);
      auto it = f.choices->by_key.find(bcr_choice_key(ncomp, ncols));
      if (it != f.choices->by_key.end()) vars = it->second;
    }
    if (vars.empty()) {
      int v = 0;
      while (v < kNumBcrVariants && !bcr_variant_takes(f, v)) ++v;
      if (v == kNumBcrVariants) throw std::runtime_error("block cyclic reduction: no variant takes the blocks");
      vars.assign(f.npass, v);
    }
  }
  bcr_run(s, f, vars, ncomp, B, ldb, X, ldx, ncols);
}

// ---- FP32 passes of the reduced-precision mean solve
namespace {
struct BcrVariant32 {
  int cb;
  int max_rows;
  decltype(&k_bcr_split32<16, 8, 1>) fn;
};
const BcrVariant32 kBcrVariants32[] = {{16, 128, k_bcr_split32<16, 8, 1>},
                                       {16, 128, k_bcr_split32<16, 8, 2>},
                                       {32, 128, k_bcr_split32<32, 8, 1>},
                                       {16, 256, k_bcr_split32<16, 16, 1>}};
constexpr int kNumBcrVariants32 = sizeof(kBcrVariants32) / sizeof(kBcrVariants32[0]);

void bcr_run32(hipStream_t s, const BcrDev& f, const std::vector<int>& vars, int ncomp, float* B, long ldb, float* X,
               long ldx, int ncols, hipEvent_t* ev = nullptr) {
  if (!f.data32) throw std::runtime_error("block cyclic reduction: factor without FP32 blocks");
  if ((int)vars.size() != f.npass) throw std::runtime_error("block cyclic reduction: variant list does not match");
  for (int v : vars)
    if (v < 0 || v >= kNumBcrVariants32 || f.maxbs > kBcrVariants32[v].max_rows)
      throw std::runtime_error("block cyclic reduction: variant does not take the factor's blocks");
  const double cols = (double)ncomp * ncols;
  ProfScope ps(KC_BCR, s, 0.0, 0.0, 0);
  for (int p = 0; p < f.npass; ++p) {
    if (ev) (void)hipEventRecord(ev[p], s);
    const int o0 = f.pass_begin[p], no = f.pass_begin[p + 1] - o0;
    if (no <= 0) continue;
    const BcrVariant32& v = kBcrVariants32[vars[p]];
    ps.add(4.0 * (f.pass_data[p] + f.pass_rows[p] * cols), 2.0 * f.pass_mk[p] * cols, 1);
    const unsigned gx = 8 * cdiv(no, 8);   // op index padded to a multiple of 8 (XCD-aware, as in FP64)
    hipLaunchKernelGGL(v.fn, dim3(gx, cdiv((long)ncomp * ncols, v.cb), cdiv(f.maxbs, 16)), dim3(256), 0, s, f.ops, o0,
                       no, f.data32, B, ldb, X, ldx, ncols, ncomp, (long)f.n);
  }
  if (ev) (void)hipEventRecord(ev[f.npass], s);
}

std::vector<int> bcr_tune32(hipStream_t s, const BcrDev& f, int ncomp, const float* B, long ldb, int ncols) {
  const int np = f.npass;
  std::vector<int> best(np, 0);
  const long rows = (long)ncomp * f.n;
  float *b0 = nullptr, *bw = nullptr, *xw = nullptr;
  g_kernel_allocs += 3;
  if (hipMalloc(&b0, sizeof(float) * rows * ncols) != hipSuccess ||
      hipMalloc(&bw, sizeof(float) * rows * ncols) != hipSuccess ||
      hipMalloc(&xw, sizeof(float) * rows * ncols) != hipSuccess) {
    (void)hipGetLastError();
    for (float* p : {b0, bw, xw})
      if (p) (void)hipFree(p);
    return best;
  }
  (void)hipMemcpy2DAsync(b0, sizeof(float) * ncols, B, sizeof(float) * ldb, sizeof(float) * ncols, rows,
                         hipMemcpyDeviceToDevice, s);
  (void)hipMemcpyAsync(xw, b0, sizeof(float) * rows * ncols, hipMemcpyDeviceToDevice, s);
  std::vector<hipEvent_t> ev(np + 1);
  for (auto& e : ev) (void)hipEventCreate(&e);
  std::vector<float> best_ms(np, 1e30f);
  for (int v = 0; v < kNumBcrVariants32; ++v) {
    if (f.maxbs > kBcrVariants32[v].max_rows) continue;
    const std::vector<int> vv(np, v);
    std::vector<float> tot(np, 0.f);
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipMemcpyAsync(bw, b0, sizeof(float) * rows * ncols, hipMemcpyDeviceToDevice, s);
      bcr_run32(s, f, vv, ncomp, bw, ncols, xw, ncols, ncols, ev.data());
      (void)hipEventSynchronize(ev[np]);
      if (rep == 0) continue;
      for (int p = 0; p < np; ++p) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[p], ev[p + 1]);
        tot[p] += ms;
      }
    }
    for (int p = 0; p < np; ++p)
      if (tot[p] < best_ms[p]) {
        best_ms[p] = tot[p];
        best[p] = v;
      }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  (void)hipStreamSynchronize(s);
  for (float* p : {b0, bw, xw}) (void)hipFree(p);
  return best;
}
}  // namespace

void bcr_solve32(hipStream_t s, const BcrDev& f, int ncomp, float* B, long ldb, float* X, long ldx, int ncols) {
  if (ncols <= 0 || f.npass == 0) return;
  if (!f.choices) throw std::runtime_error("block cyclic reduction: factor without a choice table");
  std::vector<int> vars;
  BcrChoices& ch = *f.choices;
  auto key = bcr_choice_key(ncomp, ncols);
  key.second += 64;   // FP32 choices are kept apart from the FP64 ones
  std::unique_lock<std::mutex> lk(ch.mu);
  auto it = ch.by_key.find(key);
  if (it != ch.by_key.end()) {
    vars = it->second;
  } else {
    lk.unlock();
    const unsigned was = prof_mask();
    prof_enable_mask(0u);
    vars = bcr_tune32(s, f, ncomp, B, ldb, ncols);
    prof_enable_mask(was);
    lk.lock();
    ch.by_key[key] = vars;
  }
  lk.unlock();
  bcr_run32(s, f, vars, ncomp, B, ldb, X, ldx, ncols);
}

int bcr_variant_count() { return kNumBcrVariants; }

bool bcr_is_tuned(const BcrDev& f, int ncomp, int ncols, bool f32) {
  if (ncols <= 0 || f.npass == 0) return true;   // nothing to tune: bcr_solve returns at once
  if (!f.choices) return false;
  auto key = bcr_choice_key(ncomp, ncols);
  if (f32) key.second += 64;
  std::lock_guard<std::mutex> lk(f.choices->mu);
  return f.choices->by_key.count(key) != 0;
}

bool bcr_variant_takes(const BcrDev& f, int variant) {
  return variant >= 0 && variant < kNumBcrVariants && f.maxbs <= kBcrVariants[variant].max_rows;
}

void bcr_solve_variant(hipStream_t s, const BcrDev& f, int ncomp, double* B, long ldb, double* X, long ldx, int ncols,
                       int variant) {
  if (variant < 0 || variant >= kNumBcrVariants) throw std::runtime_error("block cyclic reduction: no such variant");
  if (f.maxbs > kBcrVariants[variant].max_rows)
    throw std::runtime_error("block cyclic reduction: blocks too large for the variant");
  if (ncols <= 0 || f.npass == 0) return;
  const std::vector<int> vv(f.npass, variant);
  bcr_run(s, f, vv, ncomp, B, ldb, X, ldx, ncols);
}


void hessenberg_lsq(hipStream_t s, const double* H, int ld, int k, const double* beta, double* y, double* resid) {
  size_t shm = sizeof(double) * ((size_t)(k + 1) * k + (k + 1) + 2 * k);
  hipLaunchKernelGGL(k_hessenberg_lsq, dim3(1), dim3(64), shm, s, H, ld, k, beta, y, resid);
}

void mgs_coef(hipStream_t s, int k, const double* d, const double* GV, int ldg, double* Hcol, double* coef) {
  hipLaunchKernelGGL(k_mgs_coef, dim3(1), dim3(64), 0, s, k, d, GV, ldg, Hcol, coef);
}

void scalar_op(hipStream_t s, int kind, const double* a, const double* b, double* out) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(1), 0, s, kind, a, b, out);
}

void dot_reduce(hipStream_t s, long n, const double* w, const double* k, double* out, int accumulate) {
  hipLaunchKernelGGL(k_dot_reduce, dim3(1), dim3(1024), 0, s, n, w, k, out, accumulate);
}

void scale_by(hipStream_t s, double* p, long n, const double* dscale, int inv) {
  if (n <= 0) return;
  unsigned nb = std::min<unsigned>(cdiv(n, 256), 8192);
  hipLaunchKernelGGL(k_scale_by, dim3(nb), dim3(256), 0, s, p, n, dscale, inv);
}

void sub_arrays(hipStream_t s, const double* a, const double* b, double* out, long n) {
  unsigned nb = std::min<unsigned>(cdiv(n, 256), 8192);
  hipLaunchKernelGGL(k_sub, dim3(nb), dim3(256), 0, s, a, b, out, n);
}

void check_finite(hipStream_t s, const double* x, long n, int* flag) {
  if (n <= 0) return;
  unsigned nb = std::min<unsigned>(cdiv(n, 256), 8192);
  hipLaunchKernelGGL(k_check_finite, dim3(nb), dim3(256), 0, s, x, n, flag);
}

}  // namespace sgtt
