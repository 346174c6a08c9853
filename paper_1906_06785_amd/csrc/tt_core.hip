// Tensor-train algebra on the device: concatenation (sums), inner products,
// Gram-based truncation T_eps, TT-SVD of full tensors, expansion.
//
// Truncation (eq. 4.5-4.7, Alg. 4.1 applied to a TT input) is done with Gram
// matrices of the unfoldings (the "Gram SVD" approach to TT rounding of
// Al Daas, Ballard and Benner, SISC 2022), which keeps the O(n3 R^2) work in
// two passes over core 3 (one Gram, one projection) and reduces the SVDs to
// eigen-decompositions of small symmetric matrices:
//   bond 1: S1 = G1 K2 G1^T with K2 = sum_i G2_i K3 G2_i^T, K3 = G3^T G3,
//   bond 2: S2 = C K3 C^T with C = (U1^T G1) x_1 G2 unfolded (k1 n2) x R2,
// each truncated with delta = eps ||z|| / sqrt(2) (eq. 4.7, d = 3).
#include "tt_core.h"

#include <algorithm>
#include <condition_variable>
#include <exception>
#include <mutex>
#include <thread>
#include <cstring>

namespace sgtt {

// ------------------------------------------------------------------ pool
Pool::~Pool() {
  for (auto& kv : size_) (void)hipFree(kv.first);
  if (arena_) (void)hipFree(arena_);
}

void Pool::reserve(size_t n) {
  if (!arena_size_.empty()) throw SgttError(-1, "reserve: blocks of the current arena are in use");
  if (arena_) {
    (void)hipFree(arena_);
    arena_ = nullptr;
    arena_n_ = 0;
    arena_free_.clear();
  }
  if (n == 0) return;
  n = (n + 255) / 256 * 256;
  double* p = nullptr;
  if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    throw SgttError(-3, "reserve: device allocation of the arena failed");
  }
  ++device_allocs_;
  arena_ = p;
  arena_n_ = n;
  arena_used_ = 0;
  arena_peak_ = 0;
  arena_free_[0] = n;
}

double* Pool::arena_get(size_t want) {
  for (auto it = arena_free_.begin(); it != arena_free_.end(); ++it) {
    if (it->second < want) continue;
    const size_t off = it->first, len = it->second;
    arena_free_.erase(it);
    if (len > want) arena_free_[off + want] = len - want;
    double* p = arena_ + off;
    arena_size_[p] = want;
    arena_used_ += want;
    arena_peak_ = std::max(arena_peak_, arena_used_);
    return p;
  }
  return nullptr;
}

bool Pool::arena_put(double* p) {
  auto it = arena_size_.find(p);
  if (it == arena_size_.end()) return false;
  size_t off = (size_t)(p - arena_), len = it->second;
  arena_size_.erase(it);
  arena_used_ -= len;
  // coalesce with the free neighbours
  auto next = arena_free_.lower_bound(off);
  if (next != arena_free_.end() && next->first == off + len) {
    len += next->second;
    next = arena_free_.erase(next);
  }
  if (next != arena_free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += len;
      return true;
    }
  }
  arena_free_[off] = len;
  return true;
}

double* Pool::get(size_t n) {
  if (n == 0) n = 1;
  size_t want = (n + 255) / 256 * 256;
  if (arena_) {
    double* p = arena_get(want);
    if (p) return p;
  }
  auto it = free_.lower_bound(want);
  if (it != free_.end() && it->first <= 2 * want + (1u << 20)) {
    double* p = it->second;
    free_.erase(it);
    return p;
  }
  double* p = nullptr;
  ++device_allocs_;
  hipError_t e = hipMalloc(&p, want * sizeof(double));
  if (e != hipSuccess) {
    // release cached blocks and retry once
    for (auto& kv : free_) {
      (void)hipFree(kv.second);
      held_ -= size_[kv.second] * sizeof(double);
      size_.erase(kv.second);
    }
    free_.clear();
    (void)hipGetLastError();
    e = hipMalloc(&p, want * sizeof(double));
    if (e != hipSuccess) throw SgttError(-3, "device allocation failed");
  }
  size_[p] = want;
  held_ += want * sizeof(double);
  return p;
}

void Pool::put(double* p) {
  if (!p) return;
  if (arena_ && arena_put(p)) return;
  auto it = size_.find(p);
  if (it == size_.end()) return;
  free_.insert({it->second, p});
}

TT& TT::operator=(TT&& o) noexcept {
  if (this != &o) {
    release();
    n1 = o.n1; n2 = o.n2; n3 = o.n3; r1 = o.r1; r2 = o.r2;
    c1 = o.c1; c2 = o.c2; c3 = o.c3; pool = o.pool;
    o.c1 = o.c2 = o.c3 = nullptr;
    o.pool = nullptr;
  }
  return *this;
}

void TT::release() {
  if (pool) {
    pool->put(c1);
    pool->put(c2);
    pool->put(c3);
  }
  c1 = c2 = c3 = nullptr;
  pool = nullptr;
}

Ctx::~Ctx() {
  side_release(*this);
  if (hint) (void)hipHostFree(hint);
  if (hdbl) (void)hipHostFree(hdbl);
}

// ---------------------------------------------------------------- side lane
void side_release(Ctx& c) {
  delete c.sol;
  c.sol = nullptr;
  delete c.side;
  c.side = nullptr;
}

long side_device_allocs(const Ctx& c) {
  long n = c.side ? c.side->c.pool.device_allocs() : 0;
  if (c.sol) n += c.sol->c.pool.device_allocs() + side_device_allocs(c.sol->c);
  return n;
}
long side_roundings(const Ctx& c) {
  long n = c.side ? c.side->c.roundings : 0;
  if (c.sol) n += c.sol->c.roundings + side_roundings(c.sol->c);
  return n;
}

void pair_run(Ctx& c, const std::function<TT(Ctx&)>& fu, const std::function<TT(Ctx&)>& fp, TT& out_u, TT& out_p) {
  if (!c.side_enabled) {
    out_u = fu(c);
    out_p = fp(c);
    return;
  }
  if (!c.side) c.side = new SideLane(c.device);
  SideLane& L = *c.side;
  const int prec = gemm_precision(GP_F64);
  gemm_precision(prec);
  const int region = prof_region(0);
  prof_region(region);
  SGTT_HIP(hipEventRecord(L.fork_ev, c.s));
  L.post([&L, &fp, prec, region]() {
    SGTT_HIP(hipStreamWaitEvent(L.c.s, L.fork_ev, 0));
    // the previous result was copied out on the main stream before this
    // job's fork point, so its memory may be reused from here on
    L.held.release();
    const int p0 = gemm_precision(prec);
    const int r0 = prof_region(region);
    try {
      L.held = fp(L.c);
    } catch (...) {
      gemm_precision(p0);
      prof_region(r0);
      throw;
    }
    gemm_precision(p0);
    prof_region(r0);
    SGTT_HIP(hipEventRecord(L.join_ev, L.c.s));
  });
  try {
    out_u = fu(c);
  } catch (...) {
    (void)L.wait();   // the side job refers to the caller's data: let it finish
    throw;
  }
  if (std::exception_ptr e = L.wait()) std::rethrow_exception(e);
  SGTT_HIP(hipStreamWaitEvent(c.s, L.join_ev, 0));
  out_p = tt_copy(c, L.held);
}

double* Ctx::scratch(size_t n) {
  if (n > ws_n) {
    if (ws) pool.put(ws);
    ws = pool.get(n);
    ws_n = n;
  }
  return ws;
}

double* Ctx::scratch2(size_t n) {
  if (n > ws2_n) {
    if (ws2) pool.put(ws2);
    ws2 = pool.get(n);
    ws2_n = n;
  }
  return ws2;
}

void Ctx::sync() {
  ++syncs;
  SGTT_HIP(hipStreamSynchronize(s));
}

TT tt_new(Ctx& c, int n1, int n2, int n3, int r1, int r2) {
  TT t;
  t.n1 = n1; t.n2 = n2; t.n3 = n3; t.r1 = r1; t.r2 = r2;
  t.pool = &c.pool;
  t.c1 = c.pool.get((size_t)n1 * r1);
  t.c2 = c.pool.get((size_t)r1 * n2 * r2);
  t.c3 = c.pool.get((size_t)n3 * r2);
  return t;
}

TT tt_view(int n1, int n2, int n3, int r1, int r2, double* c1, double* c2, double* c3) {
  TT t;
  t.n1 = n1; t.n2 = n2; t.n3 = n3; t.r1 = r1; t.r2 = r2;
  t.c1 = c1; t.c2 = c2; t.c3 = c3;
  return t;
}

TT tt_copy(Ctx& c, const TT& x) {
  TT t = tt_new(c, x.n1, x.n2, x.n3, x.r1, x.r2);
  SGTT_HIP(hipMemcpyAsync(t.c1, x.c1, sizeof(double) * x.n_c1(), hipMemcpyDeviceToDevice, c.s));
  SGTT_HIP(hipMemcpyAsync(t.c2, x.c2, sizeof(double) * x.n_c2(), hipMemcpyDeviceToDevice, c.s));
  SGTT_HIP(hipMemcpyAsync(t.c3, x.c3, sizeof(double) * x.n_c3(), hipMemcpyDeviceToDevice, c.s));
  return t;
}

// Block-copy descriptors to device memory (pool) and one launch for all of
// them; the pool returns the descriptor memory in stream order.
static void run_block_copies(Ctx& c, const std::vector<BlockCopy>& d) {
  if (d.empty()) return;
  int mr = 0, mc = 0;
  for (const auto& b : d) {
    mr = std::max(mr, b.rows);
    mc = std::max(mc, b.cols);
  }
  size_t nd = (d.size() * sizeof(BlockCopy) + sizeof(double) - 1) / sizeof(double);
  double* buf = c.pool.get(nd);
  SGTT_HIP(hipMemcpyAsync(buf, d.data(), d.size() * sizeof(BlockCopy), hipMemcpyHostToDevice, c.s));
  block_copy_batched(c.s, (const BlockCopy*)buf, (int)d.size(), mr, mc);
  c.pool.put(buf);
}

TT tt_concat(Ctx& c, const std::vector<const TT*>& xs, const double* dcoef, const std::vector<double>& hcoef) {
  const TT& x0 = *xs[0];
  int R1 = 0, R2 = 0;
  for (auto* x : xs) { R1 += x->r1; R2 += x->r2; }
  TT t = tt_new(c, x0.n1, x0.n2, x0.n3, R1, R2);
  fill(c.s, t.c2, t.n_c2(), 0.0);
  int o1 = 0, o2 = 0;
  std::vector<BlockCopy> place;
  for (size_t i = 0; i < xs.size(); ++i) {
    const TT& x = *xs[i];
    double hc = hcoef.empty() ? 1.0 : hcoef[i];
    place.push_back(BlockCopy{x.c1, t.c1 + o1, dcoef ? dcoef + i : nullptr, x.r1, R1, x.n1, x.r1, 0, 0, hc});
    core2_block(c.s, x.r1, x.n2, x.r2, x.c2, nullptr, 1, 1, t.c2, R1, R2, o1, o2);
    place.push_back(BlockCopy{x.c3, t.c3 + o2, nullptr, x.r2, R2, x.n3, x.r2, 0, 0, 1.0});
    o1 += x.r1;
    o2 += x.r2;
  }
  run_block_copies(c, place);
  return t;
}

void tt_dot(Ctx& c, const TT& x, const TT& y, double* dout, int acc, double* k3_out) {
  GemmPrecisionScope f64(GP_F64);   // inner products stay FP64
  const int n1 = x.n1, n2 = x.n2;
  const int a1 = x.r1, a2 = x.r2, b1 = y.r1, b2 = y.r2;
  double* W1 = c.pool.get((size_t)a1 * b1);
  double* Z = c.pool.get((size_t)a1 * n2 * b2);
  double* W2 = c.pool.get((size_t)a2 * b2);
  double* K3 = k3_out ? k3_out : c.pool.get((size_t)a2 * b2);
  // W1 = X1^T Y1
  gemm(c.s, 1, a1, b1, n1, 1.0, x.c1, 0, 1, a1, y.c1, 0, b1, 1, 0.0, W1, 0, b1, 1);
  // Z = W1 Y2 (flattened a1 x (n2 b2))
  gemm(c.s, 1, a1, n2 * b2, b1, 1.0, W1, 0, b1, 1, y.c2, 0, (long)n2 * b2, 1, 0.0, Z, 0, (long)n2 * b2, 1);
  // W2 = X2flat^T Zflat over (a, i)
  gemm(c.s, 1, a2, b2, a1 * n2, 1.0, x.c2, 0, 1, a2, Z, 0, b2, 1, 0.0, W2, 0, b2, 1);
  // K3 = X3^T Y3 over space
  size_t wsn = gram_ws_doubles(x.n3, a2, b2);
  gram(c.s, x.n3, a2, b2, x.c3, a2, 1, y.c3, b2, 1, K3, c.scratch(wsn), wsn);
  dot_reduce(c.s, (long)a2 * b2, W2, K3, dout, acc);
  c.pool.put(W1);
  c.pool.put(Z);
  c.pool.put(W2);
  if (!k3_out) c.pool.put(K3);
}

static void read_ints(Ctx& c, const int* d, int n, int* h) {
  SGTT_HIP(hipMemcpyAsync(c.hint, d, sizeof(int) * n, hipMemcpyDeviceToHost, c.s));
  c.sync();
  std::memcpy(h, c.hint, sizeof(int) * n);
}

// Truncation of the last bond when more than 96 pivots are needed: blocked
// pivoted Cholesky of the Gram S (N x N, overwritten by Schur complements)
// until the residual trace is <= eps^2 ||x||^2 / 2, then the skeleton factor
// F = L L_P^{-1}.  The tensor is replaced by F times its rows P, whose error
// equals the residual trace.  F: N x k column-major; piv: k ints.
struct Skeleton {
  int k = 0;
  double* F = nullptr;
  double* pivbuf = nullptr;
  const int* piv() const { return (const int*)pivbuf; }
  void release(Pool& p) {
    if (F) p.put(F);
    if (pivbuf) p.put(pivbuf);
    F = pivbuf = nullptr;
  }
};

// Blocked pivoted Cholesky with a skeleton factor.  With k0 > 0 it resumes
// from the first stage of trunc_sym: k0 pivots in L0 (column-major, ld N),
// their indices in c.dpiv, the remaining Schur diagonal d0 and the stage
// state (residual trace, target, zero threshold, trace) at c.dscal + 240.
static Skeleton trunc_skeleton(Ctx& c, int N, double* S, double eps, const double* dnorm_in, double* d_kept,
                               int kcap, int rank_bound, const char* what, const double* L0 = nullptr,
                               const double* d0 = nullptr, int k0 = 0) {
  GemmPrecisionScope f64(GP_F64);
  double* L = c.pool.get((size_t)N * kcap);
  double* d = c.pool.get((size_t)N + 8);
  double* state = d + N;
  Skeleton sk;
  sk.pivbuf = c.pool.get((size_t)kcap / 2 + 1);
  int* piv = (int*)sk.pivbuf;
  int* out = c.dint + 16;
  int k = 0;
  if (k0 > 0 && k0 <= kcap) {
    copy2d(c.s, k0, N, L0, N, L, N, 1.0, nullptr, 0);
    copy2d(c.s, 1, N, d0, N, d, N, 1.0, nullptr, 0);
    copy2d(c.s, 1, 4, c.dscal + 240, 4, state, 4, 1.0, nullptr, 0);
    SGTT_HIP(hipMemcpyAsync(piv, c.dpiv, sizeof(int) * k0, hipMemcpyDeviceToDevice, c.s));
    // Schur complement after those pivots
    gemm(c.s, 1, N, N, k0, -1.0, L, 0, 1, N, L, 0, N, 1, 1.0, S, 0, N, 1);
    k = k0;
  } else {
    pc_init(c.s, N, S, eps, dnorm_in, nullptr, d, state);
  }
  for (;;) {
    const int ns = std::min(pc_panel_width(N), kcap - k);
    if (ns <= 0) {
      if (kcap < rank_bound) {
        c.pool.put(L);
        c.pool.put(d);
        sk.release(c.pool);
        throw SgttError(-4, std::string("TT rank capacity exceeded (") + what + ")");
      }
      break;
    }
    pc_panel(c.s, N, S, d, L + (size_t)k * N, piv + k, ns, state, out, d_kept);
    int h[2];
    read_ints(c, out, 2, h);
    const int k0 = k;
    k += h[0];
    if (h[1] || h[0] == 0) break;
    // Schur complement update S -= L_panel L_panel^T
    gemm(c.s, 1, N, N, h[0], -1.0, L + (size_t)k0 * N, 0, 1, N, L + (size_t)k0 * N, 0, N, 1, 1.0, S, 0, N, 1);
  }
  if (k == 0) throw SgttError(-6, "internal: empty blocked truncation");
  sk.k = k;
  sk.F = c.pool.get((size_t)N * k);
  double* LP = c.pool.get((size_t)k * k);
  skeleton_factor(c.s, N, k, L, piv, LP, sk.F);
  c.pool.put(LP);
  c.pool.put(L);
  c.pool.put(d);
  return sk;
}

namespace {
// Truncated eigen-decomposition of a Gram matrix S (N x N): the staged
// routine behind every TT truncation (same contract as the stages in
// kernels.h).  The pivoted Cholesky and the small Jacobi eigen-solver run
// in one workgroup each; the products with L and the re-orthonormalization
// (Cholesky QR, twice) are GEMMs over the whole device, at the fixed width
// km = min(96, kmax) so that nothing waits for the host: the stages read the
// pivot count and the rank from device memory.  *info = 3 reports a failed
// Cholesky QR.
void trunc_sym(Ctx& c, int N, double* S, double eps, const double* normsq_in, double* normsq_out, double* U, int kmax,
               double* Lw, int* k_out, double* kept_out, int* info, int rank_bound, int large_ok = 0) {
  GemmPrecisionScope gp(GP_F64);
  constexpr int KS = TRUNC_KSMALL;
  const int km = std::min(KS, kmax);
  int* kp_dev = c.dint + 32;
  double* state = c.dscal + 240;
  if (!c.dpiv) c.dpiv = (int*)c.pool.get(KS / 2);
  trunc_pc(c.s, N, S, eps, normsq_in, normsq_out, U, kmax, Lw, k_out, kept_out, info, rank_bound, large_ok, kp_dev,
           state, c.dpiv);
  double* small = c.pool.get((size_t)4 * KS * KS);
  double *T = small, *W = small + KS * KS, *G = small + 2 * KS * KS, *R = small + 3 * KS * KS;
  double* U0 = c.pool.get((size_t)N * km);
  double* U1 = c.pool.get((size_t)N * km);
  gemm(c.s, 1, km, km, N, 1.0, Lw, 0, N, 1, Lw, 0, 1, N, 0.0, T, 0, KS, 1);   // T = L^T L
  trunc_jacobi(c.s, km, kp_dev, T, state, W, k_out, kept_out);
  gemm(c.s, 1, N, km, km, 1.0, Lw, 0, 1, N, W, 0, KS, 1, 0.0, U0, 0, 1, N);   // U0 = L W (column-major)
  // Cholesky QR twice: U1 = U0 R0 (column-major), U0 <- U1 R1 (row-major, ld km)
  gemm(c.s, 1, km, km, N, 1.0, U0, 0, N, 1, U0, 0, 1, N, 0.0, G, 0, KS, 1);
  chol_inv_upper(c.s, km, kp_dev, k_out, G, R, info);
  gemm(c.s, 1, N, km, km, 1.0, U0, 0, 1, N, R, 0, KS, 1, 0.0, U1, 0, 1, N);
  gemm(c.s, 1, km, km, N, 1.0, U1, 0, N, 1, U1, 0, 1, N, 0.0, G, 0, KS, 1);
  chol_inv_upper(c.s, km, kp_dev, k_out, G, R, info);
  gemm(c.s, 1, N, km, km, 1.0, U1, 0, 1, N, R, 0, KS, 1, 0.0, U0, 0, km, 1);
  take_basis(c.s, kp_dev, k_out, N, U0, km, U, kmax);
  c.pool.put(U0);
  c.pool.put(U1);
  c.pool.put(small);
}

double* upload_descs(Ctx& c, const std::vector<GemmDesc>& d) {
  size_t nd = (d.size() * sizeof(GemmDesc) + sizeof(double) - 1) / sizeof(double);
  double* buf = c.pool.get(nd);
  SGTT_HIP(hipMemcpyAsync(buf, d.data(), d.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, c.s));
  return buf;
}
}  // namespace

TT tt_round_sum(Ctx& c, const std::vector<Term>& terms, double eps, double* d_normsq, double* d_kept,
                const std::vector<const double*>* cache, int maxrank) {
  ++c.roundings;
  const int k = (int)terms.size();
  const TT& t0 = *terms[0].t;
  const int n1 = t0.n1, n2 = t0.n2, n3 = t0.n3;
  std::vector<int> a(k), b(k), oa(k + 1, 0), ob(k + 1, 0);
  for (int i = 0; i < k; ++i) {
    a[i] = terms[i].t->r1;
    b[i] = terms[i].t->r2;
    oa[i + 1] = oa[i] + a[i];
    ob[i + 1] = ob[i] + b[i];
  }
  const int R1 = oa[k], R2 = ob[k];
  // GEMM descriptor lists stay alive until the stream has been synchronized
  std::vector<GemmDesc> d1, d2, dC;
  int* dk = c.dint;   // [0]=k1 [1]=info1 [2]=k2 [3]=info2
  double* dnorm = d_normsq ? d_normsq : c.dscal + 250;
  double* dkept1 = c.dscal + 251;
  double* dkept2 = d_kept ? d_kept : c.dscal + 252;
  // Gram-forming products (K3, K2, S1, S2) run in FP64 whatever the ambient
  // precision; the projections (D, C, W, new core 3) use the ambient one.
  const int amb = gemm_precision(GP_F64);
  // ---- K3 = G3^T G3 (R2 x R2) assembled from blocks (cached or computed),
  // and G1 = [c_i A_i] (n1 x R1): every block placed by one batched copy
  double* K3 = c.pool.get((size_t)R2 * R2);
  double* G1 = c.pool.get((size_t)n1 * R1);
  std::vector<BlockCopy> place;
  double* gbuf = nullptr;
  if (k == 1 && !(cache && (*cache)[0])) {
    size_t wsn = gram_ws_doubles(n3, b[0], b[0]);
    gram(c.s, n3, b[0], b[0], terms[0].t->c3, b[0], 1, terms[0].t->c3, b[0], 1, K3, c.scratch(wsn), wsn);
  } else {
    size_t need = 0;
    for (int i = 0; i < k; ++i)
      for (int j = i; j < k; ++j)
        if (!(cache && (*cache)[(size_t)i * k + j])) need += (size_t)b[i] * b[j];
    gbuf = need ? c.pool.get(need) : nullptr;
    size_t off = 0;
    for (int i = 0; i < k; ++i)
      for (int j = i; j < k; ++j) {
        const double* src = cache ? (*cache)[(size_t)i * k + j] : nullptr;
        if (!src) {
          double* g = gbuf + off;
          off += (size_t)b[i] * b[j];
          size_t wsn = gram_ws_doubles(n3, b[i], b[j]);
          gram(c.s, n3, b[i], b[j], terms[i].t->c3, b[i], 1, terms[j].t->c3, b[j], 1, g, c.scratch(wsn), wsn);
          src = g;
        }
        place.push_back(BlockCopy{src, K3 + (size_t)ob[i] * R2 + ob[j], nullptr, b[j], R2, b[i], b[j], 0, 0, 1.0});
        if (j != i)
          place.push_back(
              BlockCopy{src, K3 + (size_t)ob[j] * R2 + ob[i], nullptr, b[j], R2, b[i], b[j], 1, 0, 1.0});
      }
  }
  for (int i = 0; i < k; ++i)
    place.push_back(BlockCopy{terms[i].t->c1, G1 + oa[i], terms[i].dcoef, a[i], R1, n1, a[i], 0, 0,
                              terms[i].hcoef});
  run_block_copies(c, place);
  if (gbuf) c.pool.put(gbuf);
  // ---- K2 (R1 x R1): K2_ij = sum_l B_i,l K3_ij B_j,l^T via T_ij = B_i K3_ij
  double* K2 = c.pool.get((size_t)R1 * R1);
  {
    std::vector<size_t> toff((size_t)k * k + 1, 0);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) toff[(size_t)i * k + j + 1] = toff[(size_t)i * k + j] + (size_t)a[i] * n2 * b[j];
    double* Tb = c.pool.get(toff[(size_t)k * k]);
    int mm1 = 0, nn1 = 0, mm2 = 0, nn2 = 0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        double* Tij = Tb + toff[(size_t)i * k + j];
        // T_ij (a_i n2 x b_j) = B_iflat (a_i n2 x b_i) * K3[ob_i.., ob_j..]
        d1.push_back(GemmDesc{a[i] * n2, b[j], b[i], 1.0, 0.0, terms[i].t->c2, b[i], 1,
                              K3 + (size_t)ob[i] * R2 + ob[j], R2, 1, Tij, b[j], 1});
        mm1 = std::max(mm1, a[i] * n2);
        nn1 = std::max(nn1, b[j]);
        // K2_ij (a_i x a_j) = T_ij' (a_i x n2 b_j) * B_j'^T (n2 b_j x a_j)
        d2.push_back(GemmDesc{a[i], a[j], n2 * b[j], 1.0, 0.0, Tij, (long)n2 * b[j], 1, terms[j].t->c2, 1,
                              (long)n2 * b[j], K2 + (size_t)oa[i] * R1 + oa[j], R1, 1});
        mm2 = std::max(mm2, a[i]);
        nn2 = std::max(nn2, a[j]);
      }
    double* dd1 = upload_descs(c, d1);
    gemm_batched(c.s, (int)d1.size(), (const GemmDesc*)dd1, mm1, nn1);
    double* dd2 = upload_descs(c, d2);
    gemm_batched(c.s, (int)d2.size(), (const GemmDesc*)dd2, mm2, nn2);
    c.pool.put(dd1);
    c.pool.put(dd2);
    c.pool.put(Tb);
  }
  // ---- S1 = G1 K2 G1^T (n1 x n1), truncate bond 1
  double* T1 = c.pool.get((size_t)n1 * R1);
  gemm(c.s, 1, n1, R1, R1, 1.0, G1, 0, R1, 1, K2, 0, R1, 1, 0.0, T1, 0, R1, 1);
  double* S1 = c.pool.get((size_t)n1 * n1);
  gemm(c.s, 1, n1, n1, R1, 1.0, T1, 0, R1, 1, G1, 0, 1, R1, 0.0, S1, 0, n1, 1);
  const int kmax1 = std::min({n1, R1, maxrank, RANK_CAP});
  double* U1 = c.pool.get((size_t)n1 * kmax1);
  {
    double* Lw = c.scratch2((size_t)n1 * kmax1 + n1 + 64);
    trunc_sym(c, n1, S1, eps, nullptr, dnorm, U1, kmax1, Lw, dk, dkept1, dk + 1, std::min(n1, R1));
  }
  int h[4];
  SGTT_HIP(hipMemcpyAsync(c.hint, dk, 2 * sizeof(int), hipMemcpyDeviceToHost, c.s));
  c.sync();
  h[0] = c.hint[0];
  h[1] = c.hint[1];
  if (h[1] == 3) throw SgttError(-1, "TT truncation: orthonormalization failed (bond 1)");
  if (h[1] != 0) throw SgttError(-4, "TT rank capacity exceeded (bond 1)");
  const int k1 = h[0];
  gemm_precision(amb);
  // ---- C (k1 n2 x R2): block j = (U1^T c_j A_j) x_1 B_j
  double* D = c.pool.get((size_t)k1 * R1);
  gemm(c.s, 1, k1, R1, n1, 1.0, U1, 0, 1, kmax1, G1, 0, R1, 1, 0.0, D, 0, R1, 1);
  double* Cm = c.pool.get((size_t)k1 * n2 * R2);
  {
    std::vector<GemmDesc>& d = dC;
    int mm = 0, nn = 0;
    for (int j = 0; j < k; ++j)
      for (int l = 0; l < n2; ++l) {
        d.push_back(GemmDesc{k1, b[j], a[j], 1.0, 0.0, D + oa[j], R1, 1, terms[j].t->c2 + (size_t)l * b[j],
                             (long)n2 * b[j], 1, Cm + (size_t)l * R2 + ob[j], (long)n2 * R2, 1});
        mm = std::max(mm, k1);
        nn = std::max(nn, b[j]);
      }
    double* dd = upload_descs(c, d);
    gemm_batched(c.s, (int)d.size(), (const GemmDesc*)dd, mm, nn);
    c.pool.put(dd);
  }
  const int N2 = k1 * n2;
  gemm_precision(GP_F64);
  // ---- S2 = C K3 C^T, truncate bond 2
  double* T2 = c.pool.get((size_t)N2 * R2);
  gemm(c.s, 1, N2, R2, R2, 1.0, Cm, 0, R2, 1, K3, 0, R2, 1, 0.0, T2, 0, R2, 1);
  double* S2 = c.pool.get((size_t)N2 * N2);
  gemm(c.s, 1, N2, N2, R2, 1.0, T2, 0, R2, 1, Cm, 0, 1, R2, 0.0, S2, 0, N2, 1);
  const int kmax2 = std::min({N2, R2, maxrank, RANK_CAP});
  double* U2 = c.pool.get((size_t)N2 * kmax2);
  double* Lw = c.scratch2((size_t)N2 * kmax2 + N2 + 64);   // first-stage pivots, kept for the blocked path
  const bool direct = N2 >= TRUNC_BLOCKED_N;
  if (direct) {
    h[2] = 0;
    h[3] = 2;
  } else {
    trunc_sym(c, N2, S2, eps, dnorm, nullptr, U2, kmax2, Lw, dk + 2, dkept2, dk + 3, std::min(N2, R2), 1);
    SGTT_HIP(hipMemcpyAsync(c.hint, dk + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, c.s));
    c.sync();
    h[2] = c.hint[0];
    h[3] = c.hint[1];
  }
  if (h[3] == 3) throw SgttError(-1, "TT truncation: orthonormalization failed (bond 2)");
  if (h[3] == 1) throw SgttError(-4, "TT rank capacity exceeded (bond 2)");
  Skeleton sk;
  if (h[3] == 2)
    sk = trunc_skeleton(c, N2, S2, eps, dnorm, dkept2, std::min({N2, R2, maxrank, RANK_CAP_LARGE}),
                        std::min(N2, R2), "bond 2", direct ? nullptr : Lw,
                        direct ? nullptr : Lw + (size_t)N2 * kmax2, direct ? 0 : TRUNC_KSMALL);
  const int k2 = h[3] == 2 ? sk.k : h[2];
  gemm_precision(amb);
  // ---- W (k2 x R2) = U2^T C, or the skeleton rows C[P, :]; new G3 = sum_j C_j W_j^T
  double* W = c.pool.get((size_t)k2 * R2);
  if (h[3] == 2)
    gather_rows(c.s, k2, R2, Cm, R2, sk.piv(), W, R2);
  else
    gemm(c.s, 1, k2, R2, N2, 1.0, U2, 0, 1, kmax2, Cm, 0, R2, 1, 0.0, W, 0, R2, 1);
  TT t = tt_new(c, n1, n2, n3, k1, k2);
  copy2d(c.s, n1, k1, U1, kmax1, t.c1, k1, 1.0, nullptr, 0);
  if (h[3] == 2)
    transpose_copy(c.s, k2, N2, sk.F, N2, t.c2, k2);
  else
    copy2d(c.s, N2, k2, U2, kmax2, t.c2, k2, 1.0, nullptr, 0);
  GemmTagScope proj(GEMM_PROJ);
  for (int j = 0; j < k; ++j)
    gemm(c.s, 1, n3, k2, b[j], 1.0, terms[j].t->c3, 0, b[j], 1, W + ob[j], 0, 1, R2, j == 0 ? 0.0 : 1.0, t.c3, 0,
         k2, 1);
  sk.release(c.pool);
  for (double* p : {K3, G1, K2, T1, S1, U1, D, Cm, T2, S2, U2, W}) c.pool.put(p);
  return t;
}

TT tt_round(Ctx& c, const TT& x, double eps, double* d_normsq, double* d_kept, int maxrank) {
  return tt_round_sum(c, {Term{&x, nullptr, 1.0}}, eps, d_normsq, d_kept, nullptr, maxrank);
}

TT tt_from_full(Ctx& c, const double* X, int n1, int n2, int n3, double eps, double* d_normsq, int maxrank) {
  ++c.roundings;
  const long n23 = (long)n2 * n3;
  int* dk = c.dint + 8;
  double* dnorm = d_normsq ? d_normsq : c.dscal + 249;
  double* dkept = c.dscal + 248;
  double* S1 = c.pool.get((size_t)n1 * n1);
  size_t wsn = gram_ws_doubles(n23, n1, n1);
  gram(c.s, n23, n1, n1, X, 1, n23, X, 1, n23, S1, c.scratch(wsn), wsn);
  const int kmax1 = std::min({n1, maxrank, RANK_CAP});
  double* U1 = c.pool.get((size_t)n1 * kmax1);
  double* Lw = c.scratch2((size_t)n1 * kmax1 + n1 + 64);
  trunc_sym(c, n1, S1, eps, nullptr, dnorm, U1, kmax1, Lw, dk, dkept, dk + 1, n1);
  int h[4];
  read_ints(c, dk, 2, h);
  if (h[1] == 3) throw SgttError(-1, "TT truncation: orthonormalization failed (full bond 1)");
  if (h[1] != 0) throw SgttError(-4, "TT rank capacity exceeded (full bond 1)");
  const int k1 = h[0];
  const int N2 = k1 * n2;
  double* Y = c.pool.get((size_t)k1 * n23);
  gemm(c.s, 1, k1, (int)std::min<long>(n23, INT32_MAX), n1, 1.0, U1, 0, 1, kmax1, X, 0, n23, 1, 0.0, Y, 0, n23, 1);
  double* S2 = c.pool.get((size_t)N2 * N2);
  size_t wsn2 = gram_ws_doubles(n3, N2, N2);
  gram(c.s, n3, N2, N2, Y, 1, n3, Y, 1, n3, S2, c.scratch(wsn2), wsn2);
  const int kmax2 = std::min({N2, maxrank, RANK_CAP});
  double* U2 = c.pool.get((size_t)N2 * kmax2);
  double* Lw2 = c.scratch2((size_t)N2 * kmax2 + N2 + 64);
  const bool direct = N2 >= TRUNC_BLOCKED_N;
  if (direct) {
    h[2] = 0;
    h[3] = 2;
  } else {
    trunc_sym(c, N2, S2, eps, dnorm, nullptr, U2, kmax2, Lw2, dk + 2, dkept, dk + 3, std::min(N2, n3), 1);
    read_ints(c, dk + 2, 2, h + 2);
  }
  if (h[3] == 3) throw SgttError(-1, "TT truncation: orthonormalization failed (full bond 2)");
  if (h[3] == 1) throw SgttError(-4, "TT rank capacity exceeded (full bond 2)");
  Skeleton sk;
  if (h[3] == 2)
    sk = trunc_skeleton(c, N2, S2, eps, dnorm, dkept, std::min({N2, n3, maxrank, RANK_CAP_LARGE}), std::min(N2, n3),
                        "full bond 2", direct ? nullptr : Lw2, direct ? nullptr : Lw2 + (size_t)N2 * kmax2,
                        direct ? 0 : TRUNC_KSMALL);
  const int k2 = h[3] == 2 ? sk.k : h[2];
  TT t = tt_new(c, n1, n2, n3, k1, k2);
  copy2d(c.s, n1, k1, U1, kmax1, t.c1, k1, 1.0, nullptr, 0);
  if (h[3] == 2) {
    transpose_copy(c.s, k2, N2, sk.F, N2, t.c2, k2);
    // G3 (n3 x k2) = rows P of Y(12), transposed
    double* YP = c.pool.get((size_t)k2 * n3);
    gather_rows(c.s, k2, n3, Y, n3, sk.piv(), YP, n3);
    transpose_copy(c.s, k2, n3, YP, n3, t.c3, k2);
    c.pool.put(YP);
  } else {
    copy2d(c.s, N2, k2, U2, kmax2, t.c2, k2, 1.0, nullptr, 0);
    // G3 (n3 x k2) = Y(12)^T U2_k
    GemmTagScope proj(GEMM_PROJ);
    gemm(c.s, 1, n3, k2, N2, 1.0, Y, 0, 1, n3, U2, 0, kmax2, 1, 0.0, t.c3, 0, k2, 1);
  }
  sk.release(c.pool);
  for (double* p : {S1, U1, Y, S2, U2}) c.pool.put(p);
  return t;
}

void tt_expand(Ctx& c, const TT& x, double* out) {
  const int n1 = x.n1, n2 = x.n2, n3 = x.n3, R1 = x.r1, R2 = x.r2;
  double* Lf = c.pool.get((size_t)n1 * n2 * R2);
  gemm(c.s, 1, n1, n2 * R2, R1, 1.0, x.c1, 0, R1, 1, x.c2, 0, (long)n2 * R2, 1, 0.0, Lf, 0, (long)n2 * R2, 1);
  gemm(c.s, 1, n1 * n2, n3, R2, 1.0, Lf, 0, R2, 1, x.c3, 0, 1, R2, 0.0, out, 0, n3, 1);
  c.pool.put(Lf);
}

void tt_scale3(Ctx& c, TT& x, const double* dscale, int inv) { scale_by(c.s, x.c3, x.n_c3(), dscale, inv); }

}  // namespace sgtt
