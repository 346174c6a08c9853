// Picard-step system, operator, mean-based LSC preconditioner, low-rank
// flexible GMRES with refinement, and the C ABI (include/sgtt.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <map>
#include <unordered_map>
#include <vector>

#include "../../include/sgtt.h"
#include "checkpoint.h"
#include "host_setup.h"
#include "kernels.h"
#include "learned.h"
#include "tt_core.h"

using namespace sgtt;

// ====================================================================== context
struct sgtt_context {
  int device = 0;
  bool own_stream = false;
  double* scratch = nullptr;   // this device's allocation-free scratch (device address)
  std::string err;
  Ctx c;
  // systems and networks made on this context and not yet destroyed; a
  // context destroyed before them is released when the last one goes
  std::mutex life_mu;
  int children = 0;
  bool closing = false;
};

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class T>
T* dev_upload(Ctx& c, const std::vector<T>& h) {
  T* p = nullptr;
  size_t n = std::max<size_t>(h.size(), 1);
  SGTT_HIP(hipMalloc(&p, n * sizeof(T)));
  if (!h.empty()) SGTT_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c.s));
  return p;
}

struct DevCsr {
  int nrows = 0, ncols = 0, nnz = 0, nv = 0;
  int max_row = 0;          // most entries in one row
  int *rowptr = nullptr, *col = nullptr;
  double* vals = nullptr;   // nv value arrays of nnz each
  void free_all() {
    (void)hipFree(rowptr);
    (void)hipFree(col);
    (void)hipFree(vals);
    rowptr = col = nullptr;
    vals = nullptr;
  }
};

DevCsr upload_csr(Ctx& c, const Csr& pat, const std::vector<const double*>& valsets) {
  DevCsr d;
  d.nrows = pat.nrows;
  d.ncols = pat.ncols;
  d.nnz = pat.nnz();
  d.nv = (int)valsets.size();
  for (int r = 0; r < pat.nrows; ++r) d.max_row = std::max(d.max_row, pat.rowptr[r + 1] - pat.rowptr[r]);
  d.rowptr = dev_upload(c, pat.rowptr);
  d.col = dev_upload(c, pat.col);
  std::vector<double> all((size_t)d.nnz * std::max(d.nv, 1));
  for (int v = 0; v < d.nv; ++v) std::copy(valsets[v], valsets[v] + d.nnz, all.begin() + (size_t)v * d.nnz);
  d.vals = dev_upload(c, all);
  return d;
}

void free_bcr(BcrDev& d) {
  for (void* p : {(void*)d.ops, (void*)d.data, (void*)d.data32})
    if (p) (void)hipFree(p);
  d = BcrDev();
}

// device form of a factor: one descriptor per op.  Pass modes: 0 forward
// reduction (inputs from B, output to B), 2 top system (inputs from B,
// output to X), 1 back substitution (own block from B, neighbours from X,
// output to X).
BcrDev upload_bcr(Ctx& c, const BcrFactor& f) {
  if (f.maxbs > 256) throw SgttError(-6, "block cyclic reduction: block larger than 256");
  if (BcrFactor::NT != BCR_NT) throw SgttError(-6, "block cyclic reduction: op layout mismatch");
  BcrDev d;
  d.n = f.n;
  d.nblk = f.nblk;
  d.maxbs = f.maxbs;
  d.npass = (int)f.pass_begin.size() - 1;
  d.pass_begin = f.pass_begin;
  d.ndata = (double)f.data.size();
  std::vector<BcrOpDesc> ops(f.op_out.size());
  std::vector<double> frag;                       // blocks in fragment order
  std::map<std::tuple<long, int, int>, long> placed;
  // blocks with bitwise equal contents are stored once (slabs of equal
  // geometry give equal blocks): content hash -> (offset, size) of each
  std::unordered_map<uint64_t, std::vector<std::pair<long, long>>> by_content;
  std::vector<double> tmp;
  long blocks_seen = 0, blocks_kept = 0;
  // rows x cols of a column-major matrix with ld rows starting at off
  auto place = [&](long off, int ld, int rows, int cols) -> long {
    const auto key = std::make_tuple(off, rows, cols);
    auto it = placed.find(key);
    if (it != placed.end()) return it->second;
    const long size = bcr_fragment_size(rows, cols);
    tmp.assign(size, 0.0);
    for (int k = 0; k < cols; ++k)
      for (int i = 0; i < rows; ++i) tmp[bcr_fragment_index(i, k, cols)] = f.data[off + (long)k * ld + i];
    uint64_t h = 1469598103934665603ull ^ ((uint64_t)rows << 32 | (uint32_t)cols);
    const unsigned char* by = reinterpret_cast<const unsigned char*>(tmp.data());
    for (size_t b = 0; b < sizeof(double) * tmp.size(); ++b) h = (h ^ by[b]) * 1099511628211ull;
    ++blocks_seen;
    auto& cand = by_content[h];
    for (const auto& oc : cand)
      if (oc.second == size && std::memcmp(frag.data() + oc.first, tmp.data(), sizeof(double) * size) == 0) {
        placed[key] = oc.first;
        return oc.first;
      }
    const long at = (long)frag.size();
    frag.insert(frag.end(), tmp.begin(), tmp.end());
    cand.emplace_back(at, size);
    ++blocks_kept;
    placed[key] = at;
    return at;
  };
  for (int p = 0; p < d.npass; ++p) {
    const int mode = f.pass_mode[p];
    if (mode < 0 || mode > 2) throw SgttError(-6, "block cyclic reduction: unknown pass mode");
    for (int o = f.pass_begin[p]; o < f.pass_begin[p + 1]; ++o) {
      BcrOpDesc& q = ops[o];
      q = BcrOpDesc();
      const int ob = f.op_out[o], ld = f.start[ob + 1] - f.start[ob];
      q.r0 = f.start[ob] + f.op_row0[o];
      q.bo = f.op_rows[o];
      q.nterm = f.op_nterm[o];
      if (q.nterm > BCR_NT) throw SgttError(-6, "block cyclic reduction: too many terms");
      q.flags = (f.op_self[o] ? 1 : 0) | (mode != 0 ? 2 : 0);
      for (int t = 0; t < q.nterm; ++t) {
        const int ib = f.op_in[BCR_NT * o + t], k0 = f.op_k0[BCR_NT * o + t];
        q.in_r0[t] = f.start[ib] + k0;
        q.in_bi[t] = f.op_kn[BCR_NT * o + t];
        q.off[t] = place(f.op_off[BCR_NT * o + t] + (long)k0 * ld + f.op_row0[o], ld, q.bo, q.in_bi[t]);
        q.coef[t] = f.op_coef[BCR_NT * o + t];
        if (mode == 1 && ib != ob) q.in_x |= 1 << t;
      }
    }
  }
  d.pass_mk.assign(d.npass, 0.0);
  d.pass_data.assign(d.npass, 0.0);
  d.pass_rows.assign(d.npass, 0.0);
  for (int p = 0; p < d.npass; ++p) {
    std::map<long, long> blocks;   // distinct blocks of the pass
    for (int o = f.pass_begin[p]; o < f.pass_begin[p + 1]; ++o) {
      const BcrOpDesc& q = ops[o];
      d.pass_rows[p] += q.bo * ((q.flags & 1) ? 2.0 : 1.0);
      for (int t = 0; t < q.nterm; ++t) {
        d.pass_mk[p] += (double)q.bo * q.in_bi[t];
        d.pass_rows[p] += q.in_bi[t];
        blocks[q.off[t]] = bcr_fragment_size(q.bo, q.in_bi[t]);
      }
    }
    for (const auto& b : blocks) d.pass_data[p] += (double)b.second;
  }
  if (std::getenv("SGTT_BCR_TUNE_LOG"))
    std::fprintf(stderr, "[bcr upload] n=%d: %ld blocks, %ld distinct, %.3g MB of block data\n", f.n, blocks_seen,
                 blocks_kept, 8e-6 * (double)frag.size());
  frag.resize(frag.size() + BCR_DATA_PAD, 0.0);
  d.ndata = (double)frag.size();
  d.ops = dev_upload(c, ops);
  d.data = dev_upload(c, frag);
  // the blocks once more in FP32 for the reduced-precision mean solve
  std::vector<float> frag32(frag.begin(), frag.end());
  d.data32 = dev_upload(c, frag32);
  return d;
}

// block cyclic reduction factor of a scalar matrix on pattern `pat`
BcrDev factor_bcr(Ctx& c, const Csr& pat, const double* vals, const std::vector<int>& blocks) {
  BcrFactor f;
  std::string err;
  bcr_factor(pat, vals, blocks, f, err);
  if (!err.empty()) throw SgttError(-6, err);
  return upload_bcr(c, f);
}

}  // namespace

// 1 / diag of a scalar matrix given by values on the pattern `pat`
std::vector<double> inverse_diagonal(const Csr& pat, const double* vals) {
  std::vector<double> d(pat.nrows, 0.0);
  for (int i = 0; i < pat.nrows; ++i)
    for (int t = pat.rowptr[i]; t < pat.rowptr[i + 1]; ++t)
      if (pat.col[t] == i) d[i] = vals[t] != 0.0 ? 1.0 / vals[t] : 0.0;
  return d;
}

// ====================================================================== system
struct sgtt_system {
  sgtt_context* ctx = nullptr;
  HostProblem hp;
  sgtt_problem_desc desc{};
  int nt = 0, nxi = 0, ns = 0, nu = 0, np = 0, nall = 0;
  double tau = 0, nu0 = 0;
  // operator data
  DevCsr Kop;       // free x free scalar pattern: [M, A_0..A_{nvisc-1}, N_1..N_k2] (operator)
  DevCsr Kmean;     // the same pattern: [M, A (unit), N_1..N_k2] (mean matrix, eq. 5.20-5.21)
  DevCsr Bd, Btd;   // B (n_p x n_u), B^T (n_u x n_p)
  DevCsr Xmid;      // pressure pattern: [XM, XA, XN_1..XN_k2]
  DevCsr Fp;        // Q1 pressure pattern: [M_p, A_p, N_p(w3_1)..N_p(w3_k2)] (PCD, eq. 5.17)
  DevCsr Mpinv;     // diag(M_p)^-1 as a diagonal CSR matrix (PCD)
  double* Gvisc = nullptr; // nvisc chaos matrices (n_xi x n_xi) of the viscous terms (eq. 3.6)
  int nvisc = 1;
  int k1 = 0, k2 = 0;      // convection TT-operator ranks (0: Stokes)
  double* w1 = nullptr;    // nt x k1
  double* Hw = nullptr;    // k1 x k2 x nxi x nxi
  double* omega = nullptr; // nt x k2 (mean-mode time factors)
  BcrDev Fbt, Xbt;         // F_avg and X = B M*^-1 B^T (block cyclic reduction)
  EllGroups Me_groups;     // M in padded-row form (time coupling of the mean solve)
  double* Me_val = nullptr;
  long Me_nnz = 0;         // nonzeros of M (its padded rows hold 32)
  float* Me_val32 = nullptr;   // the same values in FP32 (reduced-precision mean solve)
  TT bu, bp;               // right-hand side
  double* Dinv = nullptr;  // 1 / diag(F_avg) on free scalar nodes
  sgtt::Mlp* mlp_collect = nullptr;   // records (r, F_avg^-1 r) pairs from mean solves
  sgtt::Mlp* mlp_apply = nullptr;     // learned mean solve in M^-1 (eq. 5.23)
  std::vector<sgtt_iter_record> hist;   // the last solve's outer iterations
  bool mlp_off = false;               // fallback taken in the current solve
  int mlp_fails = 0, mlp_calls = 0;
  double rhs_norm = 0;     // ||f|| (Stokes) or ||r|| of the untruncated nonlinear residual (Picard)
  double setup_s = 0;
  // solve scratch (device scalars)
  double* dsc = nullptr;   // 32768 doubles: outer GMRES [0,16384), inner [16384,30000), residual [30000,)
  // graph of the mean solve's time loop (solve option graph = 1): the
  // full-tensor right-hand side and solution it runs on (FP64-sized, the
  // FP32 loop uses their first halves), one executable graph per arithmetic
  // [FP64, FP32], and the device allocations made for them
  double* mg_W = nullptr;
  double* mg_V = nullptr;
  hipGraphExec_t mg_exec[2] = {nullptr, nullptr};
  long mg_allocs = 0;
  long mg_launches = 0;
  ~sgtt_system() {
    for (hipGraphExec_t& e : mg_exec)
      if (e) (void)hipGraphExecDestroy(e);
    for (double* p : {mg_W, mg_V})
      if (p) (void)hipFree(p);
    if (mlp_collect) --mlp_collect->uses;
    if (mlp_apply) --mlp_apply->uses;
    Kop.free_all();
    Kmean.free_all();
    Bd.free_all();
    Btd.free_all();
    Xmid.free_all();
    Fp.free_all();
    Mpinv.free_all();
    free_bcr(Fbt);
    free_bcr(Xbt);
    for (void* p : {(void*)Me_groups.row0, (void*)Me_groups.uptr, (void*)Me_groups.ucols, (void*)Me_groups.lidx,
                    (void*)Me_groups.rlen, (void*)Me_val, (void*)Me_val32})
      if (p) (void)hipFree(p);
    for (double* p : {Gvisc, w1, Hw, omega, dsc, Dinv}) (void)hipFree(p);
  }
};

namespace {

// ---------------------------------------------------------------- operators
// L applied to (u, p): velocity part (eq. 3.12 with eq. 4.4 and eq. 4.12)
TT apply_velocity(sgtt_system& S, const TT& u, const TT& p, Ctx& c) {
  const int r1u = u.r1, r2u = u.r2, r1p = p.r1, r2p = p.r2, k1 = S.k1, k2 = S.k2, nv = S.nvisc;
  const int R1 = 2 * r1u + k1 * r1u + r1p, R2 = (1 + nv) * r2u + k2 * r2u + r2p;
  TT o = tt_new(c, S.nt, S.nxi, S.nu, R1, R2);
  // core 1: [(I - C)/tau u1 | u1 | diag(w1_a) u1 | p1]
  core1_op(c.s, 0, S.nt, r1u, u.c1, r1u, o.c1, R1, 0, 1.0 / S.tau);
  core1_op(c.s, 1, S.nt, r1u, u.c1, r1u, o.c1, R1, r1u, 1.0);
  if (k1) core1_diag(c.s, S.nt, r1u, k1, S.w1, k1, u.c1, r1u, o.c1, R1, 2 * r1u);
  core1_op(c.s, 1, S.nt, r1p, p.c1, r1p, o.c1, R1, 2 * r1u + k1 * r1u, 1.0);
  // core 2: blocks [u2 ; (Gv_0 u2 | .. | Gv_{nv-1} u2) ; (sum_l w2(a,l,b) H_l) u2 ; p2]
  // (the viscous terms share the time factor u1 of core 1)
  fill(c.s, o.c2, o.n_c2(), 0.0);
  core2_block(c.s, r1u, S.nxi, r2u, u.c2, nullptr, 1, 1, o.c2, R1, R2, 0, 0);
  core2_block(c.s, r1u, S.nxi, r2u, u.c2, S.Gvisc, 1, nv, o.c2, R1, R2, r1u, r2u);
  if (k1) core2_block(c.s, r1u, S.nxi, r2u, u.c2, S.Hw, k1, k2, o.c2, R1, R2, 2 * r1u, (1 + nv) * r2u);
  core2_block(c.s, r1p, S.nxi, r2p, p.c2, nullptr, 1, 1, o.c2, R1, R2, 2 * r1u + k1 * r1u,
              (1 + nv) * r2u + k2 * r2u);
  // core 3: [M u3 | A_0 u3 .. A_{nv-1} u3 | N_b u3 | B^T p3]
  spmm(c.s, S.ns, 2, S.ns, S.ns, S.Kop.rowptr, S.Kop.col, S.Kop.vals, 1 + nv + k2, S.Kop.nnz, u.c3, r2u, 0, r2u,
       o.c3, R2, 0, r2u, 1.0);
  spmm(c.s, S.nu, 1, 0, 0, S.Btd.rowptr, S.Btd.col, S.Btd.vals, 1, 0, p.c3, r2p, 0, r2p, o.c3, R2,
       (1 + nv) * r2u + k2 * r2u, 0, 1.0, 0.0, S.Btd.max_row);
  return o;
}

TT apply_pressure(sgtt_system& S, const TT& u, Ctx& c) {
  TT o = tt_new(c, S.nt, S.nxi, S.np, u.r1, u.r2);
  SGTT_HIP(hipMemcpyAsync(o.c1, u.c1, sizeof(double) * u.n_c1(), hipMemcpyDeviceToDevice, c.s));
  SGTT_HIP(hipMemcpyAsync(o.c2, u.c2, sizeof(double) * u.n_c2(), hipMemcpyDeviceToDevice, c.s));
  spmm(c.s, S.np, 1, 0, 0, S.Bd.rowptr, S.Bd.col, S.Bd.vals, 1, 0, u.c3, u.r2, 0, u.r2, o.c3, u.r2, 0, 0, 1.0);
  return o;
}

// on the context c (its stream and pool); the system's own by default
Vec apply_L(sgtt_system& S, const Vec& x, Ctx* cp = nullptr) {
  Ctx& c = cp ? *cp : S.ctx->c;
  Vec y;
  y.nc = 2;
  y.c[0] = apply_velocity(S, x.c[0], x.c[1], c);
  y.c[1] = apply_pressure(S, x.c[0], c);
  return y;
}

// Kronecker sum with the mean structure of eq. 5.20-5.21:
//   tau^-1 (I - C) (x) I (x) K_0 + nu0 I (x) I (x) K_1 + sum_b diag(omega_b) (x) I (x) K_{2+b}
// on a pattern with value sets [K_0, K_1, K_2..]: used for F_0 + C (velocity,
// two components) and for B M*^-1 (F_0 + C) M*^-1 B^T (pressure).
TT apply_mean_sum(sgtt_system& S, const TT& x, const DevCsr& K, int ncomp, int ncs) {
  Ctx& c = S.ctx->c;
  const int r1 = x.r1, r2 = x.r2, k2 = S.k2;
  const int R1 = (2 + k2) * r1, R2 = (2 + k2) * r2;
  TT o = tt_new(c, S.nt, S.nxi, x.n3, R1, R2);
  core1_op(c.s, 0, S.nt, r1, x.c1, r1, o.c1, R1, 0, 1.0 / S.tau);
  core1_op(c.s, 1, S.nt, r1, x.c1, r1, o.c1, R1, r1, S.nu0);
  if (k2) core1_diag(c.s, S.nt, r1, k2, S.omega, k2, x.c1, r1, o.c1, R1, 2 * r1);
  fill(c.s, o.c2, o.n_c2(), 0.0);
  for (int b = 0; b < 2 + k2; ++b) core2_block(c.s, r1, S.nxi, r2, x.c2, nullptr, 1, 1, o.c2, R1, R2, b * r1, b * r2);
  spmm(c.s, ncs, ncomp, ncs, ncs, K.rowptr, K.col, K.vals, 2 + k2, K.nnz, x.c3, r2, 0, r2, o.c3, R2, 0, r2, 1.0);
  return o;
}

// spatial solve along the space core: out = A^-1 x3 (ranks unchanged)
TT space_solve(sgtt_system& S, const TT& x, const BcrDev& bt, int ncomp, double c1scale) {
  Ctx& c = S.ctx->c;
  TT o = tt_new(c, x.n1, x.n2, x.n3, x.r1, x.r2);
  copy2d(c.s, x.n1, x.r1, x.c1, x.r1, o.c1, x.r1, c1scale, nullptr, 0);
  SGTT_HIP(hipMemcpyAsync(o.c2, x.c2, sizeof(double) * x.n_c2(), hipMemcpyDeviceToDevice, c.s));
  double* rhs = c.pool.get(x.n_c3());
  SGTT_HIP(hipMemcpyAsync(rhs, x.c3, sizeof(double) * x.n_c3(), hipMemcpyDeviceToDevice, c.s));
  bcr_solve(c.s, bt, ncomp, rhs, x.r2, o.c3, x.r2, x.r2);
  c.pool.put(rhs);
  return o;
}

// M^-1 = (I - C)^-1 (x) I (x) F_avg^-1 (eq. 5.23): prefix sum in time,
// F_avg solve on both velocity components of core 3
// With a learned mean solve attached (and no fallback taken), F_avg^-1 is
// replaced by D^-1 + ||r|| MLP(r/||r||) on every column; with a collector
// attached, the exact solve's (r, F_avg^-1 r) pairs are recorded.
TT apply_Minv(sgtt_system& S, const TT& u) {
  Ctx& c = S.ctx->c;
  TT o = tt_new(c, u.n1, u.n2, u.n3, u.r1, u.r2);
  core1_op(c.s, 2, S.nt, u.r1, u.c1, u.r1, o.c1, u.r1, 0, 1.0);
  SGTT_HIP(hipMemcpyAsync(o.c2, u.c2, sizeof(double) * u.n_c2(), hipMemcpyDeviceToDevice, c.s));
  if (S.mlp_apply && !S.mlp_off) {
    ++S.mlp_calls;
    try {
      mlp_apply(*S.mlp_apply, S.ns, 2, u.r2, u.c3, o.c3, u.r2, S.Dinv);
    } catch (const std::exception& e) {
      throw SgttError(-2, std::string("learned mean solve: ") + e.what());
    }
    return o;
  }
  double* rhs = c.pool.get(u.n_c3());
  SGTT_HIP(hipMemcpyAsync(rhs, u.c3, sizeof(double) * u.n_c3(), hipMemcpyDeviceToDevice, c.s));
  bcr_solve(c.s, S.Fbt, 2, rhs, u.r2, o.c3, u.r2, u.r2);
  c.pool.put(rhs);
  if (S.mlp_collect) {
    try {
      mlp_collect(*S.mlp_collect, S.ns, 2, u.r2, u.c3, o.c3, u.r2, S.Dinv);
    } catch (const std::exception& e) {
      throw SgttError(-2, std::string("collecting mean-solve pairs: ") + e.what());
    }
  }
  return o;
}

// ---------------------------------------------------------------- vector helpers
Vec vec_round(Ctx& c, const Vec& x, double eps, double* d_normsq, double* d_kept) {
  // d_normsq / d_kept: device arrays of 2 (per component), may be null
  Vec y;
  y.nc = x.nc;
  if (x.nc == 2) {
    pair_run(
        c,
        [&](Ctx& cc) { return tt_round(cc, x.c[0], eps, d_normsq, d_kept); },
        [&](Ctx& cc) {
          return tt_round(cc, x.c[1], eps, d_normsq ? d_normsq + 1 : nullptr, d_kept ? d_kept + 1 : nullptr);
        },
        y.c[0], y.c[1]);
    return y;
  }
  for (int i = 0; i < x.nc; ++i)
    y.c[i] = tt_round(c, x.c[i], eps, d_normsq ? d_normsq + i : nullptr, d_kept ? d_kept + i : nullptr);
  return y;
}

Vec vec_concat(Ctx& c, const std::vector<const Vec*>& xs, const double* dcoef, const std::vector<double>& hcoef) {
  Vec y;
  y.nc = xs[0]->nc;
  for (int i = 0; i < y.nc; ++i) {
    std::vector<const TT*> parts;
    for (auto* v : xs) parts.push_back(&v->c[i]);
    y.c[i] = tt_concat(c, parts, dcoef, hcoef);
  }
  return y;
}

void vec_dot(Ctx& c, const Vec& x, const Vec& y, double* dout) {
  for (int i = 0; i < x.nc; ++i) tt_dot(c, x.c[i], y.c[i], dout, i > 0);
}

Vec vec_copy(Ctx& c, const Vec& x) {
  Vec y;
  y.nc = x.nc;
  for (int i = 0; i < x.nc; ++i) y.c[i] = tt_copy(c, x.c[i]);
  return y;
}

Vec vec_scale3(Ctx& c, Vec&& x, const double* ds, int inv) {
  for (int i = 0; i < x.nc; ++i) tt_scale3(c, x.c[i], ds, inv);
  return std::move(x);
}

double read_double(Ctx& c, const double* d) {
  SGTT_HIP(hipMemcpyAsync(c.hdbl, d, sizeof(double), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return c.hdbl[0];
}

// ---------------------------------------------------------------- Alg. 4.2
struct Space {
  virtual Vec apply(const Vec&) = 0;
  virtual Vec precond(const Vec&) = 0;
  // the residual of the iterate the next precond serves, relative to the
  // right-hand side of the current solve
  virtual void note_residual(double) {}
  // the operator on another context (stream and pool); false (and y
  // untouched) if the space cannot run there
  virtual bool can_apply_on() const { return false; }
  virtual bool apply_on(const Vec&, Ctx&, Vec&) { return false; }
  virtual ~Space() = default;
};

struct SolveCounters {
  int inner = 0, outer = 0;
  int maxr_u = 0, maxr_p = 0;
  double t_apply = 0, t_round = 0, t_prec = 0;
  int verbose = 0;
  std::vector<sgtt_iter_record>* hist = nullptr;   // outer iterations of the solve
  int cycle = 0;
  double t_start = 0;
  int f32_applications = 0;   // relaxed precision: applications run in FP32
};

void hist_ranks(const Vec& v, int* u, int* p) {
  u[0] = v.c[0].r1;
  u[1] = v.c[0].r2;
  p[0] = v.nc > 1 ? v.c[1].r1 : 0;
  p[1] = v.nc > 1 ? v.c[1].r2 : 0;
}

// Core-3 Gram blocks of a growing basis, per TT component: blk(c, i, j) for
// i <= j holds basis_i.core3^T basis_j.core3 (device, pool-owned).
struct GramCache {
  Ctx* c = nullptr;
  int nc = 2, cap = 0;
  std::vector<double*> blk;   // [comp][i][j]
  GramCache(Ctx& ctx, int ncomp, int capacity) : c(&ctx), nc(ncomp), cap(capacity) {
    blk.assign((size_t)nc * cap * cap, nullptr);
  }
  double*& at(int comp, int i, int j) { return blk[((size_t)comp * cap + i) * cap + j]; }
  ~GramCache() {
    for (double* p : blk) c->pool.put(p);
  }
};

// Low-rank flexible GMRES (Alg. 4.2) with z_0 = 0.  dscal: device scratch of
// at least (maxit+1)*maxit + (maxit+1)^2 + 3*(maxit+1) + maxit + 16 doubles.
// explicit_res = true follows Alg. 4.2 literally (z_k and s_k = T(b - L z_k)
// every iteration); false stops on the least-squares residual estimate
// |rotated rhs| and forms z once at the end of the cycle.
// relax = true truncates the k-th Krylov basis vectors (x = T(L v^_k) and
// v_{k+1}) with eps_k = eps * min(||b|| / ||r_{k-1}||, eps_max / eps): the
// relaxation of inexact Krylov methods (Simoncini & Szyld 2003); z_k and s_k
// keep eps.  relax = false is the fixed truncation of Alg. 4.2.
Vec lowrank_fgmres(Ctx& c, Space& sp, const Vec& b, double tol, double eps, int maxit, double* dscal, int& iters,
                   double& relres, SolveCounters* cnt, const char* tag, bool explicit_res, bool relax = false,
                   double eps_max = 1e-2, double rhs_eps = 0.0) {
  const int ld = maxit + 1;
  const int nc = b.nc;
  const bool inner = std::strcmp(tag, "inner") == 0;
  const int rg_apply = inner ? RG_IN_APPLY : RG_OUT_APPLY, rg_mgs = inner ? RG_IN_MGS : RG_OUT_MGS,
            rg_sol = inner ? RG_IN_SOL : RG_OUT_SOL;
  RegionScope rg0(inner ? RG_IN_RHS : RG_OUT_SOL);
  double* H = dscal;                          // ld x maxit, column-major
  double* GV = H + (size_t)ld * maxit;        // ld x ld
  double* d = GV + (size_t)ld * ld;           // ld
  double* coef = d + ld;                      // ld + 1
  double* y = coef + ld + 1;                  // maxit
  double* sc = y + maxit;                     // 16 scalars
  fill(c.s, H, (long)ld * maxit, 0.0);
  // line 1: s_0 = T(b), beta = ||s_0||, v_1 = s_0 / beta
  Vec s = vec_round(c, b, rhs_eps > eps ? rhs_eps : eps, sc + 0, sc + 2);
  scalar_op(c.s, 0, sc + 0, nc > 1 ? sc + 1 : nullptr, sc + 4);   // ||b||
  scalar_op(c.s, 0, sc + 2, nc > 1 ? sc + 3 : nullptr, sc + 5);   // beta
  SGTT_HIP(hipMemcpyAsync(c.hdbl, sc + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, c.s));
  c.sync();
  const double bnorm = c.hdbl[0], beta = c.hdbl[1];
  iters = 0;
  relres = bnorm > 0 ? beta / bnorm : 0.0;
  std::vector<Vec> V, Vh;
  if (beta == 0.0) {
    Vec z = vec_copy(c, s);
    return z;
  }
  GramCache KV(c, nc, maxit + 1), KVh(c, nc, maxit + 1), KX(c, nc, maxit + 1);
  auto dot_cached = [&](const Vec& x, const Vec& yv, double* dout, GramCache& G, int i, int j) {
    for (int q = 0; q < nc; ++q) {
      double*& slot = G.at(q, i, j);
      if (!slot) slot = c.pool.get((size_t)x.c[q].r2 * yv.c[q].r2);
      tt_dot(c, x.c[q], yv.c[q], dout, q > 0, slot);
    }
  };
  V.push_back(vec_scale3(c, std::move(s), sc + 5, 1));
  dot_cached(V[0], V[0], GV, KV, 0, 0);
  Vec z;
  double res = beta;
  int k = 0;
  // z = T(sum_i y_i vh_i) of line 13, the pair's two components side by side
  auto solution_round = [&](Vec& zz) {
    auto one = [&](Ctx& cc, int q) {
      std::vector<Term> terms;
      std::vector<const double*> cache((size_t)k * k, nullptr);
      for (int i = 0; i < k; ++i) {
        terms.push_back(Term{&Vh[i].c[q], y + i, 1.0});
        for (int j = i; j < k; ++j) cache[(size_t)i * k + j] = KVh.at(q, i, j);
      }
      return tt_round_sum(cc, terms, eps, nullptr, nullptr, &cache);
    };
    if (nc == 2)
      pair_run(c, [&](Ctx& cc) { return one(cc, 0); }, [&](Ctx& cc) { return one(cc, 1); }, zz.c[0], zz.c[1]);
    else
      zz.c[0] = one(c, 0);
  };
  // With explicit residuals (lines 13-14 every iteration) on a pair, z_k,
  // L z_k and s_k run on the context's solution lane (its own stream, pool
  // and host thread) while this thread starts the next iteration's
  // preconditioner, which needs only v_{k+1}; the lane's residual then
  // decides whether that iteration happens.  Only when the least-squares
  // estimate is not yet near the tolerance, so that the speculative
  // preconditioner is rarely thrown away.
  SideLane* lane = nullptr;
  if (explicit_res && nc == 2 && c.side_enabled && sp.can_apply_on()) {
    if (!c.sol) {
      c.sol = new SideLane(c.device);
      c.sol->c.side_enabled = true;
    }
    lane = c.sol;
  }
  Vh.reserve(maxit + 1);   // the lane reads V and Vh: their storage must not move
  V.reserve(maxit + 2);
  Vec vh_pre;
  bool have_pre = false;
  while (res > tol * bnorm && k < maxit) {
    ++k;
    double t0 = now_s();
    Vec vh;
    if (have_pre) {
      vh = std::move(vh_pre);
      have_pre = false;
    } else {
      RegionScope rg(inner ? RG_IN_MINV : RG_LSC);
      sp.note_residual(res / bnorm);
      vh = sp.precond(V[k - 1]);
    }
    double t1 = now_s();
    if (cnt) cnt->t_prec += t1 - t0;
    const double eps_k = relax ? std::min(eps_max, eps * bnorm / std::max(res, 1e-300)) : eps;
    prof_region(rg_apply);
    Vec x = vec_round(c, sp.apply(vh), eps_k, nullptr, nullptr);
    prof_region(rg_mgs);
    Vh.push_back(std::move(vh));
    // Gram blocks of the preconditioned basis (for the solution sum); with
    // the solution lane they are computed there, only their memory is taken
    // here (from this context's pool, before the lane's fork point)
    auto vh_grams = [&](Ctx& cc) {
      for (int q = 0; q < nc; ++q)
        for (int i = 0; i < k; ++i) {
          const TT& ti = Vh[i].c[q];
          const TT& tj = Vh[k - 1].c[q];
          size_t wsn = gram_ws_doubles(ti.n3, ti.r2, tj.r2);
          gram(cc.s, ti.n3, ti.r2, tj.r2, ti.c3, ti.r2, 1, tj.c3, tj.r2, 1, KVh.at(q, i, k - 1), cc.scratch(wsn), wsn);
        }
    };
    for (int q = 0; q < nc; ++q)
      for (int i = 0; i < k; ++i)
        KVh.at(q, i, k - 1) = c.pool.get((size_t)Vh[i].c[q].r2 * Vh[k - 1].c[q].r2);
    if (!lane) vh_grams(c);
    // lines 6-9: modified Gram-Schmidt coefficients from <x, v_i> and the
    // Gram matrix of the basis (exact in exact arithmetic)
    for (int i = 0; i < k; ++i) {
      for (int q = 0; q < nc; ++q) {
        double*& slot = KX.at(q, 0, i);
        c.pool.put(slot);
        slot = c.pool.get((size_t)x.c[q].r2 * V[i].c[q].r2);
        tt_dot(c, x.c[q], V[i].c[q], d + i, q > 0, slot);
      }
    }
    mgs_coef(c.s, k, d, GV, ld, H + (size_t)(k - 1) * ld, coef);
    // line 10: h_{k+1,k} = ||x - sum h v||, v_{k+1} = T(x / h)
    Vec vn;
    vn.nc = nc;
    auto mgs_round = [&](Ctx& cc, int q) {
      std::vector<Term> terms{Term{&x.c[q], coef, 1.0}};
      std::vector<const double*> cache((size_t)(k + 1) * (k + 1), nullptr);
      for (int i = 0; i < k; ++i) {
        terms.push_back(Term{&V[i].c[q], coef + 1 + i, 1.0});
        cache[(size_t)0 * (k + 1) + 1 + i] = KX.at(q, 0, i);
        for (int j = i; j < k; ++j) cache[(size_t)(1 + i) * (k + 1) + 1 + j] = KV.at(q, i, j);
      }
      return tt_round_sum(cc, terms, eps_k, sc + 6 + q, nullptr, &cache);
    };
    if (nc == 2)
      pair_run(c, [&](Ctx& cc) { return mgs_round(cc, 0); }, [&](Ctx& cc) { return mgs_round(cc, 1); }, vn.c[0],
               vn.c[1]);
    else
      vn.c[0] = mgs_round(c, 0);
    scalar_op(c.s, 0, sc + 6, nc > 1 ? sc + 7 : nullptr, H + (size_t)(k - 1) * ld + k);   // h_{k+1,k}
    double hk = read_double(c, H + (size_t)(k - 1) * ld + k);
    bool breakdown = !(hk > 1e-14 * beta);
    // Gram entries of the new basis vector (used by the next iteration's
    // Gram-Schmidt); on the solution lane when there is one
    const bool grow = !breakdown && k < maxit;
    auto new_basis_dots = [&](Ctx& cc) {
      for (int i = 0; i <= k; ++i) {
        for (int q = 0; q < nc; ++q)
          tt_dot(cc, V[i].c[q], V[k].c[q], GV + (size_t)i * ld + k, q > 0, KV.at(q, i, k));
        if (i < k)
          SGTT_HIP(hipMemcpyAsync(GV + (size_t)k * ld + i, GV + (size_t)i * ld + k, sizeof(double),
                                  hipMemcpyDeviceToDevice, cc.s));
      }
    };
    if (grow) {
      V.push_back(vec_scale3(c, std::move(vn), H + (size_t)(k - 1) * ld + k, 1));
      for (int i = 0; i <= k; ++i)
        for (int q = 0; q < nc; ++q) {
          double*& slot = KV.at(q, i, k);
          if (!slot) slot = c.pool.get((size_t)V[i].c[q].r2 * V[k].c[q].r2);
        }
      if (!lane) new_basis_dots(c);
    }
    // lines 12-13: least squares, z_k = T(V^ y)
    prof_region(rg_sol);
    hessenberg_lsq(c.s, H, ld, k, sc + 5, y, sc + 8);
    if (!explicit_res) {
      res = read_double(c, sc + 8);
      if (cnt && cnt->hist) {
        sgtt_iter_record h{};
        h.cycle = cnt->cycle;
        h.iter = k;
        h.rel = res / bnorm;
        hist_ranks(V.back(), h.rank_v_u, h.rank_v_p);
        h.seconds = now_s() - cnt->t_start;
        cnt->hist->push_back(h);
      }
      if (cnt && cnt->verbose > 1)
        fprintf(stderr, "[sgtt %s] it %d  est %.3e  ranks v=(%d,%d) x=(%d,%d) rhs=(%d,%d)\n", tag, k, res / bnorm,
                V.back().c[0].r1, V.back().c[0].r2, x.c[0].r1, x.c[0].r2, V[0].c[0].r1, V[0].c[0].r2);
      if (breakdown) break;
      continue;
    }
    // lines 13-14 on the context cc: z_k = T(V^ y), s_k = T(b - L z_k) and
    // its norm into sc[11]; returns z_k and ||s_k||
    auto solution_and_residual = [&](Ctx& cc, Vec& zz, Vec& Lzz) {
      zz = Vec();
      zz.nc = nc;
      auto zone = [&](Ctx& c2, int q) {
        std::vector<Term> terms;
        std::vector<const double*> cache((size_t)k * k, nullptr);
        for (int i = 0; i < k; ++i) {
          terms.push_back(Term{&Vh[i].c[q], y + i, 1.0});
          for (int j = i; j < k; ++j) cache[(size_t)i * k + j] = KVh.at(q, i, j);
        }
        return tt_round_sum(c2, terms, eps, nullptr, nullptr, &cache);
      };
      if (nc == 2)
        pair_run(cc, [&](Ctx& c2) { return zone(c2, 0); }, [&](Ctx& c2) { return zone(c2, 1); }, zz.c[0], zz.c[1]);
      else
        zz.c[0] = zone(cc, 0);
      if (&cc == &c) {
        Lzz = sp.apply(zz);
      } else {
        sp.apply_on(zz, cc, Lzz);
      }
      auto one = [&](Ctx& c2, int q) {
        std::vector<Term> terms{Term{&b.c[q], nullptr, 1.0}, Term{&Lzz.c[q], nullptr, -1.0}};
        return tt_round_sum(c2, terms, eps, nullptr, sc + 9 + q, nullptr);
      };
      TT sk0, sk1;
      if (nc == 2)
        pair_run(cc, [&](Ctx& c2) { return one(c2, 0); }, [&](Ctx& c2) { return one(c2, 1); }, sk0, sk1);
      else
        sk0 = one(cc, 0);
      scalar_op(cc.s, 0, sc + 9, nc > 1 ? sc + 10 : nullptr, sc + 11);
      return read_double(cc, sc + 11);
    };
    Vec Lz;
    if (lane) {
      // fork: the lane's stream starts after the least-squares solve
      SGTT_HIP(hipEventRecord(lane->fork_ev, c.s));
      double res_lane = 0.0;
      const int prec = gemm_precision(GP_F64);
      gemm_precision(prec);
      lane->post([&, prec]() {
        SGTT_HIP(hipStreamWaitEvent(lane->c.s, lane->fork_ev, 0));
        lane->keep.clear();   // the previous z_k, copied out before this fork
        const int p0 = gemm_precision(prec);
        const int r0 = prof_region(rg_sol);
        try {
          {
            GemmPrecisionScope f64(GP_F64);   // Gram entries stay FP64
            vh_grams(lane->c);
            if (grow) new_basis_dots(lane->c);
          }
          Vec zl, Lzl;
          res_lane = solution_and_residual(lane->c, zl, Lzl);
          for (int q = 0; q < nc; ++q) lane->keep.push_back(std::move(zl.c[q]));
        } catch (...) {
          gemm_precision(p0);
          prof_region(r0);
          throw;
        }
        gemm_precision(p0);
        prof_region(r0);
        SGTT_HIP(hipEventRecord(lane->join_ev, lane->c.s));
      });
      // the next iteration's preconditioner meanwhile, unless the estimate
      // says this may be the last iteration of the cycle
      try {
        const double est = read_double(c, sc + 8);
        if (!breakdown && k < maxit && est > 2.0 * tol * bnorm) {
          RegionScope rg(inner ? RG_IN_MINV : RG_LSC);
          sp.note_residual(est / bnorm);
          vh_pre = sp.precond(V[k]);
          have_pre = true;
        }
      } catch (...) {
        (void)lane->wait();
        throw;
      }
      if (std::exception_ptr e = lane->wait()) std::rethrow_exception(e);
      SGTT_HIP(hipStreamWaitEvent(c.s, lane->join_ev, 0));
      // z_k into this context's pool (the lane's copy is released by its next job)
      z = Vec();
      z.nc = nc;
      for (int q = 0; q < nc; ++q) z.c[q] = tt_copy(c, lane->keep[q]);
      res = res_lane;
    } else {
      double t2 = now_s();
      res = solution_and_residual(c, z, Lz);
      if (cnt) cnt->t_apply += now_s() - t2;
    }
    if (cnt) {
      for (int i = 0; i < nc; ++i) {
        int r2 = V.back().c[i].r2;
        if (i == 0) cnt->maxr_u = std::max(cnt->maxr_u, r2);
        else cnt->maxr_p = std::max(cnt->maxr_p, r2);
      }
    }
    if (cnt && cnt->hist) {
      sgtt_iter_record h{};
      h.cycle = cnt->cycle;
      h.iter = k;
      h.rel = res / bnorm;
      hist_ranks(V.back(), h.rank_v_u, h.rank_v_p);
      hist_ranks(z, h.rank_z_u, h.rank_z_p);
      h.seconds = now_s() - cnt->t_start;
      cnt->hist->push_back(h);
    }
    if (cnt && cnt->verbose)
      fprintf(stderr, "[sgtt %s] it %d  rel %.3e  ranks v=(%d,%d) z=(%d,%d)\n", tag, k, res / bnorm,
              V.back().c[0].r1, V.back().c[0].r2, z.c[0].r1, z.c[0].r2);
    if (breakdown) break;
  }
  iters = k;
  relres = res / bnorm;
  prof_region(rg_sol);
  if (!explicit_res && k > 0) {
    z = Vec();
    z.nc = nc;
    solution_round(z);
  }
  if (k == 0) z = vec_copy(c, V[0]);
  return z;
}

// ---------------------------------------------------------------- preconditioner
struct InnerSpace : Space {
  sgtt_system& S;
  explicit InnerSpace(sgtt_system& s) : S(s) {}
  Vec apply(const Vec& x) override {
    Vec y;
    y.nc = 1;
    y.c[0] = apply_mean_sum(S, x.c[0], S.Kmean, 2, S.ns);
    return y;
  }
  Vec precond(const Vec& x) override {
    Vec y;
    y.nc = 1;
    y.c[0] = apply_Minv(S, x.c[0]);
    return y;
  }
};

// precision option 3: the velocity block in FP32 only where the outer
// iteration's residual allows it (OuterSpace::note_residual)
constexpr int PREC_RELAXED = 3;
// relative error of the FP32 time-stepped mean solve against the FP64 one,
// bounded from above (the GPU tests measure it against the oracle)
constexpr double kF32MeanSolveError = 1e-5;

struct PrecOpts {
  double eps = 1e-6, inner_tol = 1e-1, inner_eps = 1e-3, inner_rhs_eps = 0.0;
  int inner_mode = 0;       // 0: inner GMRES with M (eq. 5.22-5.23); 1: exact mean solve; 2: M alone
  int schur = 0;            // 0: mean-based LSC (eq. 5.19); 1: mean-based PCD (eq. 5.17)
  int inner_maxit = 20;
  bool inner_explicit = false;
  int precision = GP_F64;   // dense products of the inner solve, or PREC_RELAXED
  bool relaxed_f32 = false;  // PREC_RELAXED: this application may run in FP32
  bool graph = false;       // the mean solve's time loop as a captured graph
};

// The time loop of the mean solve below on the time-major full tensors W
// (right-hand side, consumed) and V (solution): v_t = F_avg^-1 (w_t +
// tau^-1 M v_{t-1}), one mass product and one block cyclic reduction solve
// per step; f32 selects the FP32 kernels on the first halves of the buffers.
void mean_time_loop(sgtt_system& S, hipStream_t s, bool f32, double* Wd, double* Vd) {
  const int nt = S.nt, nxi = S.nxi;
  const long blk = (long)S.nu * nxi;
  if (f32) {
    float* W = reinterpret_cast<float*>(Wd);
    float* V = reinterpret_cast<float*>(Vd);
    for (int t = 0; t < nt; ++t) {
      float* Wt = W + (long)t * blk;
      if (t > 0)
        ell_spmm32(s, S.ns, 2, S.ns, S.ns, S.Me_groups, S.Me_val32, S.Me_nnz, V + (long)(t - 1) * blk, nxi, 0, nxi,
                   Wt, nxi, 0, (float)(1.0 / S.tau), 1.0f);
      bcr_solve32(s, S.Fbt, 2, Wt, nxi, V + (long)t * blk, nxi, nxi);
    }
    return;
  }
  for (int t = 0; t < nt; ++t) {
    double* Wt = Wd + (long)t * blk;
    if (t > 0)
      ell_spmm(s, S.ns, 2, S.ns, S.ns, S.Me_groups, S.Me_val, S.Me_nnz, Vd + (long)(t - 1) * blk, nxi, 0, nxi, Wt,
               nxi, 0, 1.0 / S.tau, 1.0);
    bcr_solve(s, S.Fbt, 2, Wt, nxi, Vd + (long)t * blk, nxi, nxi);
  }
}

// The system's own full-tensor buffers of the graph form (allocated on first
// use, kept until the system is destroyed): a captured graph holds their
// addresses in its kernel arguments.
bool mean_graph_buffers(sgtt_system& S) {
  if (S.mg_W && S.mg_V) return true;
  const size_t n = (size_t)S.nt * S.nu * S.nxi;
  for (double** p : {&S.mg_W, &S.mg_V}) {
    if (*p) continue;
    ++S.mg_allocs;
    if (hipMalloc(p, n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      throw SgttError(-3, "graph form of the mean solve: device allocation failed");
    }
  }
  return true;
}

// The time loop as one graph launch on the context stream: captured (on the
// system's buffers) the first time it is asked for once the spatial solve's
// pass variants are tuned for these columns (tuning times kernels on the
// GPU, which a capture cannot contain), then replayed.  Returns false when
// the caller has to run the loop itself this time.
bool mean_loop_graph(sgtt_system& S, bool f32) {
  Ctx& c = S.ctx->c;
  hipGraphExec_t& ex = S.mg_exec[f32 ? 1 : 0];
  if (!ex) {
    if (!bcr_is_tuned(S.Fbt, 2, S.nxi, f32)) return false;
    hipGraph_t gr = nullptr;
    SGTT_HIP(hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal));
    prof_hold_thread(true);
    try {
      mean_time_loop(S, c.s, f32, S.mg_W, S.mg_V);
    } catch (...) {
      (void)hipStreamEndCapture(c.s, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      (void)hipGetLastError();
      prof_hold_thread(false);
      throw;
    }
    const hipError_t e = hipStreamEndCapture(c.s, &gr);
    prof_hold_thread(false);
    SGTT_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ei != hipSuccess) {
      ex = nullptr;
      SGTT_HIP(ei);
    }
  }
  SGTT_HIP(hipGraphLaunch(ex, c.s));
  ++S.mg_launches;
  return true;
}

// (tau^-1 (I - C) (x) I (x) M + I (x) I (x) (F_avg - tau^-1 M))^-1 y: the mean
// matrix F_0 + C of eq. 5.21 with its convection N_0 replaced by the
// time-averaged one inside F_avg (eq. 5.23).  Without convection this is
// (F_0 + C)^-1 exactly.  The matrix is lower block-bidiagonal in time with
// F_avg on the diagonal and -tau^-1 M below, identity in the chaos mode:
// block forward substitution in time on the full-format velocity, then
// TT-SVD (Alg. 4.1) at eps.  The full tensor is kept time-major, W[t][x][xi]:
// each time step's right-hand side and solution are one contiguous node-major
// block (n_u x n_xi), so the mass products and the block cyclic reduction
// passes of a step stream whole cache lines and DRAM pages instead of short
// pieces of rows n_t n_xi values apart.
// The same solve in FP32 (precision option 1): the expansion writes the full
// velocity tensor in FP32 (computed in FP64, rounded on the store), the time steps
// run the FP32 ELL mass product and FP32 block cyclic reduction passes, and
// the transpose widens the result to FP64 for the TT-SVD, whose Grams, rank
// decisions and projections stay FP64.  The result is accurate to FP32
// rounding relative to the exact one, far below the inner truncation eps.
TT exact_mean_solve32(sgtt_system& S, const TT& y, double eps, bool graph) {
  Ctx& c = S.ctx->c;
  const int nt = S.nt, nxi = S.nxi, nu = S.nu;
  const long ldw = (long)nt * nxi;
  const long blk = (long)nu * nxi;               // one time step
  double* Z = c.pool.get((size_t)ldw * y.r2);   // G1 x_1 G2: (nt nxi) x r2
  gemm(c.s, 1, nt, nxi * y.r2, y.r1, 1.0, y.c1, 0, y.r1, 1, y.c2, 0, (long)nxi * y.r2, 1, 0.0, Z, 0,
       (long)nxi * y.r2, 1);
  const size_t nfull = (size_t)nt * blk;
  const bool g = graph && mean_graph_buffers(S);
  double* Wd = g ? S.mg_W : c.pool.get((nfull + 1) / 2);   // time-major FP32 tensor W[t][x][xi]
  float* W = reinterpret_cast<float*>(Wd);
  gemm_csplit_f32out(c.s, nu, (int)ldw, y.r2, y.c3, y.r2, 1, Z, 1, y.r2, W, nxi, nxi, blk);
  c.pool.put(Z);
  double* Vd = g ? S.mg_V : c.pool.get((nfull + 1) / 2);   // FP32 solution, same layout
  float* Vn = reinterpret_cast<float*>(Vd);
  if (!(g && mean_loop_graph(S, true))) mean_time_loop(S, c.s, true, Wd, Vd);
  if (!g) c.pool.put(Wd);
  double* V = c.pool.get(nfull);                 // C order (t, xi, x), FP64
  transpose_widen_batched(c.s, nt, nu, nxi, Vn, blk, nxi, V, blk, nu);
  if (!g) c.pool.put(Vd);
  TT out = tt_from_full(c, V, nt, nxi, nu, eps, nullptr);
  c.pool.put(V);
  return out;
}

TT exact_mean_solve(sgtt_system& S, const TT& y, double eps, bool graph) {
  Ctx& c = S.ctx->c;
  const int nt = S.nt, nxi = S.nxi, nu = S.nu;
  const long ldw = (long)nt * nxi;
  const long blk = (long)nu * nxi;               // one time step
  double* Z = c.pool.get((size_t)ldw * y.r2);   // G1 x_1 G2: (nt nxi) x r2
  gemm(c.s, 1, nt, nxi * y.r2, y.r1, 1.0, y.c1, 0, y.r1, 1, y.c2, 0, (long)nxi * y.r2, 1, 0.0, Z, 0,
       (long)nxi * y.r2, 1);
  const bool g = graph && mean_graph_buffers(S);
  double* W = g ? S.mg_W : c.pool.get((size_t)nt * blk);   // time-major full tensor: W[t][x][xi]
  gemm_csplit(c.s, nu, (int)ldw, y.r2, y.c3, y.r2, 1, Z, 1, y.r2, W, nxi, nxi, blk);
  c.pool.put(Z);
  double* Vn = g ? S.mg_V : c.pool.get((size_t)nt * blk);  // solution, same layout
  if (!(g && mean_loop_graph(S, false))) mean_time_loop(S, c.s, false, W, Vn);
  double* V = W;                                 // C order (t, xi, x), reusing the consumed right-hand side
  transpose_copy_batched(c.s, nt, nu, nxi, Vn, blk, nxi, V, blk, nu);
  if (!g) c.pool.put(Vn);
  TT out = tt_from_full(c, V, nt, nxi, nu, eps, nullptr);
  if (!g) c.pool.put(W);
  return out;
}

Vec lsc_precondition(sgtt_system& S, const Vec& y, const PrecOpts& po, SolveCounters* cnt) {
  Ctx& c = S.ctx->c;
  const TT& yu = y.c[0];
  const TT& yp = y.c[1];
  TT t3;
  if (po.schur == 1) {
    // p^ = -X^-1 (F_p,0 + C_p) M_p*^-1 y_p   (eq. 5.17)
    TT t1 = tt_new(c, S.nt, S.nxi, S.np, yp.r1, yp.r2);
    SGTT_HIP(hipMemcpyAsync(t1.c1, yp.c1, sizeof(double) * yp.n_c1(), hipMemcpyDeviceToDevice, c.s));
    SGTT_HIP(hipMemcpyAsync(t1.c2, yp.c2, sizeof(double) * yp.n_c2(), hipMemcpyDeviceToDevice, c.s));
    spmm(c.s, S.np, 1, 0, 0, S.Mpinv.rowptr, S.Mpinv.col, S.Mpinv.vals, 1, S.Mpinv.nnz, yp.c3, yp.r2, 0, yp.r2, t1.c3,
         yp.r2, 0, 0, 1.0, 0.0, S.Mpinv.max_row);
    TT t2 = apply_mean_sum(S, t1, S.Fp, 1, S.np);
    t3 = tt_round(c, t2, po.eps, nullptr, nullptr);
  } else {
    // p^ = -X^-1 [B M*^-1 (F_0 + C) M*^-1 B^T] X^-1 y_p   (eq. 5.19)
    TT t1 = space_solve(S, yp, S.Xbt, 1, 1.0);
    TT t2 = apply_mean_sum(S, t1, S.Xmid, 1, S.np);
    t3 = tt_round(c, t2, po.eps, nullptr, nullptr);
  }
  TT ph = space_solve(S, t3, S.Xbt, 1, -1.0);
  // right-hand side of the (1,1) solve: y_u - B^T p^
  TT bph = tt_new(c, S.nt, S.nxi, S.nu, ph.r1, ph.r2);
  copy2d(c.s, S.nt, ph.r1, ph.c1, ph.r1, bph.c1, ph.r1, -1.0, nullptr, 0);
  SGTT_HIP(hipMemcpyAsync(bph.c2, ph.c2, sizeof(double) * ph.n_c2(), hipMemcpyDeviceToDevice, c.s));
  spmm(c.s, S.nu, 1, 0, 0, S.Btd.rowptr, S.Btd.col, S.Btd.vals, 1, 0, ph.c3, ph.r2, 0, ph.r2, bph.c3, ph.r2, 0, 0,
       1.0, 0.0, S.Btd.max_row);
  Vec rhs;
  rhs.nc = 1;
  rhs.c[0] = tt_concat(c, {&yu, &bph}, nullptr, {});
  if (po.inner_mode == 2) {
    // M^-1 itself (eq. 5.23) as the velocity block: the approximation of
    // (F_0 + C)^-1 that the inner solve of eq. 5.22 is preconditioned with,
    // applied once (prefix sum in time, one F_avg solve on core 3)
    RegionScope rg(RG_IN_MINV);
    Vec out;
    out.nc = 2;
    TT m = apply_Minv(S, rhs.c[0]);
    out.c[0] = tt_round(c, m, po.inner_eps, nullptr, nullptr);
    out.c[1] = std::move(ph);
    return out;
  }
  // inner low-rank GMRES on (F_0 + C) v = rhs, preconditioned by M (eq. 5.22-5.23)
  if (po.inner_mode == 1) {
    RegionScope rg(RG_IN_MINV);
    Vec out;
    out.nc = 2;
    const bool f32 = po.precision == PREC_RELAXED ? po.relaxed_f32 : po.precision != GP_F64;
    out.c[0] = f32 ? exact_mean_solve32(S, rhs.c[0], po.inner_eps, po.graph)
                   : exact_mean_solve(S, rhs.c[0], po.inner_eps, po.graph);
    out.c[1] = std::move(ph);
    return out;
  }
  InnerSpace isp(S);
  int its = 0;
  double rr = 0;
  SolveCounters icnt;
  icnt.verbose = cnt ? cnt->verbose : 0;
  GemmPrecisionScope gp(po.precision == PREC_RELAXED ? (po.relaxed_f32 ? GP_F32 : GP_F64) : po.precision);
  Vec v = lowrank_fgmres(c, isp, rhs, po.inner_tol, po.inner_eps, po.inner_maxit, S.dsc + 16384, its, rr, &icnt,
                         "inner", po.inner_explicit, false, 1e-2, po.inner_rhs_eps);
  if (cnt) cnt->inner += its;
  // fallback: two inner solves that miss their tolerance with the learned
  // mean solve switch the rest of this solve back to the exact one
  if (S.mlp_apply && !S.mlp_off && rr > po.inner_tol && ++S.mlp_fails >= 2) S.mlp_off = true;
  Vec out;
  out.nc = 2;
  out.c[0] = std::move(v.c[0]);
  out.c[1] = std::move(ph);
  return out;
}

struct OuterSpace : Space {
  sgtt_system& S;
  PrecOpts po;
  SolveCounters* cnt;
  // PREC_RELAXED: the relative residual of the whole solve at the start of
  // the current refinement cycle, and the level below which an application
  // of the preconditioner may run its velocity block in FP32
  double cycle_rel = 1.0, f32_below = 0.0;
  OuterSpace(sgtt_system& s, const PrecOpts& p, SolveCounters* c) : S(s), po(p), cnt(c) {}
  Vec apply(const Vec& x) override { return apply_L(S, x); }
  Vec precond(const Vec& x) override { return lsc_precondition(S, x, po, cnt); }
  void note_residual(double rel) override {
    po.relaxed_f32 = po.precision == PREC_RELAXED && cycle_rel * rel <= f32_below;
    if (po.relaxed_f32 && cnt) ++cnt->f32_applications;
  }
  bool can_apply_on() const override { return true; }
  bool apply_on(const Vec& x, Ctx& cc, Vec& y) override {
    y = apply_L(S, x, &cc);
    return true;
  }
};

// exact ||b - L z|| / ||b|| in full format
double full_residual(sgtt_system& S, const Vec& b, const Vec& z, double* d_out_sq, Vec* r_tt, double eps_tt,
                     double* bnorm_cache, double* const* full_out = nullptr) {
  Ctx& c = S.ctx->c;
  RegionScope rg(RG_RESIDUAL);
  Vec Lz = apply_L(S, z);
  Vec r = vec_concat(c, {&b, &Lz}, nullptr, {1.0, -1.0});
  double tot = 0.0, bn2 = bnorm_cache ? *bnorm_cache : -1.0;
  double* ws = c.scratch(1 << 16);
  double* sq = S.dsc + 30000;
  double res_sq[2] = {0, 0};
  std::vector<TT> rt(2);
  for (int i = 0; i < 2; ++i) {
    const TT& ri = r.c[i];
    long n = (long)ri.n1 * ri.n2 * ri.n3;
    double* full = full_out ? full_out[i] : c.pool.get(n);
    tt_expand(c, ri, full);
    sumsq(c.s, full, n, sq + i, ws, 1 << 16);
    if (r_tt) rt[i] = tt_from_full(c, full, ri.n1, ri.n2, ri.n3, eps_tt, nullptr);
    if (bn2 < 0) {
      double* fb = full_out ? c.pool.get(n) : full;
      tt_expand(c, b.c[i], fb);
      sumsq(c.s, fb, n, sq + 2 + i, ws, 1 << 16);
      if (full_out) c.pool.put(fb);
    }
    if (!full_out) c.pool.put(full);
  }
  SGTT_HIP(hipMemcpyAsync(c.hdbl, sq, 4 * sizeof(double), hipMemcpyDeviceToHost, c.s));
  c.sync();
  res_sq[0] = c.hdbl[0];
  res_sq[1] = c.hdbl[1];
  if (bn2 < 0) {
    bn2 = c.hdbl[2] + c.hdbl[3];
    if (bnorm_cache) *bnorm_cache = bn2;
  }
  tot = res_sq[0] + res_sq[1];
  if (d_out_sq) *d_out_sq = tot;
  if (r_tt) {
    r_tt->nc = 2;
    r_tt->c[0] = std::move(rt[0]);
    r_tt->c[1] = std::move(rt[1]);
  }
  return bn2 > 0 ? std::sqrt(tot / bn2) : 0.0;
}

// ---------------------------------------------------------------- helpers for the ABI
// a caller's buffer that kernels will read or write: device, managed or
// pinned host memory (a kernel access to memory HIP does not know faults the
// GPU, so such a buffer is refused before anything runs)
void check_device_ptr(const void* p, const char* what) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    throw SgttError(-1, std::string(what) + " is not memory allocated through HIP");
  }
  const bool dev = a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
  const bool pinned = a.type == hipMemoryTypeHost && a.devicePointer;
  if (!dev && !pinned) throw SgttError(-1, std::string(what) + " is not accessible from the device");
}

// element type, cores and the device copy of the ranks (NULL or memory the
// device can reach) of a caller's TT
void check_dtype(const sgtt_tt& t) {
  if (t.dtype != SGTT_DTYPE_F64) throw SgttError(-1, "TT element type other than FP64");
  if (t.core1) check_device_ptr(t.core1, "core 1");
  if (t.core2) check_device_ptr(t.core2, "core 2");
  if (t.core3) check_device_ptr(t.core3, "core 3");
  if (t.d_ranks) check_device_ptr(t.d_ranks, "d_ranks");
}

// live ranks of an output TT: host fields, and the caller's device copy
void set_ranks(Ctx& c, sgtt_tt* out, int r1, int r2) {
  out->r1 = r1;
  out->r2 = r2;
  if (out->d_ranks) store_ranks(c.s, out->d_ranks, r1, r2);
}

Vec vec_from_pair(const sgtt_tt_pair* p) {
  check_dtype(p->u);
  check_dtype(p->p);
  Vec v;
  v.nc = 2;
  v.c[0] = tt_view(p->u.n1, p->u.n2, p->u.n3, p->u.r1, p->u.r2, p->u.core1, p->u.core2, p->u.core3);
  v.c[1] = tt_view(p->p.n1, p->p.n2, p->p.n3, p->p.r1, p->p.r2, p->p.core1, p->p.core2, p->p.core3);
  return v;
}

void check_tt(const sgtt_tt& t, int n1, int n2, int n3) {
  check_dtype(t);
  if (t.n1 != n1 || t.n2 != n2 || t.n3 != n3) throw SgttError(-1, "TT dimensions do not match the system");
  if (t.r1 < 1 || t.r2 < 1 || t.r1 > t.cap1 || t.r2 > t.cap2 || !t.core1 || !t.core2 || !t.core3)
    throw SgttError(-1, "invalid TT ranks or buffers");
}

void write_tt(Ctx& c, const TT& x, sgtt_tt* out) {
  check_dtype(*out);
  if (x.r1 > out->cap1 || x.r2 > out->cap2)
    throw SgttError(-4, "result rank (" + std::to_string(x.r1) + "," + std::to_string(x.r2) +
                            ") exceeds output capacity (" + std::to_string(out->cap1) + "," +
                            std::to_string(out->cap2) + ")");
  SGTT_HIP(hipMemcpyAsync(out->core1, x.c1, sizeof(double) * x.n_c1(), hipMemcpyDeviceToDevice, c.s));
  SGTT_HIP(hipMemcpyAsync(out->core2, x.c2, sizeof(double) * x.n_c2(), hipMemcpyDeviceToDevice, c.s));
  SGTT_HIP(hipMemcpyAsync(out->core3, x.c3, sizeof(double) * x.n_c3(), hipMemcpyDeviceToDevice, c.s));
  set_ranks(c, out, x.r1, x.r2);
}

void write_pair(Ctx& c, const Vec& v, sgtt_tt_pair* out) {
  check_dtype(out->u);
  check_dtype(out->p);
  if (v.c[0].r1 > out->u.cap1 || v.c[0].r2 > out->u.cap2 || v.c[1].r1 > out->p.cap1 || v.c[1].r2 > out->p.cap2)
    throw SgttError(-4, "result rank exceeds output capacity");
  write_tt(c, v.c[0], &out->u);
  write_tt(c, v.c[1], &out->p);
}

PrecOpts prec_opts(const sgtt_solve_opts* o) {
  PrecOpts p;
  if (o) {
    p.eps = o->eps_krylov;
    p.inner_tol = o->inner_tol;
    p.inner_eps = o->inner_eps;
    p.inner_maxit = o->inner_maxit;
    p.inner_explicit = o->inner_explicit != 0;
    if (o->precision < 0 || o->precision > PREC_RELAXED) throw SgttError(-1, "invalid precision option");
    if (o->inner_rhs_eps < 0.0 || o->cycle_rhs_factor < 0.0) throw SgttError(-1, "invalid truncation option");
    p.inner_rhs_eps = o->inner_rhs_eps;
    if (o->inner_mode < 0 || o->inner_mode > 2) throw SgttError(-1, "invalid inner_mode option");
    p.inner_mode = o->inner_mode;
    p.precision = o->precision;
    if (o->schur < 0 || o->schur > 1) throw SgttError(-1, "invalid schur option");
    p.schur = o->schur;
    if (o->graph < 0 || o->graph > 1) throw SgttError(-1, "invalid graph option");
    p.graph = o->graph == 1;
  }
  return p;
}

sgtt_solve_opts default_opts() {
  sgtt_solve_opts o;
  o.tol = 1e-8;
  o.eps_krylov = 1e-6;
  o.tol_cycle = 1e-4;
  o.restart = 30;
  o.max_cycles = 8;
  o.inner_tol = 1e-1;
  o.inner_eps = 1e-3;
  o.inner_maxit = 20;
  o.verbose = 0;
  o.outer_explicit = 1;
  o.inner_explicit = 0;
  o.relax = 0;
  o.precision = 0;
  o.inner_rhs_eps = 0.0;
  o.cycle_rhs_factor = 0.0;
  o.inner_mode = 0;
  o.schur = 0;
  o.graph = 0;
  return o;
}

// ---------------------------------------------------------------- assembly
void build_convection(sgtt_system& S, Ctx& c, const TT& wtil) {
  // w~ (all-node velocity TT) -> host: N(w3_b) values, Hw, omega, avg coefficients
  HostProblem& hp = S.hp;
  const int nall = S.nall, nxi = S.nxi, nt = S.nt;
  const int k1 = wtil.r1, k2 = wtil.r2;
  std::vector<double> h1((size_t)nt * k1), h2((size_t)k1 * nxi * k2), h3((size_t)2 * nall * k2);
  SGTT_HIP(hipMemcpyAsync(h1.data(), wtil.c1, h1.size() * 8, hipMemcpyDeviceToHost, c.s));
  SGTT_HIP(hipMemcpyAsync(h2.data(), wtil.c2, h2.size() * 8, hipMemcpyDeviceToHost, c.s));
  SGTT_HIP(hipMemcpyAsync(h3.data(), wtil.c3, h3.size() * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  S.k1 = k1;
  S.k2 = k2;
  const int nnz = hp.Kff.nnz(), nnzx = hp.Xmid.nnz(), nnzq = hp.Qp.nnz();
  std::vector<std::vector<double>> Nv(k2, std::vector<double>(nnz)), XNv(k2, std::vector<double>(nnzx));
  std::vector<std::vector<double>> NPv(k2, std::vector<double>(nnzq));
  std::vector<double> w1(nall), w2(nall);
  for (int b = 0; b < k2; ++b) {
    for (int i = 0; i < nall; ++i) {
      w1[i] = h3[(size_t)i * k2 + b];
      w2[i] = h3[(size_t)(nall + i) * k2 + b];
    }
    convection_values(hp, w1.data(), w2.data(), Nv[b].data(), nullptr);
    lsc_middle_values(hp, Nv[b].data(), XNv[b].data());
    pressure_convection_values(hp, w1.data(), w2.data(), NPv[b].data());
  }
  // Hw[a,b] = sum_l w2(a,l,b) H_l ; omega[t,b] = sum_a w1[t,a] w2(a,0,b)
  std::vector<double> Hw((size_t)k1 * k2 * nxi * nxi, 0.0), om((size_t)nt * k2, 0.0), avg(k2, 0.0);
  for (int a = 0; a < k1; ++a)
    for (int b = 0; b < k2; ++b)
      for (int l = 0; l < nxi; ++l) {
        double wv = h2[((size_t)a * nxi + l) * k2 + b];
        if (wv == 0.0) continue;
        const double* Hl = hp.H.data() + (size_t)l * nxi * nxi;
        double* dst = Hw.data() + ((size_t)a * k2 + b) * nxi * nxi;
        for (int q = 0; q < nxi * nxi; ++q) dst[q] += wv * Hl[q];
      }
  for (int t = 0; t < nt; ++t)
    for (int b = 0; b < k2; ++b) {
      double s = 0;
      for (int a = 0; a < k1; ++a) s += h1[(size_t)t * k1 + a] * h2[((size_t)a * nxi + 0) * k2 + b];
      om[(size_t)t * k2 + b] = s;
      avg[b] += s / nt;
    }
  S.w1 = dev_upload(c, h1);
  S.Hw = dev_upload(c, Hw);
  S.omega = dev_upload(c, om);
  // operator value sets
  std::vector<const double*> vs{hp.Mff.data()}, vm{hp.Mff.data(), hp.Aff.data()};
  for (const auto& a : hp.Aff_visc) vs.push_back(a.data());
  for (int b = 0; b < k2; ++b) {
    vs.push_back(Nv[b].data());
    vm.push_back(Nv[b].data());
  }
  S.Kop.free_all();
  S.Kmean.free_all();
  S.Kop = upload_csr(c, hp.Kff, vs);
  S.Kmean = upload_csr(c, hp.Kff, vm);
  std::vector<const double*> xs{hp.XM.data(), hp.XA.data()};
  for (int b = 0; b < k2; ++b) xs.push_back(XNv[b].data());
  S.Xmid = upload_csr(c, hp.Xmid, xs);
  std::vector<const double*> ps{hp.Mp.data(), hp.Ap.data()};
  for (int b = 0; b < k2; ++b) ps.push_back(NPv[b].data());
  S.Fp.free_all();
  S.Fp = upload_csr(c, hp.Qp, ps);
  // F_avg = tau^-1 M + nu0 A + N(w_avg), N linear in the wind
  std::vector<double> F(nnz);
  for (int t = 0; t < nnz; ++t) {
    double v = hp.Mff[t] / S.tau + S.nu0 * hp.Aff[t];
    for (int b = 0; b < k2; ++b) v += avg[b] * Nv[b][t];
    F[t] = v;
  }
  if (S.Dinv) (void)hipFree(S.Dinv);
  S.Dinv = dev_upload(c, inverse_diagonal(hp.Kff, F.data()));
  free_bcr(S.Fbt);
  S.Fbt = factor_bcr(c, hp.Kff, F.data(), hp.vel_blocks);
}

}  // namespace

// ====================================================================== C ABI
namespace {
template <class F>
int guarded(sgtt_context* ctx, F&& f) {
  try {
    f();
    return SGTT_OK;
  } catch (const SgttError& e) {
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return SGTT_E_INVALID;
  }
}
}  // namespace

// Device scratch of the allocation-free spatial solve (sgtt_bcr_apply_noalloc):
// the working copy of the right-hand side that the reduction overwrites.
// Every GPU the library runs on holds its own copy until the process ends.
// Host code never uses the array's name as an address: it takes the
// per-device address that hipGetSymbolAddress returns (noalloc_scratch).
static __device__ __align__(256) double scratch[SGTT_NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch; resolved once per device, with that
// device current (the caller has made it current).
double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) throw SgttError(SGTT_E_INVALID, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    SGTT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw SgttError(SGTT_E_HIP, "scratch symbol has no device address");
    g_scratch_ptr[device] = (double*)p;
  }
  return g_scratch_ptr[device];
}
}  // namespace

extern "C" {

const char* sgtt_version(void) { return "sgtt 0.1 gfx950 fp64"; }

int sgtt_abi_sizes(long* sizes, int n) {
  const long all[] = {(long)sizeof(sgtt_tt),          (long)sizeof(sgtt_tt_pair),     (long)sizeof(sgtt_problem_desc),
                      (long)sizeof(sgtt_system_info), (long)sizeof(sgtt_solve_opts),  (long)sizeof(sgtt_solve_stats),
                      (long)sizeof(sgtt_memory_info), (long)sizeof(sgtt_picard_opts), (long)sizeof(sgtt_picard_stats),
                      (long)sizeof(sgtt_iter_record)};
  const int total = (int)(sizeof(all) / sizeof(all[0]));
  for (int i = 0; sizes && i < n && i < total; ++i) sizes[i] = all[i];
  return total;
}

static thread_local std::string g_create_err;

int sgtt_context_create(int device, void* stream, sgtt_context** out) {
  if (!out) return SGTT_E_INVALID;
  sgtt_context* ctx = new sgtt_context();
  try {
    ctx->device = device;
    ctx->c.device = device;
    {
      // the pressure TT of a pair is rounded on a second stream beside the
      // velocity TT (SGTT_SIDE_LANE=0 rounds them one after the other)
      const char* e = std::getenv("SGTT_SIDE_LANE");
      ctx->c.side_enabled = !(e && e[0] == '0');
    }
    SGTT_HIP(hipSetDevice(device));
    if (stream) {
      ctx->c.s = (hipStream_t)stream;
    } else {
      SGTT_HIP(hipStreamCreate(&ctx->c.s));   // blocking: ordered after the legacy default stream
      ctx->own_stream = true;
    }
    ctx->scratch = noalloc_scratch(device);
    SGTT_HIP(hipHostMalloc((void**)&ctx->c.hint, 64 * sizeof(int), hipHostMallocDefault));
    SGTT_HIP(hipHostMalloc((void**)&ctx->c.hdbl, 256 * sizeof(double), hipHostMallocDefault));
    ctx->c.dint = (int*)ctx->c.pool.get(64);
    ctx->c.dscal = ctx->c.pool.get(256);
  } catch (const SgttError& e) {
    g_create_err = e.what();
    delete ctx;
    return e.code;
  }
  *out = ctx;
  return SGTT_OK;
}

int sgtt_context_reserve(sgtt_context* ctx, size_t bytes) {
  if (!ctx) return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    ctx->c.sync();
    ctx->c.pool.reserve(bytes / sizeof(double));
    splitk_reserve(ctx->c.s);
  });
}

int sgtt_context_memory(const sgtt_context* ctx, sgtt_memory_info* out) {
  if (!ctx || !out) return SGTT_E_INVALID;
  const Pool& p = ctx->c.pool;
  out->arena_bytes = p.arena_bytes();
  out->arena_peak_bytes = p.arena_peak_bytes();
  out->cached_bytes = p.bytes_held();
  out->device_allocs = p.device_allocs();
  return SGTT_OK;
}

namespace {
void context_finalize(sgtt_context* ctx) {
  (void)hipStreamSynchronize(ctx->c.s);
  hipStream_t s = ctx->c.s;
  bool own = ctx->own_stream;
  delete ctx;
  if (own) {
    splitk_release(s);
    (void)hipStreamDestroy(s);
  }
}
void context_add_child(sgtt_context* ctx) {
  std::lock_guard<std::mutex> lk(ctx->life_mu);
  ++ctx->children;
}
// a system or network of ctx is gone; releases a closing context with it
void context_release_child(sgtt_context* ctx) {
  bool fin;
  {
    std::lock_guard<std::mutex> lk(ctx->life_mu);
    fin = --ctx->children == 0 && ctx->closing;
  }
  if (fin) context_finalize(ctx);
}
}  // namespace

int sgtt_context_destroy(sgtt_context* ctx) {
  if (!ctx) return SGTT_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(ctx->life_mu);
    if (ctx->children > 0) {
      // systems or networks still refer to it: release it with the last one
      ctx->closing = true;
      (void)hipStreamSynchronize(ctx->c.s);
      return SGTT_OK;
    }
  }
  context_finalize(ctx);
  return SGTT_OK;
}

const char* sgtt_last_error(const sgtt_context* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

// Builds a system (throws SgttError); see sgtt_assemble.
sgtt_system* assemble_internal(sgtt_context* ctx, const sgtt_problem_desc* desc, const sgtt_tt_pair* prior) {
  double t0 = now_s();
  auto S = std::make_unique<sgtt_system>();
  S->ctx = ctx;
  S->desc = *desc;
  Ctx& c = ctx->c;
  ProblemParams prm;
  prm.h = desc->h;
  prm.L = desc->L;
  prm.m = desc->m;
  prm.p = desc->p;
  prm.nt = desc->nt;
  prm.tau = desc->tau;
  prm.nu0 = desc->nu0;
  prm.nu_coef = desc->nu_coef;
  prm.ramp = desc->ramp;
  prm.visc_law = desc->viscosity_law;
  prm.corr_length = desc->corr_length;
  try {
    build_problem(prm, S->hp);
  } catch (const std::exception& e) {
    throw SgttError(-6, std::string("setup: ") + e.what());
  }
  HostProblem& hp = S->hp;
  S->nt = hp.nt;
  S->nxi = hp.n_xi;
  S->ns = hp.n_s;
  S->nu = hp.n_u;
  S->np = hp.n_p;
  S->nall = hp.n_all;
  S->tau = prm.tau;
  S->nu0 = prm.nu0;
  SGTT_HIP(hipMalloc(&S->dsc, 32768 * sizeof(double)));
  S->nvisc = hp.nvisc;
  S->Gvisc = dev_upload(c, hp.Gvisc);
  S->Bd = upload_csr(c, hp.B, {hp.B.val.data()});
  S->Btd = upload_csr(c, hp.Bt, {hp.Bt.val.data()});
  S->Xbt = factor_bcr(c, hp.Xp, hp.Xp.val.data(), hp.p_blocks);
  {
    const Csr& K = hp.Kff;
    std::vector<double> ev((size_t)K.nrows * ELL_WIDTH, 0.0);
    for (int r = 0; r < K.nrows; ++r) {
      const int n = K.rowptr[r + 1] - K.rowptr[r];
      if (n > ELL_WIDTH) throw SgttError(-6, "mass matrix row longer than the padded width");
      for (int q = 0; q < n; ++q) ev[(size_t)r * ELL_WIDTH + q] = hp.Mff[K.rowptr[r] + q];
    }
    std::vector<int> row0, uptr, ucols, lidx, rlen;
    ell_groups_build(K.nrows, K.rowptr.data(), K.col.data(), row0, uptr, ucols, lidx, rlen, S->Me_groups.umax);
    S->Me_groups.ngroups = (int)row0.size() - 1;
    S->Me_groups.row0 = dev_upload(c, row0);
    S->Me_groups.uptr = dev_upload(c, uptr);
    S->Me_groups.ucols = dev_upload(c, ucols);
    S->Me_groups.lidx = dev_upload(c, lidx);
    S->Me_groups.rlen = dev_upload(c, rlen);
    S->Me_nnz = K.rowptr[K.nrows];
    S->Me_val32 = dev_upload(c, std::vector<float>(ev.begin(), ev.end()));
    S->Me_val = dev_upload(c, ev);
  }
  const int nt = S->nt, nxi = S->nxi, nall = S->nall, ns = S->ns;
  // Dirichlet lift TT over all nodes: ramp (x) e_1 (x) g_all
  std::vector<double> e1(nxi, 0.0);
  e1[0] = 1.0;
  TT lift = tt_new(c, nt, nxi, 2 * nall, 1, 1);
  SGTT_HIP(hipMemcpyAsync(lift.c1, hp.ramp.data(), nt * 8, hipMemcpyHostToDevice, c.s));
  SGTT_HIP(hipMemcpyAsync(lift.c2, e1.data(), nxi * 8, hipMemcpyHostToDevice, c.s));
  SGTT_HIP(hipMemcpyAsync(lift.c3, hp.g_all.data(), 2 * nall * 8, hipMemcpyHostToDevice, c.s));
  c.sync();
  {
    // diag(M_p)^-1 of the PCD approximation (eq. 5.17) as a diagonal matrix
    Csr d;
    d.nrows = d.ncols = hp.n_p;
    d.rowptr.resize(hp.n_p + 1);
    d.col.resize(hp.n_p);
    d.val.resize(hp.n_p);
    for (int k = 0; k <= hp.n_p; ++k) d.rowptr[k] = k;
    for (int k = 0; k < hp.n_p; ++k) {
      d.col[k] = k;
      d.val[k] = 1.0 / hp.Mpstar[k];
    }
    S->Mpinv = upload_csr(c, d, {d.val.data()});
  }
  if (!prior) {
    // Stokes system: no convection; f = -L_{free,all}(0) lift (ranks 2 and 1)
    S->k1 = S->k2 = 0;
    {
      std::vector<const double*> vs{hp.Mff.data()};
      for (const auto& a : hp.Aff_visc) vs.push_back(a.data());
      S->Kop = upload_csr(c, hp.Kff, vs);
      S->Kmean = upload_csr(c, hp.Kff, {hp.Mff.data(), hp.Aff.data()});
    }
    S->Xmid = upload_csr(c, hp.Xmid, {hp.XM.data(), hp.XA.data()});
    S->Fp = upload_csr(c, hp.Qp, {hp.Mp.data(), hp.Ap.data()});
    std::vector<double> F(hp.Kff.nnz());
    for (int t = 0; t < hp.Kff.nnz(); ++t) F[t] = hp.Mff[t] / S->tau + S->nu0 * hp.Aff[t];
    S->Dinv = dev_upload(c, inverse_diagonal(hp.Kff, F.data()));
    S->Fbt = factor_bcr(c, hp.Kff, F.data(), hp.vel_blocks);
    // f^u: core1 [(I-C)a/tau | a], core2 [e1 ; (Gv_0 e1 | .. | Gv_{nv-1} e1)],
    // core3 -[M_fa g | A_0,fa g | .. | A_{nv-1},fa g]
    const int nv = hp.nvisc, rb = 1 + nv;
    std::vector<double> Ca(nt), c1((size_t)nt * 2), c2((size_t)2 * nxi * rb, 0.0);
    for (int k = 0; k < nt; ++k) {
      c1[(size_t)k * 2 + 0] = (hp.ramp[k] - (k > 0 ? hp.ramp[k - 1] : 0.0)) / S->tau;
      c1[(size_t)k * 2 + 1] = hp.ramp[k];
    }
    for (int i = 0; i < nxi; ++i) {
      c2[((size_t)0 * nxi + i) * rb + 0] = e1[i];
      for (int v = 0; v < nv; ++v)
        c2[((size_t)1 * nxi + i) * rb + 1 + v] = hp.Gvisc[((size_t)v * nxi + i) * nxi + 0];
    }
    std::vector<double> c3((size_t)2 * ns * rb, 0.0), pc3(hp.n_p, 0.0);
    for (int comp = 0; comp < 2; ++comp)
      for (int i = 0; i < ns; ++i) {
        double sm = 0;
        for (int t = hp.Kfa.rowptr[i]; t < hp.Kfa.rowptr[i + 1]; ++t)
          sm += hp.Mfa[t] * hp.g_all[(size_t)comp * nall + hp.Kfa.col[t]];
        c3[((size_t)comp * ns + i) * rb + 0] = -sm;
        for (int v = 0; v < nv; ++v) {
          double sa = 0;
          for (int t = hp.Kfa.rowptr[i]; t < hp.Kfa.rowptr[i + 1]; ++t)
            sa += hp.Afa_visc[v][t] * hp.g_all[(size_t)comp * nall + hp.Kfa.col[t]];
          c3[((size_t)comp * ns + i) * rb + 1 + v] = -sa;
        }
      }
    for (int k = 0; k < hp.n_p; ++k) {
      double s = 0;
      for (int t = hp.Ball.rowptr[k]; t < hp.Ball.rowptr[k + 1]; ++t) s += hp.Ball.val[t] * hp.g_all[hp.Ball.col[t]];
      pc3[k] = -s;
    }
    S->bu = tt_new(c, nt, nxi, hp.n_u, 2, rb);
    SGTT_HIP(hipMemcpyAsync(S->bu.c1, c1.data(), c1.size() * 8, hipMemcpyHostToDevice, c.s));
    SGTT_HIP(hipMemcpyAsync(S->bu.c2, c2.data(), c2.size() * 8, hipMemcpyHostToDevice, c.s));
    SGTT_HIP(hipMemcpyAsync(S->bu.c3, c3.data(), c3.size() * 8, hipMemcpyHostToDevice, c.s));
    S->bp = tt_new(c, nt, nxi, hp.n_p, 1, 1);
    SGTT_HIP(hipMemcpyAsync(S->bp.c1, hp.ramp.data(), nt * 8, hipMemcpyHostToDevice, c.s));
    SGTT_HIP(hipMemcpyAsync(S->bp.c2, e1.data(), nxi * 8, hipMemcpyHostToDevice, c.s));
    SGTT_HIP(hipMemcpyAsync(S->bp.c3, pc3.data(), hp.n_p * 8, hipMemcpyHostToDevice, c.s));
    tt_dot(c, S->bu, S->bu, S->dsc + 30010, 0);
    tt_dot(c, S->bp, S->bp, S->dsc + 30010, 1);
    SGTT_HIP(hipMemcpyAsync(c.hdbl, S->dsc + 30010, sizeof(double), hipMemcpyDeviceToHost, c.s));
    c.sync();
    S->rhs_norm = std::sqrt(std::max(c.hdbl[0], 0.0));
  } else {
    check_tt(prior->u, nt, nxi, hp.n_u);
    check_tt(prior->p, nt, nxi, hp.n_p);
    // wind over all nodes: embed free velocity, then add the lift
    const sgtt_tt& pu = prior->u;
    TT wemb = tt_new(c, nt, nxi, 2 * nall, pu.r1, pu.r2);
    SGTT_HIP(hipMemcpyAsync(wemb.c1, pu.core1, sizeof(double) * pu.n1 * pu.r1, hipMemcpyDeviceToDevice, c.s));
    SGTT_HIP(hipMemcpyAsync(wemb.c2, pu.core2, sizeof(double) * pu.r1 * pu.n2 * pu.r2, hipMemcpyDeviceToDevice, c.s));
    {
      std::vector<double> hu((size_t)hp.n_u * pu.r2), ha((size_t)2 * nall * pu.r2, 0.0);
      SGTT_HIP(hipMemcpyAsync(hu.data(), pu.core3, hu.size() * 8, hipMemcpyDeviceToHost, c.s));
      c.sync();
      for (int comp = 0; comp < 2; ++comp)
        for (int i = 0; i < ns; ++i) {
          int node = hp.mesh.free_nodes[i];
          std::memcpy(&ha[((size_t)comp * nall + node) * pu.r2], &hu[((size_t)comp * ns + i) * pu.r2],
                      sizeof(double) * pu.r2);
        }
      SGTT_HIP(hipMemcpyAsync(wemb.c3, ha.data(), ha.size() * 8, hipMemcpyHostToDevice, c.s));
      c.sync();
    }
    TT wall = tt_concat(c, {&wemb, &lift}, nullptr, {});
    TT wtil = tt_round(c, wall, desc->eps_conv, nullptr, nullptr);
    build_convection(*S, c, wtil);
    // right-hand side r = -(L_{free,all}(w) w_all + B^T p) with the
    // untruncated wind (eq. 3.15, sec. 4.3): the linear terms as an exact
    // TT, expanded to full format, minus the stochastic Galerkin
    // convection N(w_all) w_all evaluated in full format element by
    // element (its TT ranks would be the squares of the iterate's)
    {
      if (nxi > 64) throw SgttError(-1, "Picard residual: n_xi > 64 not supported");
      std::vector<const double*> fa{hp.Mfa.data()};
      for (const auto& a : hp.Afa_visc) fa.push_back(a.data());
      DevCsr Kfa = upload_csr(c, hp.Kfa, fa);
      const int nv = hp.nvisc;
      DevCsr Ball = upload_csr(c, hp.Ball, {hp.Ball.val.data()});
      const TT& w = wall;
      TT pview = tt_view(prior->p.n1, prior->p.n2, prior->p.n3, prior->p.r1, prior->p.r2, prior->p.core1,
                         prior->p.core2, prior->p.core3);
      TT uview = tt_view(pu.n1, pu.n2, pu.n3, pu.r1, pu.r2, pu.core1, pu.core2, pu.core3);
      const TT& p = pview;
      const int r1u = w.r1, r2u = w.r2, r1p = p.r1, r2p = p.r2;
      const int R1 = 2 * r1u + r1p, R2 = (1 + nv) * r2u + r2p;
      TT ru = tt_new(c, nt, nxi, hp.n_u, R1, R2);
      core1_op(c.s, 0, nt, r1u, w.c1, r1u, ru.c1, R1, 0, 1.0 / S->tau);
      core1_op(c.s, 1, nt, r1u, w.c1, r1u, ru.c1, R1, r1u, 1.0);
      core1_op(c.s, 1, nt, r1p, p.c1, r1p, ru.c1, R1, 2 * r1u, 1.0);
      copy2d(c.s, nt, R1, ru.c1, R1, ru.c1, R1, -1.0, nullptr, 0);   // r = -(...)
      fill(c.s, ru.c2, ru.n_c2(), 0.0);
      core2_block(c.s, r1u, nxi, r2u, w.c2, nullptr, 1, 1, ru.c2, R1, R2, 0, 0);
      core2_block(c.s, r1u, nxi, r2u, w.c2, S->Gvisc, 1, nv, ru.c2, R1, R2, r1u, r2u);
      core2_block(c.s, r1p, nxi, r2p, p.c2, nullptr, 1, 1, ru.c2, R1, R2, 2 * r1u, (1 + nv) * r2u);
      spmm(c.s, ns, 2, nall, ns, Kfa.rowptr, Kfa.col, Kfa.vals, 1 + nv, Kfa.nnz, w.c3, r2u, 0, r2u, ru.c3, R2, 0,
           r2u, 1.0);
      spmm(c.s, hp.n_u, 1, 0, 0, S->Btd.rowptr, S->Btd.col, S->Btd.vals, 1, 0, p.c3, r2p, 0, r2p, ru.c3, R2,
           (1 + nv) * r2u, 0, 1.0, 0.0, S->Btd.max_row);
      TT rp = tt_new(c, nt, nxi, hp.n_p, r1u, r2u);
      copy2d(c.s, nt, r1u, w.c1, r1u, rp.c1, r1u, -1.0, nullptr, 0);
      SGTT_HIP(hipMemcpyAsync(rp.c2, w.c2, sizeof(double) * w.n_c2(), hipMemcpyDeviceToDevice, c.s));
      spmm(c.s, hp.n_p, 1, 0, 0, Ball.rowptr, Ball.col, Ball.vals, 1, 0, w.c3, r2u, 0, r2u, rp.c3, r2u, 0, 0, 1.0);
      // device copies of the mesh, lift and chaos triple products
      std::vector<int> conn9((size_t)hp.mesh.conn.size() * 9);
      for (size_t e = 0; e < hp.mesh.conn.size(); ++e)
        for (int a = 0; a < 9; ++a) conn9[e * 9 + a] = hp.mesh.conn[e][a];
      std::vector<int> hrow(nxi + 1, 0), hl, hk;
      std::vector<double> hv;
      for (int i = 0; i < nxi; ++i) {
        for (int l = 0; l < nxi; ++l)
          for (int k = 0; k < nxi; ++k) {
            double v = hp.H[((size_t)l * nxi + i) * nxi + k];
            if (v == 0.0) continue;
            hl.push_back(l);
            hk.push_back(k);
            hv.push_back(v);
          }
        hrow[i + 1] = (int)hv.size();
      }
      std::vector<double> reft(252);
      reference_tables(reft.data());
      int* d_conn = dev_upload(c, conn9);
      int* d_fid = dev_upload(c, hp.mesh.free_id);
      int* d_hrow = dev_upload(c, hrow);
      int* d_hl = dev_upload(c, hl);
      int* d_hk = dev_upload(c, hk);
      double* d_hv = dev_upload(c, hv);
      double* d_ref = dev_upload(c, reft);
      double* d_ramp = dev_upload(c, hp.ramp);
      double* d_gall = dev_upload(c, hp.g_all);
      const long nu_full = (long)nt * nxi * hp.n_u;
      double* R = c.pool.get(nu_full);
      double* U = c.pool.get(nu_full);
      tt_expand(c, ru, R);
      tt_expand(c, uview, U);
      sg_convection_full(c.s, nt, nxi, hp.n_u, ns, nall, (int)hp.mesh.conn.size(), d_conn, d_fid, U, d_ramp, d_gall,
                         d_hrow, d_hl, d_hk, d_hv, d_ref, 0.5 * hp.prm.h, -1.0, R);
      c.pool.put(U);
      // ||r||^2 of the untruncated nonlinear residual (Alg. 3.1, line 7)
      double* ws = c.scratch(1 << 16);
      double* sq = S->dsc + 30010;
      sumsq(c.s, R, nu_full, sq, ws, 1 << 16);
      S->bu = tt_from_full(c, R, nt, nxi, hp.n_u, desc->eps_rhs, nullptr);
      c.pool.put(R);
      const long np_full = (long)nt * nxi * hp.n_p;
      double* Rp = c.pool.get(np_full);
      tt_expand(c, rp, Rp);
      sumsq(c.s, Rp, np_full, sq + 1, ws, 1 << 16);
      S->bp = tt_from_full(c, Rp, nt, nxi, hp.n_p, desc->eps_rhs, nullptr);
      c.pool.put(Rp);
      SGTT_HIP(hipMemcpyAsync(c.hdbl, sq, 2 * sizeof(double), hipMemcpyDeviceToHost, c.s));
      c.sync();
      S->rhs_norm = std::sqrt(c.hdbl[0] + c.hdbl[1]);
      Kfa.free_all();
      Ball.free_all();
      for (void* q : {(void*)d_conn, (void*)d_fid, (void*)d_hrow, (void*)d_hl, (void*)d_hk, (void*)d_hv,
                      (void*)d_ref, (void*)d_ramp, (void*)d_gall})
        (void)hipFree(q);
    }
  }
  c.sync();
  S->setup_s = now_s() - t0;
  return S.release();
}

int sgtt_assemble(sgtt_context* ctx, const sgtt_problem_desc* desc, const sgtt_tt_pair* prior, sgtt_system** out) {
  if (!ctx || !desc || !out) return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    *out = assemble_internal(ctx, desc, prior);
    context_add_child(ctx);
  });
}

int sgtt_system_destroy(sgtt_system* sys) {
  if (!sys) return SGTT_E_INVALID;
  sgtt_context* ctx = sys->ctx;
  (void)hipStreamSynchronize(ctx->c.s);
  delete sys;
  context_release_child(ctx);
  return SGTT_OK;
}

int sgtt_system_info_get(const sgtt_system* S, sgtt_system_info* info) {
  if (!S || !info) return SGTT_E_INVALID;
  info->n_s = S->ns;
  info->n_u = S->nu;
  info->n_p = S->np;
  info->n_xi = S->nxi;
  info->nt = S->nt;
  info->n_all = S->nall;
  info->conv_r1 = S->k1;
  info->conv_r2 = S->k2;
  info->rhs_r1u = S->bu.r1;
  info->rhs_r2u = S->bu.r2;
  info->rhs_r1p = S->bp.r1;
  info->rhs_r2p = S->bp.r2;
  info->setup_seconds = S->setup_s;
  info->rhs_norm = S->rhs_norm;
  return SGTT_OK;
}

int sgtt_rhs(sgtt_system* S, sgtt_tt_pair* b) {
  if (!S || !b) return SGTT_E_INVALID;
  sgtt_context* ctx = S->ctx;
  return guarded(ctx, [&]() {
    Vec v;
    v.nc = 2;
    v.c[0] = tt_view(S->bu.n1, S->bu.n2, S->bu.n3, S->bu.r1, S->bu.r2, S->bu.c1, S->bu.c2, S->bu.c3);
    v.c[1] = tt_view(S->bp.n1, S->bp.n2, S->bp.n3, S->bp.r1, S->bp.r2, S->bp.c1, S->bp.c2, S->bp.c3);
    write_pair(ctx->c, v, b);
    ctx->c.sync();
  });
}

int sgtt_apply(sgtt_system* S, const sgtt_tt_pair* x, sgtt_tt_pair* y, double eps) {
  if (!S || !x || !y) return SGTT_E_INVALID;
  sgtt_context* ctx = S->ctx;
  return guarded(ctx, [&]() {
    check_tt(x->u, S->nt, S->nxi, S->nu);
    check_tt(x->p, S->nt, S->nxi, S->np);
    Vec xv = vec_from_pair(x);
    Vec yv = apply_L(*S, xv);
    if (eps > 0) yv = vec_round(ctx->c, yv, eps, nullptr, nullptr);
    write_pair(ctx->c, yv, y);
    ctx->c.sync();
  });
}

int sgtt_precondition(sgtt_system* S, const sgtt_tt_pair* r, sgtt_tt_pair* z, const sgtt_solve_opts* opts,
                      sgtt_solve_stats* stats) {
  if (!S || !r || !z) return SGTT_E_INVALID;
  sgtt_context* ctx = S->ctx;
  return guarded(ctx, [&]() {
    check_tt(r->u, S->nt, S->nxi, S->nu);
    check_tt(r->p, S->nt, S->nxi, S->np);
    sgtt_solve_opts o = opts ? *opts : default_opts();
    Vec rv = vec_from_pair(r);
    SolveCounters cnt;
    Vec zv = lsc_precondition(*S, rv, prec_opts(&o), &cnt);
    write_pair(ctx->c, zv, z);
    ctx->c.sync();
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->inner_iters = cnt.inner;
    }
  });
}

int sgtt_bcr_variant_count(void) { return bcr_variant_count(); }

int sgtt_bcr_apply(sgtt_system* S, int which, int variant, int ncols, const double* b, double* x) {
  if (!S || !b || !x || ncols <= 0 || (which != 0 && which != 1) || variant < -1 ||
      variant >= bcr_variant_count())
    return SGTT_E_INVALID;
  sgtt_context* ctx = S->ctx;
  return guarded(ctx, [&]() {
    Ctx& c = ctx->c;
    const BcrDev& f = which == 0 ? S->Fbt : S->Xbt;
    const int ncomp = which == 0 ? 2 : 1;
    if (variant >= 0 && !bcr_variant_takes(f, variant))
      throw SgttError(SGTT_E_INVALID, "block cyclic reduction: blocks too large for the variant");
    const size_t n = (size_t)ncomp * f.n * ncols;
    // the reduction overwrites its right-hand side: it works on a copy, which
    // goes back to the pool on every way out
    struct Held {
      Pool& pool;
      double* p;
      ~Held() { pool.put(p); }
    } w{c.pool, c.pool.get(n)};
    SGTT_HIP(hipMemcpyAsync(w.p, b, sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
    if (variant < 0)
      bcr_solve(c.s, f, ncomp, w.p, ncols, x, ncols, ncols);
    else
      bcr_solve_variant(c.s, f, ncomp, w.p, ncols, x, ncols, ncols, variant);
    c.sync();
  });
}

int sgtt_bcr_apply_noalloc(sgtt_system* S, int which, int variant, int ncols, const double* b, double* x) {
  if (!S || !b || !x || ncols <= 0 || (which != 0 && which != 1) || variant < -1 ||
      variant >= bcr_variant_count())
    return SGTT_E_INVALID;
  sgtt_context* ctx = S->ctx;
  return guarded(ctx, [&]() {
    Ctx& c = ctx->c;
    const BcrDev& f = which == 0 ? S->Fbt : S->Xbt;
    const int ncomp = which == 0 ? 2 : 1;
    const size_t n = (size_t)ncomp * f.n * ncols;
    if (n > (size_t)SGTT_NOALLOC_SCRATCH_DOUBLES)
      throw SgttError(SGTT_E_INVALID, "sgtt_bcr_apply_noalloc: " + std::to_string(n) +
                                          " right-hand-side values exceed the scratch of " +
                                          std::to_string((long)SGTT_NOALLOC_SCRATCH_DOUBLES) + " doubles");
    if (!ctx->scratch) throw SgttError(SGTT_E_INVALID, "context has no scratch address");
    // the whole working copy is overwritten before the reduction reads it,
    // so what an earlier call left in the scratch is never seen
    SGTT_HIP(hipMemcpyAsync(ctx->scratch, b, sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
    bcr_solve_untuned(c.s, f, ncomp, ctx->scratch, ncols, x, ncols, ncols, variant);
    SGTT_HIP(hipGetLastError());
  });
}

int sgtt_round(sgtt_context* ctx, sgtt_tt* x, double eps, int max_rank) {
  if (!ctx || !x) return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    check_dtype(*x);
    if (x->r1 < 1 || x->r2 < 1 || x->r1 > x->cap1 || x->r2 > x->cap2) throw SgttError(-1, "invalid TT");
    TT v = tt_view(x->n1, x->n2, x->n3, x->r1, x->r2, x->core1, x->core2, x->core3);
    TT r = tt_round(ctx->c, v, eps, nullptr, nullptr, max_rank > 0 ? max_rank : RANK_CAP_LARGE);
    write_tt(ctx->c, r, x);
    ctx->c.sync();
  });
}

int sgtt_dot(sgtt_context* ctx, const sgtt_tt_pair* x, const sgtt_tt_pair* y, double* out) {
  if (!ctx || !x || !y || !out) return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    Vec xv = vec_from_pair(x), yv = vec_from_pair(y);
    vec_dot(ctx->c, xv, yv, ctx->c.dscal + 200);
    *out = read_double(ctx->c, ctx->c.dscal + 200);
    if (!std::isfinite(*out)) throw SgttError(-5, "non-finite inner product");
  });
}

int sgtt_axpby(sgtt_context* ctx, double alpha, const sgtt_tt_pair* x, double beta, sgtt_tt_pair* y) {
  if (!ctx || !x || !y) return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    Vec xv = vec_from_pair(x), yv = vec_from_pair(y);
    Vec s = vec_concat(ctx->c, {&xv, &yv}, nullptr, {alpha, beta});
    write_pair(ctx->c, s, y);
    ctx->c.sync();
  });
}

int sgtt_expand(sgtt_context* ctx, const sgtt_tt* x, double* out) {
  if (!ctx || !x || !out) return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    check_dtype(*x);
    TT v = tt_view(x->n1, x->n2, x->n3, x->r1, x->r2, x->core1, x->core2, x->core3);
    tt_expand(ctx->c, v, out);
    ctx->c.sync();
  });
}

int sgtt_hessenberg_lsq(sgtt_context* ctx, const double* H, int k, double beta, double* y, double* resid) {
  if (!ctx || !H || !y || k < 1 || k > 120) return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    Ctx& c = ctx->c;
    double* dH = c.pool.get((size_t)(k + 1) * k + k + 4);
    double* dy = dH + (size_t)(k + 1) * k;
    double* db = dy + k;
    SGTT_HIP(hipMemcpyAsync(dH, H, sizeof(double) * (k + 1) * k, hipMemcpyHostToDevice, c.s));
    SGTT_HIP(hipMemcpyAsync(db, &beta, sizeof(double), hipMemcpyHostToDevice, c.s));
    hessenberg_lsq(c.s, dH, k + 1, k, db, dy, db + 1);
    SGTT_HIP(hipMemcpyAsync(y, dy, sizeof(double) * k, hipMemcpyDeviceToHost, c.s));
    double r = 0;
    SGTT_HIP(hipMemcpyAsync(c.hdbl, db + 1, sizeof(double), hipMemcpyDeviceToHost, c.s));
    c.sync();
    r = c.hdbl[0];
    if (resid) *resid = r;
    c.pool.put(dH);
  });
}

int sgtt_gemm(sgtt_context* ctx, int m, int n, int k, double alpha, const double* A, long lda, const double* B,
              long ldb, double beta, double* C, long ldc) {
  if (!ctx || !C || m < 1 || n < 1 || k < 0 || ldc < n || (k > 0 && (!A || !B || lda < k || ldb < n)))
    return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    GemmPrecisionScope f64(GP_F64);
    gemm(ctx->c.s, 1, m, n, k, alpha, A, 0, lda, 1, B, 0, ldb, 1, beta, C, 0, ldc, 1);
    ctx->c.sync();
  });
}

int sgtt_solve_history(const sgtt_system* S, int max_records, sgtt_iter_record* out, int* nrecords) {
  if (!S || !nrecords || max_records < 0 || (max_records > 0 && !out)) return SGTT_E_INVALID;
  const int n = (int)S->hist.size();
  *nrecords = n;
  for (int i = 0; i < n && i < max_records; ++i) out[i] = S->hist[i];
  return SGTT_OK;
}

int sgtt_pair_save(sgtt_context* ctx, const sgtt_tt_pair* x, const char* path) {
  if (!ctx || !x || !path) return SGTT_E_INVALID;
  int st = SGTT_OK;
  const int g = guarded(ctx, [&]() {
    const sgtt_tt* t[2] = {&x->u, &x->p};
    int dims[10];
    std::vector<double> host[6];
    for (int q = 0; q < 2; ++q) {
      const sgtt_tt& a = *t[q];
      check_dtype(a);
      if (a.r1 < 1 || a.r2 < 1 || a.r1 > a.cap1 || a.r2 > a.cap2 || !a.core1 || !a.core2 || !a.core3)
        throw SgttError(SGTT_E_INVALID, "checkpoint: invalid TT");
      const int d[5] = {a.n1, a.n2, a.n3, a.r1, a.r2};
      std::memcpy(dims + 5 * q, d, sizeof(d));
      const double* src[3] = {a.core1, a.core2, a.core3};
      const long len[3] = {(long)a.n1 * a.r1, (long)a.r1 * a.n2 * a.r2, (long)a.n3 * a.r2};
      for (int w = 0; w < 3; ++w) {
        host[3 * q + w].resize((size_t)len[w]);
        SGTT_HIP(hipMemcpyAsync(host[3 * q + w].data(), src[w], sizeof(double) * len[w], hipMemcpyDeviceToHost,
                                ctx->c.s));
      }
    }
    ctx->c.sync();
    const double* cores[6];
    for (int i = 0; i < 6; ++i) cores[i] = host[i].data();
    st = pair_file_write(path, dims, cores);
    if (st != SGTT_OK) ctx->err = std::string("checkpoint: cannot write ") + path;
  });
  return g != SGTT_OK ? g : st;
}

int sgtt_pair_load(sgtt_context* ctx, const char* path, sgtt_tt_pair* x) {
  if (!ctx || !x || !path) return SGTT_E_INVALID;
  int st = SGTT_OK;
  const int g = guarded(ctx, [&]() {
    sgtt_tt* t[2] = {&x->u, &x->p};
    int caps[10], dims[10];
    std::vector<double> host[6];
    double* cores[6];
    for (int q = 0; q < 2; ++q) {
      const sgtt_tt& a = *t[q];
      check_dtype(a);
      if (a.cap1 < 1 || a.cap2 < 1 || !a.core1 || !a.core2 || !a.core3)
        throw SgttError(SGTT_E_INVALID, "checkpoint: invalid destination TT");
      const int c[5] = {a.n1, a.n2, a.n3, a.cap1, a.cap2};
      std::memcpy(caps + 5 * q, c, sizeof(c));
      const long len[3] = {(long)a.n1 * a.cap1, (long)a.cap1 * a.n2 * a.cap2, (long)a.n3 * a.cap2};
      for (int w = 0; w < 3; ++w) {
        host[3 * q + w].resize((size_t)len[w]);
        cores[3 * q + w] = host[3 * q + w].data();
      }
    }
    st = pair_file_read(path, caps, cores, dims);
    if (st != SGTT_OK) {
      ctx->err = std::string("checkpoint: cannot load ") + path;
      return;
    }
    for (int q = 0; q < 2; ++q) {
      sgtt_tt& a = *t[q];
      const int r1 = dims[5 * q + 3], r2 = dims[5 * q + 4];
      double* dst[3] = {a.core1, a.core2, a.core3};
      const long len[3] = {(long)a.n1 * r1, (long)r1 * a.n2 * r2, (long)a.n3 * r2};
      for (int w = 0; w < 3; ++w)
        SGTT_HIP(hipMemcpyAsync(dst[w], host[3 * q + w].data(), sizeof(double) * len[w], hipMemcpyHostToDevice,
                                ctx->c.s));
      set_ranks(ctx->c, &a, r1, r2);
    }
    ctx->c.sync();
  });
  return g != SGTT_OK ? g : st;
}

int sgtt_residual(sgtt_system* S, const sgtt_tt_pair* b, const sgtt_tt_pair* x, double* rel) {
  if (!S || !b || !x || !rel) return SGTT_E_INVALID;
  sgtt_context* ctx = S->ctx;
  return guarded(ctx, [&]() {
    check_tt(x->u, S->nt, S->nxi, S->nu);
    check_tt(x->p, S->nt, S->nxi, S->np);
    Vec bv = vec_from_pair(b), xv = vec_from_pair(x);
    *rel = full_residual(*S, bv, xv, nullptr, nullptr, 0.0, nullptr);
  });
}

int sgtt_residual_tensor(sgtt_system* S, const sgtt_tt_pair* b, const sgtt_tt_pair* x, double* ru, double* rp,
                         double* rel) {
  if (!S || !b || !x || !ru || !rp || !rel) return SGTT_E_INVALID;
  sgtt_context* ctx = S->ctx;
  return guarded(ctx, [&]() {
    check_tt(b->u, S->nt, S->nxi, S->nu);
    check_tt(b->p, S->nt, S->nxi, S->np);
    check_tt(x->u, S->nt, S->nxi, S->nu);
    check_tt(x->p, S->nt, S->nxi, S->np);
    Vec bv = vec_from_pair(b), xv = vec_from_pair(x);
    double* outs[2] = {ru, rp};
    *rel = full_residual(*S, bv, xv, nullptr, nullptr, 0.0, nullptr, outs);
  });
}

// Refinement cycles of Alg. 4.2 until the exact relative residual is <= tol
// (throws SgttError).  Returns SGTT_OK or SGTT_W_NOT_CONVERGED; z is the
// exact sum of the cycle corrections.
int solve_internal(sgtt_system* S, const Vec& bv, const sgtt_solve_opts& o, Vec& z, sgtt_solve_stats* stats) {
  Ctx& c = S->ctx->c;
  if (o.restart < 1 || o.restart > 60 || o.max_cycles < 1 || o.inner_maxit < 1 || o.inner_maxit > 60)
    throw SgttError(-1, "invalid solve options");
  double t0 = now_s();
  long r0 = c.roundings + side_roundings(c);
  const long a0 = c.pool.device_allocs() + kernel_device_allocs() + side_device_allocs(c) + S->mg_allocs;
  const long g0 = S->mg_launches;
  SolveCounters cnt;
  cnt.verbose = o.verbose;
  cnt.t_start = t0;
  S->hist.clear();
  cnt.hist = &S->hist;
  OuterSpace sp(*S, prec_opts(&o), &cnt);
  // an FP32 application adds at most kF32MeanSolveError of itself to the
  // solution, and its size follows the residual it is applied to: below
  // this level that stays under the refinement cycle's compression
  sp.f32_below = 0.05 * o.tol / kF32MeanSolveError;
  S->mlp_off = false;
  S->mlp_fails = 0;
  S->mlp_calls = 0;
  {
    // a non-finite right-hand side is refused before any rounding sees it
    // (the inner product is plain products and sums)
    double* d = S->dsc + 30020;
    vec_dot(c, bv, bv, d);
    if (!std::isfinite(read_double(c, d))) throw SgttError(-5, "non-finite right-hand side");
  }
  std::vector<Vec> terms;
  Vec r = vec_copy(c, bv);
  double bn2 = -1.0, rel = 1.0;
  int cycles = 0;
  for (int cyc = 0; cyc < o.max_cycles; ++cyc) {
    int its = 0;
    double rr = 0;
    cnt.cycle = cyc;
    sp.cycle_rel = rel;   // the cycle solves L d = r_j, ||r_j|| = rel ||b||
    Vec d = lowrank_fgmres(c, sp, r, o.tol_cycle, o.eps_krylov, o.restart, S->dsc, its, rr, &cnt, "outer",
                           o.outer_explicit != 0, o.relax != 0);
    cnt.outer += its;
    ++cycles;
    terms.push_back(std::move(d));
    std::vector<const Vec*> parts;
    for (auto& t : terms) parts.push_back(&t);
    z = vec_concat(c, parts, nullptr, {});
    Vec rnext;
    // the correction equation L d = r_j only has to be solved to relative
    // accuracy tol ||b|| / ||r_j||, so its right-hand side is compressed
    // to a fraction of that (never finer than eps_krylov)
    double eps_r = o.eps_krylov;
    rel = full_residual(*S, bv, z, nullptr, nullptr, 0.0, &bn2);
    if (rel > o.tol && cyc + 1 < o.max_cycles) {
      const double fac = o.cycle_rhs_factor > 0.0 ? o.cycle_rhs_factor : 0.05;
      eps_r = std::max(o.eps_krylov, std::min(1e-3, fac * o.tol / std::max(rel, 1e-300)));
      full_residual(*S, bv, z, nullptr, &rnext, eps_r, &bn2);
    }
    {
      // end of a refinement cycle: the exact residual of the accumulated
      // solution against b, and that solution's ranks
      sgtt_iter_record h{};
      h.cycle = cyc;
      h.iter = -1;
      h.rel = rel;
      hist_ranks(z, h.rank_z_u, h.rank_z_p);
      h.seconds = now_s() - t0;
      S->hist.push_back(h);
    }
    if (o.verbose) fprintf(stderr, "[sgtt] cycle %d: outer its %d, exact rel residual %.3e\n", cyc, its, rel);
    if (!std::isfinite(rel)) throw SgttError(-5, "non-finite residual");
    if (rel <= o.tol) break;
    if (o.verbose) fprintf(stderr, "[sgtt] next right-hand side truncated at %.2e\n", eps_r);
    r = std::move(rnext);
  }
  if (stats) {
    stats->cycles = cycles;
    stats->outer_iters = cnt.outer;
    stats->inner_iters = cnt.inner;
    stats->rel_residual = rel;
    stats->seconds = now_s() - t0;
    stats->max_rank_krylov_u = cnt.maxr_u;
    stats->max_rank_krylov_p = cnt.maxr_p;
    stats->roundings = (int)(c.roundings + side_roundings(c) - r0);
    stats->t_apply = cnt.t_apply;
    stats->t_round = 0;
    stats->t_precond = cnt.t_prec;
    stats->t_residual = 0;
    stats->learned_calls = S->mlp_calls;
    stats->learned_fallback = S->mlp_off ? 1 : 0;
    stats->f32_applications = cnt.f32_applications;
    stats->device_allocs =
        c.pool.device_allocs() + kernel_device_allocs() + side_device_allocs(c) + S->mg_allocs - a0;
    stats->graph_launches = S->mg_launches - g0;
  }
  return rel > o.tol ? SGTT_W_NOT_CONVERGED : SGTT_OK;
}

int sgtt_solve(sgtt_system* S, const sgtt_tt_pair* b, sgtt_tt_pair* x, const sgtt_solve_opts* opts,
               sgtt_solve_stats* stats) {
  if (!S || !b || !x) return SGTT_E_INVALID;
  sgtt_context* ctx = S->ctx;
  int status = SGTT_OK;
  try {
    check_tt(b->u, S->nt, S->nxi, S->nu);
    check_tt(b->p, S->nt, S->nxi, S->np);
    sgtt_solve_opts o = opts ? *opts : default_opts();
    Vec z;
    status = solve_internal(S, vec_from_pair(b), o, z, stats);
    write_pair(ctx->c, z, x);
    ctx->c.sync();
  } catch (const SgttError& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return SGTT_E_INVALID;
  }
  return status;
}

int sgtt_solve_batched(sgtt_system* const* systems, int n, const sgtt_tt_pair* const* b, sgtt_tt_pair* const* x,
                       const sgtt_solve_opts* opts, sgtt_solve_stats* stats, int* status) {
  if (n < 0 || (n > 0 && (!systems || !b || !x || !status))) return SGTT_E_INVALID;
  for (int i = 0; i < n; ++i)
    if (!systems[i] || !b[i] || !x[i]) return SGTT_E_INVALID;
  // one worker per context: its problems run in order on its stream, the
  // contexts' streams run concurrently on the device
  std::vector<sgtt_context*> ctxs;
  std::vector<std::vector<int>> work;
  for (int i = 0; i < n; ++i) {
    sgtt_context* c = systems[i]->ctx;
    size_t w = 0;
    while (w < ctxs.size() && ctxs[w] != c) ++w;
    if (w == ctxs.size()) {
      ctxs.push_back(c);
      work.emplace_back();
    }
    work[w].push_back(i);
  }
  // with several contexts their streams already fill the device, and a
  // process has few hardware queues (four by default): each context's side
  // lanes (the pressure rounding and solution lanes) would queue behind the
  // other contexts' main streams, so they are switched off for the batch
  const bool lanes = ctxs.size() == 1;
  auto run = [&](size_t w) {
    Ctx& c = ctxs[w]->c;
    const bool was = c.side_enabled;
    c.side_enabled = was && lanes;
    for (int i : work[w]) {
      sgtt_solve_stats st{};
      status[i] = sgtt_solve(systems[i], b[i], x[i], opts, &st);
      if (stats) stats[i] = st;
    }
    c.side_enabled = was;
  };
  std::vector<std::thread> th;
  for (size_t w = 1; w < ctxs.size(); ++w) th.emplace_back(run, w);
  if (!ctxs.empty()) run(0);
  for (auto& t : th) t.join();
  int worst = SGTT_OK;
  for (int i = 0; i < n; ++i) {
    if (status[i] < 0) return SGTT_E_INVALID;
    if (status[i] > worst) worst = status[i];
  }
  return worst;
}

// Picard's method (Alg. 3.1) with truncated iterates (eq. 4.8).
int sgtt_picard(sgtt_context* ctx, const sgtt_problem_desc* desc, const sgtt_picard_opts* opts, sgtt_tt_pair* x,
                sgtt_picard_stats* stats) {
  if (!ctx || !desc || !opts || !x) return SGTT_E_INVALID;
  if (opts->max_steps < 0 || opts->max_steps > SGTT_PICARD_MAX_STEPS) return SGTT_E_INVALID;
  if (opts->update_mode != 0 && opts->update_mode != 1) return SGTT_E_INVALID;
  int status = SGTT_OK;
  try {
    Ctx& c = ctx->c;
    const double t0 = now_s();
    sgtt_picard_stats st;
    std::memset(&st, 0, sizeof(st));
    // line 1: Stokes solve for the initial iterate
    double ta = now_s();
    std::unique_ptr<sgtt_system> S(assemble_internal(ctx, desc, nullptr));
    st.assemble_seconds[0] = now_s() - ta;
    const double fnorm = S->rhs_norm;
    auto record = [&](int i, const sgtt_solve_stats& ls, const Vec& it) {
      st.linear_residual[i] = ls.rel_residual;
      st.outer_iters[i] = ls.outer_iters;
      st.inner_iters[i] = ls.inner_iters;
      st.solve_seconds[i] = ls.seconds;
      st.stored_rank_u[i][0] = it.c[0].r1;
      st.stored_rank_u[i][1] = it.c[0].r2;
      st.stored_rank_p[i][0] = it.c[1].r1;
      st.stored_rank_p[i][1] = it.c[1].r2;
      if (opts->update_mode == 1 && opts->eps_soln > 0 && i > 0) {
        // the ranks eq. 4.8 would give: the stored sum rounded at eps_soln
        Vec r = vec_round(c, it, opts->eps_soln, nullptr, nullptr);
        st.rank_u[i][0] = r.c[0].r1;
        st.rank_u[i][1] = r.c[0].r2;
        st.rank_p[i][0] = r.c[1].r1;
        st.rank_p[i][1] = r.c[1].r2;
      } else {
        st.rank_u[i][0] = it.c[0].r1;
        st.rank_u[i][1] = it.c[0].r2;
        st.rank_p[i][0] = it.c[1].r1;
        st.rank_p[i][1] = it.c[1].r2;
      }
    };
    Vec cur;
    {
      Vec b;
      b.c[0] = tt_view(S->bu.n1, S->bu.n2, S->bu.n3, S->bu.r1, S->bu.r2, S->bu.c1, S->bu.c2, S->bu.c3);
      b.c[1] = tt_view(S->bp.n1, S->bp.n2, S->bp.n3, S->bp.r1, S->bp.r2, S->bp.c1, S->bp.c2, S->bp.c3);
      Vec z;
      sgtt_solve_stats ls{};
      if (solve_internal(S.get(), b, opts->solve, z, &ls) != SGTT_OK) status = SGTT_W_NOT_CONVERGED;
      cur = opts->eps_soln > 0 ? vec_round(c, z, opts->eps_soln, nullptr, nullptr) : std::move(z);
      record(0, ls, cur);
    }
    S.reset();
    int i = 0;
    for (;;) {
      // lines 6-7: convection matrix and nonlinear residual of the current iterate
      sgtt_tt_pair prior{};
      for (int q = 0; q < 2; ++q) {
        sgtt_tt& t = q == 0 ? prior.u : prior.p;
        const TT& src = cur.c[q];
        t.n1 = src.n1;
        t.n2 = src.n2;
        t.n3 = src.n3;
        t.r1 = t.cap1 = src.r1;
        t.r2 = t.cap2 = src.r2;
        t.core1 = src.c1;
        t.core2 = src.c2;
        t.core3 = src.c3;
      }
      ta = now_s();
      S.reset(assemble_internal(ctx, desc, &prior));
      st.assemble_seconds[i + 1] = now_s() - ta;
      st.nonlinear_residual[i] = fnorm > 0 ? S->rhs_norm / fnorm : 0.0;
      if (opts->solve.verbose)
        fprintf(stderr, "[sgtt picard] step %d: nonlinear residual %.3e, ranks u (%d,%d)\n", i,
                st.nonlinear_residual[i], cur.c[0].r1, cur.c[0].r2);
      if (st.nonlinear_residual[i] <= opts->tol_picard || i >= opts->max_steps) break;
      ++i;
      // lines 4-5: solve for the update and truncate the new iterate (eq. 4.8)
      Vec b;
      b.c[0] = tt_view(S->bu.n1, S->bu.n2, S->bu.n3, S->bu.r1, S->bu.r2, S->bu.c1, S->bu.c2, S->bu.c3);
      b.c[1] = tt_view(S->bp.n1, S->bp.n2, S->bp.n3, S->bp.r1, S->bp.r2, S->bp.c1, S->bp.c2, S->bp.c3);
      Vec d;
      sgtt_solve_stats ls{};
      if (solve_internal(S.get(), b, opts->solve, d, &ls) != SGTT_OK) status = SGTT_W_NOT_CONVERGED;
      if (opts->update_mode == 1) {
        // u^(i) = u^(i-1) + T(du): the update is truncated relative to its
        // own norm and the sum is kept exact, so the iterate carries no
        // rounding error of the size of the Gram-based rounding's floor
        // (about sqrt(machine epsilon) of ||u||)
        Vec dr = opts->eps_soln > 0 ? vec_round(c, d, opts->eps_soln, nullptr, nullptr) : std::move(d);
        cur = vec_concat(c, {&cur, &dr}, nullptr, {});
      } else {
        Vec next = vec_concat(c, {&cur, &d}, nullptr, {});
        cur = opts->eps_soln > 0 ? vec_round(c, next, opts->eps_soln, nullptr, nullptr) : std::move(next);
      }
      record(i, ls, cur);
    }
    S.reset();
    st.steps = i;
    write_pair(c, cur, x);
    c.sync();
    st.seconds = now_s() - t0;
    if (stats) *stats = st;
  } catch (const SgttError& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return SGTT_E_INVALID;
  }
  return status;
}

// ---------------------------------------------------------------- learned mean solve
struct sgtt_mlp {
  sgtt_context* ctx = nullptr;
  std::unique_ptr<Mlp> m;
};

int sgtt_mlp_create(sgtt_context* ctx, int n, int width, long capacity, unsigned seed, sgtt_mlp** out) {
  if (!ctx || !out || n < 1 || width < 1 || capacity < 0) return SGTT_E_INVALID;
  return guarded(ctx, [&]() {
    auto h = std::make_unique<sgtt_mlp>();
    h->ctx = ctx;
    h->m.reset(mlp_create(ctx->c.s, n, width, capacity, seed));
    *out = h.release();
    context_add_child(ctx);
  });
}

int sgtt_mlp_destroy(sgtt_mlp* m) {
  if (!m) return SGTT_OK;
  if (m->m && m->m->uses > 0) {
    // a system still holds the network: detach it first (attach / collect NULL)
    if (m->ctx) m->ctx->err = "network still attached to (or collecting for) a system";
    return SGTT_E_INVALID;
  }
  sgtt_context* ctx = m->ctx;
  if (ctx) (void)hipStreamSynchronize(ctx->c.s);
  delete m;
  if (ctx) context_release_child(ctx);
  return SGTT_OK;
}

int sgtt_mlp_size(const sgtt_mlp* m, long* nparam, long* npairs) {
  if (!m) return SGTT_E_INVALID;
  if (nparam) *nparam = (long)m->m->nparam;
  if (npairs) *npairs = m->m->count;
  return SGTT_OK;
}

int sgtt_mlp_set_params(sgtt_mlp* m, const float* host) {
  if (!m || !host) return SGTT_E_INVALID;
  return guarded(m->ctx, [&]() { mlp_set_params(*m->m, host); });
}

int sgtt_mlp_get_params(sgtt_mlp* m, float* host) {
  if (!m || !host) return SGTT_E_INVALID;
  return guarded(m->ctx, [&]() { mlp_get_params(*m->m, host); });
}

int sgtt_mlp_save(sgtt_mlp* m, const char* path) {
  if (!m || !path) return SGTT_E_INVALID;
  int st = SGTT_OK;
  const int g = guarded(m->ctx, [&]() {
    std::vector<float> p(m->m->nparam);
    mlp_get_params(*m->m, p.data());
    st = net_file_write(path, m->m->n, m->m->w, (long)m->m->nparam, p.data());
    if (st != SGTT_OK) m->ctx->err = std::string("network file: cannot write ") + path;
  });
  return g != SGTT_OK ? g : st;
}

int sgtt_mlp_load(sgtt_mlp* m, const char* path) {
  if (!m || !path) return SGTT_E_INVALID;
  int st = SGTT_OK;
  const int g = guarded(m->ctx, [&]() {
    std::vector<float> p(m->m->nparam);
    st = net_file_read(path, m->m->n, m->m->w, p.data());
    if (st != SGTT_OK) {
      m->ctx->err = std::string("network file: cannot load ") + path;
      return;
    }
    mlp_set_params(*m->m, p.data());
  });
  return g != SGTT_OK ? g : st;
}

int sgtt_mlp_forward(sgtt_mlp* m, const float* x, int batch, float* y) {
  if (!m || !x || !y || batch < 1) return SGTT_E_INVALID;
  return guarded(m->ctx, [&]() { mlp_forward_host(*m->m, x, batch, y, false); });
}

int sgtt_mlp_forward_f16(sgtt_mlp* m, const float* x, int batch, float* y) {
  if (!m || !x || !y || batch < 1) return SGTT_E_INVALID;
  return guarded(m->ctx, [&]() { mlp_forward_host(*m->m, x, batch, y, true); });
}

int sgtt_mlp_loss_grad(sgtt_mlp* m, const float* x, const float* t, int batch, double* loss, float* grad) {
  if (!m || !x || !t || batch < 1) return SGTT_E_INVALID;
  return guarded(m->ctx, [&]() {
    double L = mlp_loss_grad_host(*m->m, x, t, batch, grad);
    if (loss) *loss = L;
  });
}

int sgtt_mlp_train(sgtt_mlp* m, int steps, int batch, double lr, unsigned seed, double* losses) {
  if (!m || steps < 0 || batch < 1 || !(lr > 0)) return SGTT_E_INVALID;
  return guarded(m->ctx, [&]() { mlp_train(*m->m, steps, batch, lr, seed, losses); });
}

int sgtt_mlp_add_pairs(sgtt_mlp* m, const float* x, const float* t, long count, long* added) {
  if (!m || !x || !t || count < 0) return SGTT_E_INVALID;
  return guarded(m->ctx, [&]() {
    long k = mlp_add_pairs(*m->m, x, t, count);
    if (added) *added = k;
  });
}

int sgtt_mlp_collect(sgtt_system* S, sgtt_mlp* m) {
  if (!S) return SGTT_E_INVALID;
  if (m && (m->ctx != S->ctx || m->m->n != S->ns)) {
    S->ctx->err = "network and system do not match (context or spatial size)";
    return SGTT_E_INVALID;
  }
  if (S->mlp_collect) --S->mlp_collect->uses;
  S->mlp_collect = m ? m->m.get() : nullptr;
  if (S->mlp_collect) ++S->mlp_collect->uses;
  return SGTT_OK;
}

int sgtt_mlp_attach(sgtt_system* S, sgtt_mlp* m) {
  if (!S) return SGTT_E_INVALID;
  if (m && (m->ctx != S->ctx || m->m->n != S->ns)) {
    S->ctx->err = "network and system do not match (context or spatial size)";
    return SGTT_E_INVALID;
  }
  if (S->mlp_apply) --S->mlp_apply->uses;
  S->mlp_apply = m ? m->m.get() : nullptr;
  if (S->mlp_apply) ++S->mlp_apply->uses;
  return SGTT_OK;
}

int sgtt_profile_enable(sgtt_context* ctx, int enable) {
  if (!ctx) return SGTT_E_INVALID;
  (void)hipStreamSynchronize(ctx->c.s);
  prof_reset();
  prof_enable(enable != 0);
  return SGTT_OK;
}

int sgtt_profile_enable_classes(sgtt_context* ctx, unsigned class_mask) {
  if (!ctx) return SGTT_E_INVALID;
  (void)hipStreamSynchronize(ctx->c.s);
  prof_reset();
  prof_enable_mask(class_mask);
  return SGTT_OK;
}

int sgtt_profile_sample(sgtt_context* ctx, int period) {
  if (!ctx || period < 1) return SGTT_E_INVALID;
  (void)hipStreamSynchronize(ctx->c.s);
  prof_sample_period(period);
  return SGTT_OK;
}

int sgtt_profile_read(sgtt_context* ctx, int max_classes, double* seconds, double* bytes, double* flops,
                      long* launches, int* nclasses) {
  if (!ctx || !seconds || !bytes || !flops || !launches) return SGTT_E_INVALID;
  (void)hipStreamSynchronize(ctx->c.s);
  double s[KC_COUNT], b[KC_COUNT], f[KC_COUNT];
  long l[KC_COUNT];
  prof_read(s, b, f, l);
  int n = std::min(max_classes, (int)KC_COUNT);
  for (int i = 0; i < n; ++i) {
    seconds[i] = s[i];
    bytes[i] = b[i];
    flops[i] = f[i];
    launches[i] = l[i];
  }
  if (nclasses) *nclasses = KC_COUNT;
  return SGTT_OK;
}

const char* sgtt_profile_class_name(int cls) { return kernel_class_name(cls); }

int sgtt_profile_read_regions(sgtt_context* ctx, int max_regions, int max_classes, double* seconds, int* nregions) {
  if (!ctx || !seconds || max_regions < 0 || max_classes < 0) return SGTT_E_INVALID;
  (void)hipStreamSynchronize(ctx->c.s);
  std::vector<double> all((size_t)RG_COUNT * KC_COUNT);
  prof_read_regions(all.data());
  for (int r = 0; r < std::min(max_regions, (int)RG_COUNT); ++r)
    for (int k = 0; k < std::min(max_classes, (int)KC_COUNT); ++k)
      seconds[(size_t)r * max_classes + k] = all[(size_t)r * KC_COUNT + k];
  if (nregions) *nregions = RG_COUNT;
  return SGTT_OK;
}

const char* sgtt_profile_region_name(int region) { return region_name(region); }

// ---------------------------------------------------------------- host-only
struct sgtt_host_problem {
  HostProblem hp;
};

int sgtt_host_problem_create(const sgtt_problem_desc* desc, sgtt_host_problem** out) {
  if (!desc || !out) return SGTT_E_INVALID;
  try {
    auto h = std::make_unique<sgtt_host_problem>();
    ProblemParams prm;
    prm.h = desc->h;
    prm.L = desc->L;
    prm.m = desc->m;
    prm.p = desc->p;
    prm.nt = desc->nt;
    prm.tau = desc->tau;
    prm.nu0 = desc->nu0;
    prm.nu_coef = desc->nu_coef;
    prm.ramp = desc->ramp;
    prm.visc_law = desc->viscosity_law;
    prm.corr_length = desc->corr_length;
    build_problem(prm, h->hp);
    *out = h.release();
  } catch (...) {
    return SGTT_E_SETUP;
  }
  return SGTT_OK;
}

int sgtt_host_problem_destroy(sgtt_host_problem* h) {
  delete h;
  return SGTT_OK;
}

int sgtt_host_sizes(const sgtt_host_problem* h, int* sizes) {
  if (!h || !sizes) return SGTT_E_INVALID;
  sizes[0] = h->hp.n_s;
  sizes[1] = h->hp.n_u;
  sizes[2] = h->hp.n_p;
  sizes[3] = h->hp.n_xi;
  sizes[4] = h->hp.nt;
  sizes[5] = h->hp.n_all;
  return SGTT_OK;
}

int sgtt_host_csr(const sgtt_host_problem* h, int which, int* nrows, int* ncols, int* nnz, int* rowptr, int* col,
                  double* val) {
  if (!h) return SGTT_E_INVALID;
  const HostProblem& hp = h->hp;
  const Csr* pat = nullptr;
  const double* v = nullptr;
  switch (which) {
    case 0: pat = &hp.Kff; v = hp.Mff.data(); break;
    case 1: pat = &hp.Kff; v = hp.Aff.data(); break;
    case 2: pat = &hp.B; v = hp.B.val.data(); break;
    case 3: pat = &hp.Xp; v = hp.Xp.val.data(); break;
    case 4: pat = &hp.Xmid; v = hp.XM.data(); break;
    case 5: pat = &hp.Xmid; v = hp.XA.data(); break;
    case 6: pat = &hp.Qp; v = hp.Mp.data(); break;
    case 7: pat = &hp.Qp; v = hp.Ap.data(); break;
    default:
      if (which >= 8 && which < 8 + hp.nvisc) {
        pat = &hp.Kff;
        v = hp.Aff_visc[which - 8].data();
        break;
      }
      return SGTT_E_INVALID;
  }
  if (nrows) *nrows = pat->nrows;
  if (ncols) *ncols = pat->ncols;
  if (nnz) *nnz = pat->nnz();
  if (rowptr) std::copy(pat->rowptr.begin(), pat->rowptr.end(), rowptr);
  if (col) std::copy(pat->col.begin(), pat->col.end(), col);
  if (val) std::copy(v, v + pat->nnz(), val);
  return SGTT_OK;
}

int sgtt_host_kl(const sgtt_host_problem* h, int* nmodes, int* nvisc, double* beta, double* modes) {
  if (!h) return SGTT_E_INVALID;
  const HostProblem& hp = h->hp;
  const int m = (int)hp.kl_beta.size();
  if (nmodes) *nmodes = m;
  if (nvisc) *nvisc = hp.nvisc;
  if (beta) std::copy(hp.kl_beta.begin(), hp.kl_beta.end(), beta);
  if (modes) std::copy(hp.kl_modes.begin(), hp.kl_modes.end(), modes);
  return SGTT_OK;
}

int sgtt_host_bcr_solve(const sgtt_host_problem* h, int which, double tau, double nu, int ncols, const double* b,
                        double* x, int* npass) {
  if (!h || !b || !x || ncols <= 0 || (which != 0 && which != 1) || (which == 0 && !(tau > 0.0)))
    return SGTT_E_INVALID;
  try {
    const HostProblem& hp = h->hp;
    BcrFactor f;
    std::string err;
    if (which == 0) {
      std::vector<double> F(hp.Kff.nnz());
      for (int t = 0; t < hp.Kff.nnz(); ++t) F[t] = hp.Mff[t] / tau + nu * hp.Aff[t];
      bcr_factor(hp.Kff, F.data(), hp.vel_blocks, f, err);
    } else {
      bcr_factor(hp.Xp, hp.Xp.val.data(), hp.p_blocks, f, err);
    }
    if (!err.empty()) return -6;
    bcr_apply_host(f, ncols, b, x);
    if (npass) *npass = (int)f.pass_begin.size() - 1;
    return SGTT_OK;
  } catch (...) {
    return -6;
  }
}

int sgtt_host_gpc(const sgtt_host_problem* h, int which, double* out) {
  if (!h || !out) return SGTT_E_INVALID;
  const HostProblem& hp = h->hp;
  const std::vector<double>* src = which == 0 ? &hp.G : which == 1 ? &hp.H : which == 2 ? &hp.Gnu
                                  : which == 3 ? &hp.Gvisc : nullptr;
  if (!src) return SGTT_E_INVALID;
  std::copy(src->begin(), src->end(), out);
  return SGTT_OK;
}

int sgtt_host_mesh(const sgtt_host_problem* h, double* coords, int* free_nodes, double* g_all) {
  if (!h) return SGTT_E_INVALID;
  const HostProblem& hp = h->hp;
  const double s = hp.prm.h / 2.0;
  if (coords)
    for (int i = 0; i < hp.n_all; ++i) {
      coords[2 * i] = hp.mesh.I[i] * s;
      coords[2 * i + 1] = hp.mesh.J[i] * s;
    }
  if (free_nodes) std::copy(hp.mesh.free_nodes.begin(), hp.mesh.free_nodes.end(), free_nodes);
  if (g_all) std::copy(hp.g_all.begin(), hp.g_all.end(), g_all);
  return SGTT_OK;
}

}  // extern "C"
