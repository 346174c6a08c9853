// Host-side self-check for sanitizer builds (AddressSanitizer and
// UndefinedBehaviorSanitizer): runs the plain-C++ parts of the library on a
// small problem and checks their results against invariants, so that a
// sanitizer run covers problem assembly, the KL expansion (sec. 6.1), the
// block cyclic reduction factor and its host application, convection
// values (eq. 3.7) and checkpoint files.  Not part of the library build.
//
//   g++ -std=c++17 -fsanitize=address,undefined -I include -I <csrc> \
//       host_check.cpp host_setup.cpp checkpoint.cpp -o host_check
//   ./host_check <scratch directory>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "checkpoint.h"
#include "host_setup.h"
#include "sgtt.h"

using namespace sgtt;

namespace {

int failures = 0;
void check(bool ok, const char* what) {
  std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) ++failures;
}

// y = A x for a scalar CSR pattern with the given values
void csr_mv(const Csr& K, const double* vals, const double* x, double* y) {
  for (int r = 0; r < K.nrows; ++r) {
    double s = 0.0;
    for (int t = K.rowptr[r]; t < K.rowptr[r + 1]; ++t) s += vals[t] * x[K.col[t]];
    y[r] = s;
  }
}

}  // namespace

int main(int argc, char** argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  // the Table 6.1 mesh size with the KL law, few time steps
  ProblemParams prm;
  prm.h = 0.25;
  prm.m = 3;
  prm.p = 2;
  prm.nt = 4;
  prm.tau = 1.0 / 64;
  prm.nu_coef = 0.01;
  prm.visc_law = 1;
  HostProblem hp;
  build_problem(prm, hp);
  check(hp.n_s > 0 && hp.n_u == 2 * hp.n_s && hp.n_p > 0, "problem sizes");
  check(hp.nvisc == prm.m + 1 && (int)hp.Aff_visc.size() == hp.nvisc, "one stiffness per KL term plus the mean");
  // KL modes: descending eigenvalues, M_p-orthonormal modes
  bool desc = true;
  for (size_t l = 1; l < hp.kl_beta.size(); ++l) desc = desc && hp.kl_beta[l] <= hp.kl_beta[l - 1];
  check(desc && hp.kl_beta.size() == (size_t)prm.m, "KL eigenvalues descending");
  double orth = 0.0;
  std::vector<double> t(hp.n_p);
  for (int a = 0; a < prm.m; ++a) {
    csr_mv(hp.Qp, hp.Mp.data(), &hp.kl_modes[(size_t)a * hp.n_p], t.data());
    for (int b = 0; b < prm.m; ++b) {
      double s = 0.0;
      for (int i = 0; i < hp.n_p; ++i) s += hp.kl_modes[(size_t)b * hp.n_p + i] * t[i];
      orth = std::fmax(orth, std::fabs(s - (a == b ? 1.0 : 0.0)));
    }
  }
  check(orth < 1e-10, "KL modes M_p-orthonormal");
  // mass times the constant vector sums to the free nodes' share of the area
  std::vector<double> one(hp.n_s, 1.0), m1(hp.n_s);
  csr_mv(hp.Kff, hp.Mff.data(), one.data(), m1.data());
  double area = 0.0;
  for (double v : m1) area += v;
  check(area > 0.0 && area < 2.0 * (hp.prm.L + 1.0), "mass matrix row sums");
  // block cyclic reduction of F = M / tau + nu0 A against its own product
  std::vector<double> F(hp.Mff.size());
  for (size_t i = 0; i < F.size(); ++i) F[i] = hp.Mff[i] / prm.tau + prm.nu0 * hp.Aff[i];
  BcrFactor f;
  std::string err;
  bcr_factor(hp.Kff, F.data(), hp.vel_blocks, f, err);
  check(err.empty(), "block cyclic reduction factor");
  const int ncols = 3;
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  std::vector<double> x((size_t)hp.n_s * ncols), b((size_t)hp.n_s * ncols), y((size_t)hp.n_s * ncols);
  for (double& v : x) v = nd(rng);
  for (int c = 0; c < ncols; ++c)
    for (int r = 0; r < hp.n_s; ++r) {
      double s = 0.0;
      for (int q = hp.Kff.rowptr[r]; q < hp.Kff.rowptr[r + 1]; ++q) s += F[q] * x[(size_t)hp.Kff.col[q] * ncols + c];
      b[(size_t)r * ncols + c] = s;
    }
  bcr_apply_host(f, ncols, b.data(), y.data());
  double e = 0.0, n = 0.0;
  for (size_t i = 0; i < x.size(); ++i) {
    e += (y[i] - x[i]) * (y[i] - x[i]);
    n += x[i] * x[i];
  }
  check(std::sqrt(e / n) < 1e-10, "block cyclic reduction solves F x = b");
  // convection of a constant wind: N 1 = 0 on interior rows (eq. 3.7)
  std::vector<double> w1(hp.n_all, 1.0), w2(hp.n_all, 0.0), nv(hp.Kff.nnz()), nfa(hp.Kfa.nnz());
  convection_values(hp, w1.data(), w2.data(), nv.data(), nfa.data());
  std::vector<double> ones_all(hp.n_all, 1.0), r(hp.n_s);
  csr_mv(hp.Kfa, nfa.data(), ones_all.data(), r.data());
  double rmax = 0.0;
  for (double v : r) rmax = std::fmax(rmax, std::fabs(v));
  check(rmax < 1e-12, "convection of a constant field vanishes");
  // checkpoint round trip and a damaged file
  int dims[10] = {4, 6, 9, 2, 3, 4, 6, 5, 1, 2};
  std::vector<double> cores[6];
  const double* cp[6];
  double* rp[6];
  std::vector<double> back[6];
  for (int q = 0; q < 2; ++q) {
    const int* d = dims + 5 * q;
    const long len[3] = {(long)d[0] * d[3], (long)d[3] * d[1] * d[4], (long)d[2] * d[4]};
    for (int w = 0; w < 3; ++w) {
      cores[3 * q + w].resize(len[w]);
      for (double& v : cores[3 * q + w]) v = nd(rng);
      back[3 * q + w].assign(len[w], 0.0);
      cp[3 * q + w] = cores[3 * q + w].data();
      rp[3 * q + w] = back[3 * q + w].data();
    }
  }
  const std::string path = dir + "/host_check.sgtt";
  check(pair_file_write(path.c_str(), dims, cp) == SGTT_OK, "checkpoint written");
  int got[10];
  check(pair_file_read(path.c_str(), dims, rp, got) == SGTT_OK, "checkpoint read");
  bool same = true;
  for (int i = 0; i < 6; ++i) same = same && back[i] == cores[i];
  check(same, "checkpoint round trip bit-exact");
  {
    FILE* fp = std::fopen(path.c_str(), "r+b");
    std::fseek(fp, 100, SEEK_SET);
    int ch = std::fgetc(fp);
    std::fseek(fp, 100, SEEK_SET);
    std::fputc(ch ^ 1, fp);
    std::fclose(fp);
  }
  check(pair_file_read(path.c_str(), dims, rp, got) == SGTT_E_IO, "damaged checkpoint refused");
  std::remove(path.c_str());
  // network parameter files
  {
    const int n = 37, w = 5;
    const long np = (long)w * n + w + w * w + w + (long)n * w + n;
    std::vector<float> par(np), bk(np, 0.f);
    for (float& v : par) v = (float)nd(rng);
    const std::string npath = dir + "/host_check.sgmlp";
    check(net_file_write(npath.c_str(), n, w, np, par.data()) == SGTT_OK, "network file written");
    int fn = 0, fw = 0;
    long fp = 0;
    check(net_file_info(npath.c_str(), &fn, &fw, &fp) == SGTT_OK && fn == n && fw == w && fp == np,
          "network file header");
    check(net_file_read(npath.c_str(), n, w, bk.data()) == SGTT_OK && bk == par, "network round trip bit-exact");
    check(net_file_read(npath.c_str(), n + 1, w, bk.data()) == SGTT_E_INVALID, "network of another shape refused");
    check(net_file_write(npath.c_str(), n, w, np + 1, par.data()) == SGTT_E_INVALID, "inconsistent count refused");
    std::remove(npath.c_str());
  }
  std::printf("%d failures\n", failures);
  return failures ? 1 : 0;
}
