// Host-side setup: step mesh, Q2-Q1 assembly, chaos matrices, LSC pressure
// matrices and block-tridiagonal factorizations.  See host_setup.h.
#include "host_setup.h"

#include <algorithm>
#include <climits>
#include <functional>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <tuple>
#include <atomic>
#include <thread>
#include <vector>

namespace sgtt {

namespace {

inline int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// ---------------------------------------------------------------- reference element
struct RefTables {
  double w[9];          // Gauss weights (tensor 3x3)
  double phi[9][9];     // [g][k]  Q2, k = a + 3 b
  double dxi[9][9];     // d/dxi
  double deta[9][9];    // d/deta
  double psi[9][4];     // Q1, k = a + 2 b
  double pdxi[9][4];    // Q1 d/dxi
  double pdeta[9][4];   // Q1 d/deta
};

RefTables make_ref() {
  RefTables t;
  const double gp[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)};
  const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
  auto q2 = [](double x, int a) {
    return a == 0 ? 0.5 * x * (x - 1) : (a == 1 ? 1 - x * x : 0.5 * x * (x + 1));
  };
  auto dq2 = [](double x, int a) { return a == 0 ? x - 0.5 : (a == 1 ? -2 * x : x + 0.5); };
  auto q1 = [](double x, int a) { return a == 0 ? 0.5 * (1 - x) : 0.5 * (1 + x); };
  for (int jb = 0; jb < 3; ++jb)
    for (int ia = 0; ia < 3; ++ia) {
      int g = ia + 3 * jb;
      double xi = gp[ia], eta = gp[jb];
      t.w[g] = gw[ia] * gw[jb];
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
          int k = a + 3 * b;
          t.phi[g][k] = q2(xi, a) * q2(eta, b);
          t.dxi[g][k] = dq2(xi, a) * q2(eta, b);
          t.deta[g][k] = q2(xi, a) * dq2(eta, b);
        }
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          t.psi[g][a + 2 * b] = q1(xi, a) * q1(eta, b);
          t.pdxi[g][a + 2 * b] = (a == 0 ? -0.5 : 0.5) * q1(eta, b);
          t.pdeta[g][a + 2 * b] = q1(xi, a) * (b == 0 ? -0.5 : 0.5);
        }
    }
  return t;
}

const RefTables& ref() {
  static RefTables t = make_ref();
  return t;
}

// ---------------------------------------------------------------- CSR helpers
void finalize_pattern(std::vector<std::vector<int>>& rows, int ncols, Csr& c) {
  c.nrows = (int)rows.size();
  c.ncols = ncols;
  c.rowptr.assign(c.nrows + 1, 0);
  for (int i = 0; i < c.nrows; ++i) {
    auto& r = rows[i];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    c.rowptr[i + 1] = c.rowptr[i] + (int)r.size();
  }
  c.col.resize(c.rowptr[c.nrows]);
  for (int i = 0; i < c.nrows; ++i)
    std::copy(rows[i].begin(), rows[i].end(), c.col.begin() + c.rowptr[i]);
  c.val.assign(c.col.size(), 0.0);
}

inline int find_pos(const Csr& c, int i, int j) {
  auto b = c.col.begin() + c.rowptr[i], e = c.col.begin() + c.rowptr[i + 1];
  auto it = std::lower_bound(b, e, j);
  if (it == e || *it != j) throw std::runtime_error("pattern miss");
  return (int)(it - c.col.begin());
}

// ---------------------------------------------------------------- mesh
void build_mesh(double h, double L, Mesh& m) {
  m.h = h;
  m.L = L;
  int q = (int)std::lround(1.0 / h);
  if (std::fabs(q * h - 1.0) > 1e-12 || q % 2) throw std::runtime_error("1/h must be an even integer");
  m.q = q;
  int nL = (int)std::lround(q * L);
  std::vector<std::pair<int, int>> elems;
  for (int ec = -q; ec < 0; ++ec)
    for (int er = -q / 2; er < q / 2; ++er) elems.push_back({ec, er});
  for (int ec = 0; ec < nL; ++ec)
    for (int er = -q; er < q; ++er) elems.push_back({ec, er});
  // dense lattice index maps
  int I0 = -2 * q, I1 = 2 * nL, J0 = -2 * q, J1 = 2 * q;
  int NI = I1 - I0 + 1, NJ = J1 - J0 + 1;
  std::vector<int> vmark((size_t)NI * NJ, -1), pmark((size_t)NI * NJ, -1);
  for (auto& e : elems)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        int I = 2 * e.first + a, J = 2 * e.second + b;
        vmark[(size_t)(I - I0) * NJ + (J - J0)] = 1;
        if (a % 2 == 0 && b % 2 == 0) pmark[(size_t)(I - I0) * NJ + (J - J0)] = 1;
      }
  // sorted by (I, J) lexicographically == scan I outer, J inner
  for (int I = I0; I <= I1; ++I)
    for (int J = J0; J <= J1; ++J) {
      size_t k = (size_t)(I - I0) * NJ + (J - J0);
      if (vmark[k] >= 0) {
        vmark[k] = (int)m.I.size();
        m.I.push_back(I);
        m.J.push_back(J);
      }
      if (pmark[k] >= 0) {
        pmark[k] = (int)m.pI.size();
        m.pI.push_back(I);
        m.pJ.push_back(J);
      }
    }
  for (auto& e : elems) {
    std::array<int, 9> c;
    std::array<int, 4> pc;
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a)
        c[a + 3 * b] = vmark[(size_t)(2 * e.first + a - I0) * NJ + (2 * e.second + b - J0)];
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        pc[a + 2 * b] = pmark[(size_t)(2 * e.first + 2 * a - I0) * NJ + (2 * e.second + 2 * b - J0)];
    m.conn.push_back(c);
    m.pconn.push_back(pc);
  }
  int n = m.n_all();
  m.free_id.assign(n, -1);
  m.dir_id.assign(n, -1);
  m.g1.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    int I = m.I[k], J = m.J[k];
    bool inflow = (I == -2 * q);
    bool inlet_wall = (std::abs(J) == q) && (I <= 0);
    bool channel_wall = (std::abs(J) == 2 * q);
    bool step_face = (I == 0) && (std::abs(J) >= q);
    if (inflow || inlet_wall || channel_wall || step_face) {
      m.dir_id[k] = (int)m.dir_nodes.size();
      m.dir_nodes.push_back(k);
      if (inflow) {
        double x2 = J * h / 2.0;
        m.g1[k] = 1.0 - 4.0 * x2 * x2;
      }
    } else {
      m.free_id[k] = (int)m.free_nodes.size();
      m.free_nodes.push_back(k);
    }
  }
}

// ---------------------------------------------------------------- chaos
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pnm1 = (n == 1) ? 1.0 : p0;
      double dp = n * (z * pn - pnm1) / (z * z - 1);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? z : p1, pnm1 = (n == 1) ? 1.0 : p0;
    double dp = n * (z * pn - pnm1) / (z * z - 1);
    x[i] = z;
    w[i] = 2.0 / ((1 - z * z) * dp * dp);
  }
}

// orthonormal Legendre sqrt(2n+1) P_n at x, n = 0..p
void psi_all(int p, double x, double* out) {
  double p0 = 1, p1 = x;
  out[0] = 1.0;
  if (p >= 1) out[1] = std::sqrt(3.0) * x;
  for (int k = 2; k <= p; ++k) {
    double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
    out[k] = std::sqrt(2.0 * k + 1) * p2;
  }
}

void build_gpc(int m, int p, HostProblem& hp) {
  // multi-indices: graded, descending lexicographic within each degree
  std::vector<std::vector<int>> all;
  for (int deg = 0; deg <= p; ++deg) {
    std::vector<std::vector<int>> lev;
    std::vector<int> a(m, 0);
    // enumerate all tuples with entries in [0, deg] and sum == deg
    std::function<void(int, int)> rec = [&](int pos, int rem) {
      if (pos == m - 1) {
        a[pos] = rem;
        lev.push_back(a);
        return;
      }
      for (int v = rem; v >= 0; --v) {
        a[pos] = v;
        rec(pos + 1, rem - v);
      }
    };
    rec(0, deg);
    std::sort(lev.begin(), lev.end(), std::greater<std::vector<int>>());
    for (auto& t : lev) all.push_back(t);
  }
  hp.midx = all;
  int n = (int)all.size();
  hp.n_xi = n;
  // 1-D tables by Gauss-Legendre quadrature (expectation = integral / 2)
  int npts = (3 * p + 2) / 2 + 2;
  std::vector<double> gx, gw;
  gauss_legendre(npts, gx, gw);
  std::vector<double> P((size_t)npts * (p + 1));
  for (int g = 0; g < npts; ++g) psi_all(p, gx[g], &P[(size_t)g * (p + 1)]);
  auto T3 = [&](int a, int b, int c) {
    double s = 0;
    for (int g = 0; g < npts; ++g)
      s += 0.5 * gw[g] * P[g * (p + 1) + a] * P[g * (p + 1) + b] * P[g * (p + 1) + c];
    return s;
  };
  auto X2 = [&](int a, int b) {
    double s = 0;
    for (int g = 0; g < npts; ++g) s += 0.5 * gw[g] * gx[g] * P[g * (p + 1) + a] * P[g * (p + 1) + b];
    return s;
  };
  hp.G.assign((size_t)(m + 1) * n * n, 0.0);
  for (int r = 0; r < n; ++r) hp.G[(size_t)r * n + r] = 1.0;
  for (int l = 0; l < m; ++l)
    for (int r = 0; r < n; ++r)
      for (int s = 0; s < n; ++s) {
        bool same = true;
        for (int k = 0; k < m; ++k)
          if (k != l && all[r][k] != all[s][k]) same = false;
        if (same) hp.G[((size_t)(l + 1) * n + r) * n + s] = X2(all[r][l], all[s][l]);
      }
  hp.H.assign((size_t)n * n * n, 0.0);
  for (int l = 0; l < n; ++l)
    for (int r = 0; r < n; ++r)
      for (int s = 0; s < n; ++s) {
        double v = 1.0;
        for (int k = 0; k < m; ++k) v *= T3(all[l][k], all[r][k], all[s][k]);
        hp.H[((size_t)l * n + r) * n + s] = v;
      }
}

}  // namespace

// ---------------------------------------------------------------- problem
void build_problem(const ProblemParams& prm, HostProblem& hp) {
  hp.prm = prm;
  Mesh& m = hp.mesh;
  build_mesh(prm.h, prm.L, m);
  const int ns = m.n_s(), na = m.n_all(), np = m.n_p();
  hp.n_s = ns;
  hp.n_u = 2 * ns;
  hp.n_p = np;
  hp.n_all = na;
  hp.nt = prm.nt;
  const RefTables& R = ref();
  const double h = prm.h, jac = 0.25 * h * h;
  // element matrices (identical on every square)
  double Me[9][9], Ae[9][9], B1e[4][9], B2e[4][9];
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      double sm = 0, sa = 0;
      for (int g = 0; g < 9; ++g) {
        sm += R.w[g] * R.phi[g][i] * R.phi[g][j];
        sa += R.w[g] * (R.dxi[g][i] * R.dxi[g][j] + R.deta[g][i] * R.deta[g][j]);
      }
      Me[i][j] = sm * jac;
      Ae[i][j] = sa;          // (2/h)^2 * jac = 1
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 9; ++j) {
      double s1 = 0, s2 = 0;
      for (int g = 0; g < 9; ++g) {
        s1 += R.w[g] * R.psi[g][i] * R.dxi[g][j];
        s2 += R.w[g] * R.psi[g][i] * R.deta[g][j];
      }
      B1e[i][j] = -s1 * jac * (2.0 / h);
      B2e[i][j] = -s2 * jac * (2.0 / h);
    }
  // patterns
  std::vector<std::vector<int>> rff(ns), rfa(ns), rb(np), rball(np);
  for (size_t e = 0; e < m.conn.size(); ++e) {
    const auto& c = m.conn[e];
    for (int i = 0; i < 9; ++i) {
      int fi = m.free_id[c[i]];
      if (fi < 0) continue;
      for (int j = 0; j < 9; ++j) {
        rfa[fi].push_back(c[j]);
        int fj = m.free_id[c[j]];
        if (fj >= 0) rff[fi].push_back(fj);
      }
    }
    for (int i = 0; i < 4; ++i) {
      int k = m.pconn[e][i];
      for (int j = 0; j < 9; ++j) {
        rball[k].push_back(c[j]);
        rball[k].push_back(na + c[j]);
        int fj = m.free_id[c[j]];
        if (fj >= 0) {
          rb[k].push_back(fj);
          rb[k].push_back(ns + fj);
        }
      }
    }
  }
  finalize_pattern(rff, ns, hp.Kff);
  finalize_pattern(rfa, na, hp.Kfa);
  finalize_pattern(rb, 2 * ns, hp.B);
  finalize_pattern(rball, 2 * na, hp.Ball);
  hp.Mff.assign(hp.Kff.nnz(), 0.0);
  hp.Aff.assign(hp.Kff.nnz(), 0.0);
  hp.Mfa.assign(hp.Kfa.nnz(), 0.0);
  hp.Afa.assign(hp.Kfa.nnz(), 0.0);
  for (size_t e = 0; e < m.conn.size(); ++e) {
    const auto& c = m.conn[e];
    for (int i = 0; i < 9; ++i) {
      int fi = m.free_id[c[i]];
      if (fi < 0) continue;
      for (int j = 0; j < 9; ++j) {
        int pa = find_pos(hp.Kfa, fi, c[j]);
        hp.Mfa[pa] += Me[i][j];
        hp.Afa[pa] += Ae[i][j];
        int fj = m.free_id[c[j]];
        if (fj >= 0) {
          int pf = find_pos(hp.Kff, fi, fj);
          hp.Mff[pf] += Me[i][j];
          hp.Aff[pf] += Ae[i][j];
        }
      }
    }
    for (int i = 0; i < 4; ++i) {
      int k = m.pconn[e][i];
      for (int j = 0; j < 9; ++j) {
        hp.Ball.val[find_pos(hp.Ball, k, c[j])] += B1e[i][j];
        hp.Ball.val[find_pos(hp.Ball, k, na + c[j])] += B2e[i][j];
        int fj = m.free_id[c[j]];
        if (fj >= 0) {
          hp.B.val[find_pos(hp.B, k, fj)] += B1e[i][j];
          hp.B.val[find_pos(hp.B, k, ns + fj)] += B2e[i][j];
        }
      }
    }
  }
  // B^T (n_u x n_p)
  {
    std::vector<std::vector<int>> rt(2 * ns);
    for (int k = 0; k < np; ++k)
      for (int t = hp.B.rowptr[k]; t < hp.B.rowptr[k + 1]; ++t) rt[hp.B.col[t]].push_back(k);
    finalize_pattern(rt, np, hp.Bt);
    for (int k = 0; k < np; ++k)
      for (int t = hp.B.rowptr[k]; t < hp.B.rowptr[k + 1]; ++t)
        hp.Bt.val[find_pos(hp.Bt, hp.B.col[t], k)] = hp.B.val[t];
  }
  // chaos and viscosity
  build_gpc(prm.m, prm.p, hp);
  const int nx = hp.n_xi;
  hp.visc.assign(prm.m + 1, 0.0);
  hp.visc[0] = prm.nu0;
  for (int k = 1; k <= prm.m; ++k) hp.visc[k] = prm.nu_coef * prm.nu0 / ((double)k * k);
  hp.Gnu.assign((size_t)nx * nx, 0.0);
  for (int l = 0; l <= prm.m; ++l)
    for (int i = 0; i < nx * nx; ++i) hp.Gnu[i] += hp.visc[l] * hp.G[(size_t)l * nx * nx + i];
  // time ramp
  hp.ramp.resize(prm.nt);
  for (int k = 0; k < prm.nt; ++k) hp.ramp[k] = 1.0 - std::exp(-prm.ramp * prm.tau * (k + 1));
  // Dirichlet lift
  hp.g_all.assign(2 * na, 0.0);
  for (int k = 0; k < na; ++k)
    if (m.dir_id[k] >= 0) hp.g_all[k] = m.g1[k];
  // M_* = diag(M)
  hp.Mstar.assign(ns, 0.0);
  for (int i = 0; i < ns; ++i) hp.Mstar[i] = hp.Mff[find_pos(hp.Kff, i, i)];
  // X = B M*^-1 B^T pattern/values, and the LSC middle pattern
  {
    std::vector<std::vector<int>> rx(np), rmid(np);
    std::vector<int> mark(np, -1), mark2(np, -1);
    for (int k = 0; k < np; ++k) {
      for (int t = hp.B.rowptr[k]; t < hp.B.rowptr[k + 1]; ++t) {
        int cj = hp.B.col[t];
        for (int u = hp.Bt.rowptr[cj]; u < hp.Bt.rowptr[cj + 1]; ++u) {
          int k2 = hp.Bt.col[u];
          if (mark[k2] != k) { mark[k2] = k; rx[k].push_back(k2); }
        }
        int c = cj / ns, j = cj % ns;
        for (int s = hp.Kff.rowptr[j]; s < hp.Kff.rowptr[j + 1]; ++s) {
          int l = hp.Kff.col[s];
          int cl = c * ns + l;
          for (int u = hp.Bt.rowptr[cl]; u < hp.Bt.rowptr[cl + 1]; ++u) {
            int k2 = hp.Bt.col[u];
            if (mark2[k2] != k) { mark2[k2] = k; rmid[k].push_back(k2); }
          }
        }
      }
    }
    finalize_pattern(rx, np, hp.Xp);
    finalize_pattern(rmid, np, hp.Xmid);
    std::vector<double> acc(np, 0.0);
    for (int k = 0; k < np; ++k) {
      for (int t = hp.B.rowptr[k]; t < hp.B.rowptr[k + 1]; ++t) {
        int cj = hp.B.col[t];
        double w = hp.B.val[t] / hp.Mstar[cj % ns];
        for (int u = hp.Bt.rowptr[cj]; u < hp.Bt.rowptr[cj + 1]; ++u) acc[hp.Bt.col[u]] += w * hp.Bt.val[u];
      }
      for (int t = hp.Xp.rowptr[k]; t < hp.Xp.rowptr[k + 1]; ++t) {
        hp.Xp.val[t] = acc[hp.Xp.col[t]];
        acc[hp.Xp.col[t]] = 0.0;
      }
    }
    hp.XM.assign(hp.Xmid.nnz(), 0.0);
    hp.XA.assign(hp.Xmid.nnz(), 0.0);
    lsc_middle_values(hp, hp.Mff.data(), hp.XM.data());
    lsc_middle_values(hp, hp.Aff.data(), hp.XA.data());
  }
  // Q1 pressure-space matrices of the PCD approximation (sec. 5.1, eq. 5.17):
  // mass M_p and unit-viscosity stiffness A_p on the Q1 pattern, no boundary
  // condition imposed
  {
    std::vector<std::vector<int>> rq(np);
    for (size_t e = 0; e < m.pconn.size(); ++e)
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) rq[m.pconn[e][i]].push_back(m.pconn[e][j]);
    finalize_pattern(rq, np, hp.Qp);
    double Mpe[4][4], Ape[4][4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double sm = 0, sa = 0;
        for (int g = 0; g < 9; ++g) {
          sm += R.w[g] * R.psi[g][i] * R.psi[g][j];
          sa += R.w[g] * (R.pdxi[g][i] * R.pdxi[g][j] + R.pdeta[g][i] * R.pdeta[g][j]);
        }
        Mpe[i][j] = sm * jac;
        Ape[i][j] = sa;   // (2/h)^2 * jac = 1
      }
    hp.Mp.assign(hp.Qp.nnz(), 0.0);
    hp.Ap.assign(hp.Qp.nnz(), 0.0);
    for (size_t e = 0; e < m.pconn.size(); ++e)
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          const int t = find_pos(hp.Qp, m.pconn[e][i], m.pconn[e][j]);
          hp.Mp[t] += Mpe[i][j];
          hp.Ap[t] += Ape[i][j];
        }
    hp.Mpstar.assign(np, 0.0);
    for (int k = 0; k < np; ++k) hp.Mpstar[k] = hp.Mp[find_pos(hp.Qp, k, k)];
  }
  // viscous terms (eq. 3.6): one for the law nu0 (1 + sigma sum xi_k/k^2),
  // m + 1 for the KL law (sec. 6.1)
  {
    const int nx = hp.n_xi, nnz = hp.Kff.nnz(), nnzfa = hp.Kfa.nnz();
    hp.Aff_visc.assign(1, hp.Aff);
    hp.Afa_visc.assign(1, hp.Afa);
    if (prm.visc_law == 1) {
      kl_expansion(hp, prm.corr_length, prm.m, hp.kl_beta, hp.kl_modes);
      hp.nvisc = prm.m + 1;
      hp.Gvisc.assign((size_t)hp.nvisc * nx * nx, 0.0);
      for (int i = 0; i < nx; ++i) hp.Gvisc[(size_t)i * nx + i] = prm.nu0;
      for (int l = 1; l <= prm.m; ++l) {
        for (int i = 0; i < nx * nx; ++i)
          hp.Gvisc[(size_t)l * nx * nx + i] = std::sqrt(3.0) * hp.G[(size_t)l * nx * nx + i];
        std::vector<double> vff(nnz), vfa(nnzfa);
        weighted_stiffness_values(hp, &hp.kl_modes[(size_t)(l - 1) * np], vff.data(), vfa.data());
        const double cl = prm.nu0 * prm.nu_coef * std::sqrt(hp.kl_beta[l - 1]);
        for (auto& v : vff) v *= cl;
        for (auto& v : vfa) v *= cl;
        hp.Aff_visc.push_back(std::move(vff));
        hp.Afa_visc.push_back(std::move(vfa));
      }
    } else if (prm.visc_law == 0) {
      hp.nvisc = 1;
      hp.Gvisc = hp.Gnu;
    } else {
      throw std::runtime_error("unknown viscosity law");
    }
  }
  // slab partitions: velocity node column I -> slab floor(I/2); pressure
  // vertex column I -> slab floor(I/4).  Both orderings are sorted by I first.
  {
    hp.vel_blocks.clear();
    int prev = INT32_MIN;
    for (int i = 0; i < ns; ++i) {
      int s = floordiv(m.I[m.free_nodes[i]], 2);
      if (s != prev) { hp.vel_blocks.push_back(i); prev = s; }
    }
    hp.vel_blocks.push_back(ns);
    hp.p_blocks.clear();
    prev = INT32_MIN;
    for (int k = 0; k < np; ++k) {
      int s = floordiv(m.pI[k], 4);
      if (s != prev) { hp.p_blocks.push_back(k); prev = s; }
    }
    hp.p_blocks.push_back(np);
  }
}

void lsc_middle_values(const HostProblem& hp, const double* S, double* out) {
  const int ns = hp.n_s, np = hp.n_p;
  std::vector<double> acc(np, 0.0);
  for (int k = 0; k < np; ++k) {
    for (int t = hp.B.rowptr[k]; t < hp.B.rowptr[k + 1]; ++t) {
      int cj = hp.B.col[t];
      int c = cj / ns, j = cj % ns;
      double w = hp.B.val[t] / hp.Mstar[j];
      for (int s = hp.Kff.rowptr[j]; s < hp.Kff.rowptr[j + 1]; ++s) {
        int l = hp.Kff.col[s];
        double v = w * S[s] / hp.Mstar[l];
        int cl = c * ns + l;
        for (int u = hp.Bt.rowptr[cl]; u < hp.Bt.rowptr[cl + 1]; ++u) acc[hp.Bt.col[u]] += v * hp.Bt.val[u];
      }
    }
    for (int t = hp.Xmid.rowptr[k]; t < hp.Xmid.rowptr[k + 1]; ++t) {
      out[t] = acc[hp.Xmid.col[t]];
      acc[hp.Xmid.col[t]] = 0.0;
    }
  }
}

void reference_tables(double* out) {
  const RefTables& R = ref();
  for (int g = 0; g < 9; ++g) out[g] = R.w[g];
  for (int g = 0; g < 9; ++g)
    for (int k = 0; k < 9; ++k) {
      out[9 + g * 9 + k] = R.phi[g][k];
      out[90 + g * 9 + k] = R.dxi[g][k];
      out[171 + g * 9 + k] = R.deta[g][k];
    }
}

void convection_values(const HostProblem& hp, const double* w1, const double* w2, double* vff,
                       double* vfa) {
  const Mesh& m = hp.mesh;
  const RefTables& R = ref();
  const double hh = 0.5 * hp.prm.h;   // jac * (2/h)
  std::fill(vff, vff + hp.Kff.nnz(), 0.0);
  if (vfa) std::fill(vfa, vfa + hp.Kfa.nnz(), 0.0);
  for (size_t e = 0; e < m.conn.size(); ++e) {
    const auto& c = m.conn[e];
    double W1[9], W2[9];
    for (int g = 0; g < 9; ++g) {
      double a = 0, b = 0;
      for (int k = 0; k < 9; ++k) {
        a += w1[c[k]] * R.phi[g][k];
        b += w2[c[k]] * R.phi[g][k];
      }
      W1[g] = a;
      W2[g] = b;
    }
    for (int i = 0; i < 9; ++i) {
      int fi = m.free_id[c[i]];
      if (fi < 0) continue;
      for (int j = 0; j < 9; ++j) {
        double s = 0;
        for (int g = 0; g < 9; ++g) s += R.w[g] * (W1[g] * R.dxi[g][j] + W2[g] * R.deta[g][j]) * R.phi[g][i];
        s *= hh;
        if (vfa) vfa[find_pos(hp.Kfa, fi, c[j])] += s;
        int fj = m.free_id[c[j]];
        if (fj >= 0) vff[find_pos(hp.Kff, fi, fj)] += s;
      }
    }
  }
}

void weighted_stiffness_values(const HostProblem& hp, const double* a, double* vff, double* vfa) {
  const Mesh& m = hp.mesh;
  const RefTables& R = ref();
  std::fill(vff, vff + hp.Kff.nnz(), 0.0);
  if (vfa) std::fill(vfa, vfa + hp.Kfa.nnz(), 0.0);
  for (size_t e = 0; e < m.conn.size(); ++e) {
    const auto& c = m.conn[e];
    double ag[9];
    for (int g = 0; g < 9; ++g) {
      double v = 0;
      for (int k = 0; k < 4; ++k) v += a[m.pconn[e][k]] * R.psi[g][k];
      ag[g] = v;
    }
    for (int i = 0; i < 9; ++i) {
      const int fi = m.free_id[c[i]];
      if (fi < 0) continue;
      for (int j = 0; j < 9; ++j) {
        double v = 0;   // (2/h)^2 * jac = 1
        for (int g = 0; g < 9; ++g) v += R.w[g] * ag[g] * (R.dxi[g][i] * R.dxi[g][j] + R.deta[g][i] * R.deta[g][j]);
        if (vfa) vfa[find_pos(hp.Kfa, fi, c[j])] += v;
        const int fj = m.free_id[c[j]];
        if (fj >= 0) vff[find_pos(hp.Kff, fi, fj)] += v;
      }
    }
  }
}

namespace {
// eigen-decomposition of a small symmetric q x q matrix (row-major) by
// cyclic Jacobi rotations: w eigenvalues, V columns eigenvectors
void sym_eigen_small(int q, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)q * q, 0.0);
  for (int i = 0; i < q; ++i) V[(size_t)i * q + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        const double x = A[(size_t)i * q + j] * A[(size_t)i * q + j];
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < q; ++p)
      for (int r = p + 1; r < q; ++r) {
        const double apr = A[(size_t)p * q + r];
        if (apr == 0.0) continue;
        const double app = A[(size_t)p * q + p], arr = A[(size_t)r * q + r];
        const double th = 0.5 * (arr - app) / apr;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < q; ++k) {   // rows p, r
          const double a1 = A[(size_t)p * q + k], a2 = A[(size_t)r * q + k];
          A[(size_t)p * q + k] = cs * a1 - sn * a2;
          A[(size_t)r * q + k] = sn * a1 + cs * a2;
        }
        for (int k = 0; k < q; ++k) {   // columns p, r
          const double a1 = A[(size_t)k * q + p], a2 = A[(size_t)k * q + r];
          A[(size_t)k * q + p] = cs * a1 - sn * a2;
          A[(size_t)k * q + r] = sn * a1 + cs * a2;
        }
        for (int k = 0; k < q; ++k) {
          const double v1 = V[(size_t)k * q + p], v2 = V[(size_t)k * q + r];
          V[(size_t)k * q + p] = cs * v1 - sn * v2;
          V[(size_t)k * q + r] = sn * v1 + cs * v2;
        }
      }
  }
  w.resize(q);
  for (int i = 0; i < q; ++i) w[i] = A[(size_t)i * q + i];
}
}  // namespace

void kl_expansion(const HostProblem& hp, double b, int m, std::vector<double>& beta, std::vector<double>& modes) {
  const Mesh& M = hp.mesh;
  const RefTables& R = ref();
  const int n = hp.n_p, ne = (int)M.pconn.size(), ng = 9 * ne;
  if (ng > 16000) throw std::runtime_error("KL expansion: mesh too fine for the dense covariance quadrature");
  if (m < 1 || m > n) throw std::runtime_error("KL expansion: bad number of modes");
  const double h = hp.prm.h, jw = 0.25 * h * h;
  const double gp[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)};
  std::vector<double> X((size_t)ng), Y((size_t)ng), W((size_t)ng);
  for (int e = 0; e < ne; ++e) {
    const int v0 = M.pconn[e][0];
    const double x0 = M.pI[v0] * h / 2.0, y0 = M.pJ[v0] * h / 2.0;
    for (int g = 0; g < 9; ++g) {
      X[(size_t)e * 9 + g] = x0 + (gp[g % 3] + 1.0) * h / 2.0;
      Y[(size_t)e * 9 + g] = y0 + (gp[g / 3] + 1.0) * h / 2.0;
      W[(size_t)e * 9 + g] = R.w[g] * jw;
    }
  }
  // T = K W Psi (ng x n), then C = Psi^T W T (n x n)
  std::vector<double> T((size_t)ng * n, 0.0);
  for (int gq = 0; gq < ng; ++gq) {
    double* Tg = &T[(size_t)gq * n];
    for (int e = 0; e < ne; ++e)
      for (int g = 0; g < 9; ++g) {
        const int hq = e * 9 + g;
        const double kv = std::exp(-(std::fabs(X[gq] - X[hq]) + std::fabs(Y[gq] - Y[hq])) / b) * W[hq];
        for (int k = 0; k < 4; ++k) Tg[M.pconn[e][k]] += kv * R.psi[g][k];
      }
  }
  std::vector<double> C((size_t)n * n, 0.0);
  for (int e = 0; e < ne; ++e)
    for (int g = 0; g < 9; ++g) {
      const int gq = e * 9 + g;
      for (int k = 0; k < 4; ++k) {
        const double f = W[gq] * R.psi[g][k];
        double* Ck = &C[(size_t)M.pconn[e][k] * n];
        const double* Tg = &T[(size_t)gq * n];
        for (int l = 0; l < n; ++l) Ck[l] += f * Tg[l];
      }
    }
  T.clear();
  T.shrink_to_fit();
  // M_p = L L^T (dense Cholesky), B = L^-1 C L^-T
  std::vector<double> L((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k)
    for (int t = hp.Qp.rowptr[k]; t < hp.Qp.rowptr[k + 1]; ++t) L[(size_t)k * n + hp.Qp.col[t]] = hp.Mp[t];
  for (int j = 0; j < n; ++j) {
    double d = L[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0)) throw std::runtime_error("KL expansion: mass matrix not positive definite");
    d = std::sqrt(d);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = L[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = v / d;
    }
    for (int i = 0; i < j; ++i) L[(size_t)i * n + j] = 0.0;
  }
  auto lower_solve = [&](double* x) {   // x <- L^-1 x
    for (int i = 0; i < n; ++i) {
      double v = x[i];
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * x[k];
      x[i] = v / L[(size_t)i * n + i];
    }
  };
  auto upper_solve = [&](double* x) {   // x <- L^-T x
    for (int i = n - 1; i >= 0; --i) {
      double v = x[i];
      for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * x[k];
      x[i] = v / L[(size_t)i * n + i];
    }
  };
  // B = L^-1 C L^-T: columns of C solved, then rows (C symmetric)
  std::vector<double> Bm(C);
  std::vector<double> col(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) col[i] = Bm[(size_t)i * n + j];
    lower_solve(col.data());
    for (int i = 0; i < n; ++i) Bm[(size_t)i * n + j] = col[i];
  }
  for (int i = 0; i < n; ++i) lower_solve(&Bm[(size_t)i * n]);
  // subspace iteration for the m largest eigenpairs of B (symmetric)
  const int q = std::min(n, m + 8);
  std::vector<double> Xs((size_t)n * q), Z((size_t)n * q);
  uint64_t st = 0x9e3779b97f4a7c15ull;
  for (auto& v : Xs) {
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    v = (double)(st >> 11) / 9007199254740992.0 - 0.5;
  }
  std::vector<double> w, V, prev(m, 0.0);
  auto orthonormalize = [&](std::vector<double>& Q) {   // columns, modified Gram-Schmidt twice
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < q; ++j) {
        for (int k = 0; k < j; ++k) {
          double d = 0;
          for (int i = 0; i < n; ++i) d += Q[(size_t)i * q + k] * Q[(size_t)i * q + j];
          for (int i = 0; i < n; ++i) Q[(size_t)i * q + j] -= d * Q[(size_t)i * q + k];
        }
        double nr = 0;
        for (int i = 0; i < n; ++i) nr += Q[(size_t)i * q + j] * Q[(size_t)i * q + j];
        nr = std::sqrt(nr);
        for (int i = 0; i < n; ++i) Q[(size_t)i * q + j] /= nr;
      }
  };
  orthonormalize(Xs);
  bool done = false;
  for (int it = 0; it < 5000 && !done; ++it) {
    // Z = B Xs
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < q; ++j) {
        double v = 0;
        for (int k = 0; k < n; ++k) v += Bm[(size_t)i * n + k] * Xs[(size_t)k * q + j];
        Z[(size_t)i * q + j] = v;
      }
    orthonormalize(Z);
    // Rayleigh-Ritz: H = Z^T B Z
    std::vector<double> BZ((size_t)n * q), H((size_t)q * q, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < q; ++j) {
        double v = 0;
        for (int k = 0; k < n; ++k) v += Bm[(size_t)i * n + k] * Z[(size_t)k * q + j];
        BZ[(size_t)i * q + j] = v;
      }
    for (int a = 0; a < q; ++a)
      for (int c = 0; c < q; ++c) {
        double v = 0;
        for (int i = 0; i < n; ++i) v += Z[(size_t)i * q + a] * BZ[(size_t)i * q + c];
        H[(size_t)a * q + c] = v;
      }
    for (int a = 0; a < q; ++a)
      for (int c = a + 1; c < q; ++c) H[(size_t)a * q + c] = H[(size_t)c * q + a] = 0.5 * (H[(size_t)a * q + c] + H[(size_t)c * q + a]);
    sym_eigen_small(q, H, w, V);
    std::vector<int> ord(q);
    for (int i = 0; i < q; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return w[x] > w[y]; });
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < q; ++j) {
        double v = 0;
        for (int k = 0; k < q; ++k) v += Z[(size_t)i * q + k] * V[(size_t)k * q + ord[j]];
        Xs[(size_t)i * q + j] = v;
      }
    // converged when the m leading Ritz pairs have residuals ||B x - th x|| <= 1e-13 th_1
    double worst = 0;
    for (int j = 0; j < m; ++j) {
      const double th = w[ord[j]];
      double r2 = 0;
      for (int i = 0; i < n; ++i) {
        double v = 0;
        for (int k = 0; k < n; ++k) v += Bm[(size_t)i * n + k] * Xs[(size_t)k * q + j];
        v -= th * Xs[(size_t)i * q + j];
        r2 += v * v;
      }
      worst = std::max(worst, std::sqrt(r2));
      prev[j] = th;
    }
    done = worst <= 1e-13 * std::fabs(w[ord[0]]);
  }
  if (!done) throw std::runtime_error("KL expansion: subspace iteration did not converge");
  beta.assign(prev.begin(), prev.end());
  modes.assign((size_t)m * n, 0.0);
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < n; ++i) col[i] = Xs[(size_t)i * q + j];
    upper_solve(col.data());
    double amax = 0;
    for (int i = 0; i < n; ++i) amax = std::max(amax, std::fabs(col[i]));
    int first = 0;
    while (std::fabs(col[first]) < 0.5 * amax) ++first;
    const double sgn = col[first] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) modes[(size_t)j * n + i] = sgn * col[i];
  }
}

void pressure_convection_values(const HostProblem& hp, const double* w1, const double* w2, double* out) {
  const Mesh& m = hp.mesh;
  const RefTables& R = ref();
  const double hh = 0.5 * hp.prm.h;   // jac * (2/h)
  std::fill(out, out + hp.Qp.nnz(), 0.0);
  for (size_t e = 0; e < m.conn.size(); ++e) {
    const auto& c = m.conn[e];
    double W1[9], W2[9];
    for (int g = 0; g < 9; ++g) {
      double a = 0, b = 0;
      for (int k = 0; k < 9; ++k) {
        a += w1[c[k]] * R.phi[g][k];
        b += w2[c[k]] * R.phi[g][k];
      }
      W1[g] = a;
      W2[g] = b;
    }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double v = 0;
        for (int g = 0; g < 9; ++g) v += R.w[g] * (W1[g] * R.pdxi[g][j] + W2[g] * R.pdeta[g][j]) * R.psi[g][i];
        out[find_pos(hp.Qp, m.pconn[e][i], m.pconn[e][j])] += v * hh;
      }
  }
}

// ---------------------------------------------------------------- block tridiagonal
namespace {
// in-place inverse of a dense column-major n x n matrix (Gauss-Jordan with
// partial pivoting); returns false if singular
bool dense_inverse(int n, double* A) {
  std::vector<int> piv(n);
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  auto at = [&](std::vector<double>& M, int r, int c) -> double& { return M[(size_t)c * n + r]; };
  std::vector<double> a(A, A + (size_t)n * n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(at(a, k, k));
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(at(a, r, k)) > best) { best = std::fabs(at(a, r, k)); p = r; }
    if (best == 0.0) return false;
    if (p != k)
      for (int c = 0; c < n; ++c) {
        std::swap(at(a, k, c), at(a, p, c));
        std::swap(at(inv, k, c), at(inv, p, c));
      }
    double d = 1.0 / at(a, k, k);
    for (int c = 0; c < n; ++c) { at(a, k, c) *= d; at(inv, k, c) *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      double f = at(a, r, k);
      if (f == 0.0) continue;
      for (int c = 0; c < n; ++c) {
        at(a, r, c) -= f * at(a, k, c);
        at(inv, r, c) -= f * at(inv, k, c);
      }
    }
  }
  std::copy(inv.begin(), inv.end(), A);
  return true;
}

// C (m x n) = A (m x k) * B (k x n), column-major
void gemm_cm(int m, int n, int k, const double* A, const double* B, double* C, double alpha, double beta) {
  for (int j = 0; j < n; ++j) {
    double* cj = C + (size_t)j * m;
    for (int i = 0; i < m; ++i) cj[i] *= beta;
    for (int l = 0; l < k; ++l) {
      double b = alpha * B[(size_t)j * k + l];
      if (b == 0.0) continue;
      const double* al = A + (size_t)l * m;
      for (int i = 0; i < m; ++i) cj[i] += al[i] * b;
    }
  }
}
}  // namespace

namespace {
// run f(i) for i < n on up to 16 host threads
template <class F>
void parallel_for(int n, F&& f) {
  const int nt = std::max(1, std::min<int>({n, 16, (int)std::thread::hardware_concurrency()}));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int i = next++; i < n; i = next++) f(i);
    });
  for (auto& t : th) t.join();
}
}  // namespace

namespace {
// in-place inverse of a dense row-major n x n matrix by Gauss-Jordan with
// partial pivoting; the row updates of each pivot run on host threads
bool dense_inverse_rowmajor_par(int n, double* A) {
  std::vector<double> I((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + k]) > best) { best = std::fabs(A[(size_t)r * n + k]); p = r; }
    if (best == 0.0) return false;
    if (p != k)
      for (int c = 0; c < n; ++c) {
        std::swap(A[(size_t)k * n + c], A[(size_t)p * n + c]);
        std::swap(I[(size_t)k * n + c], I[(size_t)p * n + c]);
      }
    const double inv = 1.0 / A[(size_t)k * n + k];
    for (int c = 0; c < n; ++c) {
      A[(size_t)k * n + c] *= inv;
      I[(size_t)k * n + c] *= inv;
    }
    const double* ak = A + (size_t)k * n;
    const double* ik = I.data() + (size_t)k * n;
    const int nchunk = std::min(n, 64);
    parallel_for(nchunk, [&](int ch) {
      for (int r = ch; r < n; r += nchunk) {
        if (r == k) continue;
        const double fct = A[(size_t)r * n + k];
        if (fct == 0.0) continue;
        double* ar = A + (size_t)r * n;
        double* ir = I.data() + (size_t)r * n;
        for (int c = 0; c < n; ++c) {
          ar[c] -= fct * ak[c];
          ir[c] -= fct * ik[c];
        }
      }
    });
  }
  std::copy(I.begin(), I.end(), A);
  return true;
}
}  // namespace

void bcr_factor(const Csr& pat, const double* vals, const std::vector<int>& blocks, BcrFactor& f,
                std::string& err) {
  const int n = pat.nrows, nb = (int)blocks.size() - 1;
  f = BcrFactor();
  f.n = n;
  f.nblk = nb;
  f.start = blocks;
  std::vector<int> blk(n);
  for (int b = 0; b < nb; ++b) {
    f.maxbs = std::max(f.maxbs, blocks[b + 1] - blocks[b]);
    for (int i = blocks[b]; i < blocks[b + 1]; ++i) blk[i] = b;
  }
  for (int i = 0; i < n; ++i)
    for (int t = pat.rowptr[i]; t < pat.rowptr[i + 1]; ++t)
      if (std::abs(blk[i] - blk[pat.col[t]]) > 1) {
        err = "matrix is not block tridiagonal in the slab ordering";
        return;
      }
  auto bs = [&](int b) { return blocks[b + 1] - blocks[b]; };
  auto extract = [&](int b, int c, std::vector<double>& out) {
    int r0 = blocks[b], nr = bs(b), c0 = blocks[c], nc = bs(c);
    out.assign((size_t)nr * nc, 0.0);
    for (int i = 0; i < nr; ++i)
      for (int t = pat.rowptr[r0 + i]; t < pat.rowptr[r0 + i + 1]; ++t) {
        int j = pat.col[t] - c0;
        if (j >= 0 && j < nc) out[(size_t)j * nr + i] += vals[t];
      }
  };
  // level-l system: positions p -> original block ob[p], dense D, L, U
  std::vector<int> ob(nb);
  std::vector<std::vector<double>> D(nb), L(nb), U(nb);
  for (int b = 0; b < nb; ++b) {
    ob[b] = b;
    extract(b, b, D[b]);
    if (b > 0) extract(b, b - 1, L[b]);
    if (b + 1 < nb) extract(b, b + 1, U[b]);
  }
  auto put = [&](const std::vector<double>& m) {
    int64_t off = (int64_t)f.data.size();
    f.data.insert(f.data.end(), m.begin(), m.end());
    return off;
  };
  constexpr int NT = BcrFactor::NT, NTOP = 8;
  struct Op {
    int out, self, nterm, in[NT];
    int64_t off[NT];
    double coef[NT];
  };
  std::vector<std::vector<Op>> fwd, bwd;
  bool ok = true;
  int np = nb;
  while (np > NTOP) {
    // odd positions: D^-1, D^-1 L, D^-1 U
    const int nodd = np / 2, nev = (np + 1) / 2;
    std::vector<std::vector<double>> Dinv(np), Bt(np), Dl(np);
    std::vector<std::vector<double>> alpha(np), gamma(np);
    std::atomic<bool> bad(false);
    parallel_for(nodd, [&](int q) {
      const int p = 2 * q + 1, b = ob[p];
      Dinv[p] = D[p];
      if (!dense_inverse(bs(b), Dinv[p].data())) {
        bad = true;
        return;
      }
      const int bl = ob[p - 1];
      Bt[p].assign((size_t)bs(b) * bs(bl), 0.0);
      gemm_cm(bs(b), bs(bl), bs(b), Dinv[p].data(), L[p].data(), Bt[p].data(), 1.0, 0.0);
      if (p + 1 < np) {
        const int br = ob[p + 1];
        Dl[p].assign((size_t)bs(b) * bs(br), 0.0);
        gemm_cm(bs(b), bs(br), bs(b), Dinv[p].data(), U[p].data(), Dl[p].data(), 1.0, 0.0);
      }
    });
    if (bad) {
      ok = false;
      break;
    }
    // even positions: alpha = L D_{p-1}^-1, gamma = U D_{p+1}^-1, reduced blocks
    std::vector<std::vector<double>> D2(nev), L2(nev), U2(nev);
    parallel_for(nev, [&](int q) {
      const int p = 2 * q, b = ob[p];
      D2[q] = D[p];
      if (p - 1 >= 0) {
        const int bl = ob[p - 1];
        alpha[p].assign((size_t)bs(b) * bs(bl), 0.0);
        gemm_cm(bs(b), bs(bl), bs(bl), L[p].data(), Dinv[p - 1].data(), alpha[p].data(), 1.0, 0.0);
        gemm_cm(bs(b), bs(b), bs(bl), alpha[p].data(), U[p - 1].data(), D2[q].data(), -1.0, 1.0);
        if (p - 2 >= 0) {
          L2[q].assign((size_t)bs(b) * bs(ob[p - 2]), 0.0);
          gemm_cm(bs(b), bs(ob[p - 2]), bs(bl), alpha[p].data(), L[p - 1].data(), L2[q].data(), -1.0, 0.0);
        }
      }
      if (p + 1 < np) {
        const int br = ob[p + 1];
        gamma[p].assign((size_t)bs(b) * bs(br), 0.0);
        gemm_cm(bs(b), bs(br), bs(br), U[p].data(), Dinv[p + 1].data(), gamma[p].data(), 1.0, 0.0);
        gemm_cm(bs(b), bs(b), bs(br), gamma[p].data(), L[p + 1].data(), D2[q].data(), -1.0, 1.0);
        if (p + 2 < np) {
          U2[q].assign((size_t)bs(b) * bs(ob[p + 2]), 0.0);
          gemm_cm(bs(b), bs(ob[p + 2]), bs(br), gamma[p].data(), U[p + 1].data(), U2[q].data(), -1.0, 0.0);
        }
      }
    });
    std::vector<Op> fo, bo;
    for (int p = 0; p < np; p += 2) {
      Op o{};
      o.out = ob[p];
      o.self = 1;
      if (p - 1 >= 0) {
        o.in[o.nterm] = ob[p - 1];
        o.off[o.nterm] = put(alpha[p]);
        o.coef[o.nterm++] = -1.0;
      }
      if (p + 1 < np) {
        o.in[o.nterm] = ob[p + 1];
        o.off[o.nterm] = put(gamma[p]);
        o.coef[o.nterm++] = -1.0;
      }
      fo.push_back(o);
    }
    for (int p = 1; p < np; p += 2) {
      Op o{};
      o.out = ob[p];
      o.self = 0;
      o.in[o.nterm] = ob[p];
      o.off[o.nterm] = put(Dinv[p]);
      o.coef[o.nterm++] = 1.0;
      o.in[o.nterm] = ob[p - 1];
      o.off[o.nterm] = put(Bt[p]);
      o.coef[o.nterm++] = -1.0;
      if (p + 1 < np) {
        o.in[o.nterm] = ob[p + 1];
        o.off[o.nterm] = put(Dl[p]);
        o.coef[o.nterm++] = -1.0;
      }
      bo.push_back(o);
    }
    fwd.push_back(fo);
    bwd.push_back(bo);
    // next level
    std::vector<int> ob2(nev);
    for (int q = 0; q < nev; ++q) ob2[q] = ob[2 * q];
    ob.swap(ob2);
    D.swap(D2);
    L.swap(L2);
    U.swap(U2);
    np = nev;
  }
  std::vector<Op> top;
  if (ok) {
    // dense system of the remaining np <= NTOP positions, inverted on the host
    std::vector<int> off0(np + 1, 0);
    for (int p = 0; p < np; ++p) off0[p + 1] = off0[p] + bs(ob[p]);
    const int nd = off0[np];
    std::vector<double> A((size_t)nd * nd, 0.0);   // row-major
    auto place = [&](int p, int q, const std::vector<double>& m) {   // m: bs(p) x bs(q), column-major
      const int np_ = bs(ob[p]), nq = bs(ob[q]);
      for (int c = 0; c < nq; ++c)
        for (int r = 0; r < np_; ++r) A[(size_t)(off0[p] + r) * nd + off0[q] + c] = m[(size_t)c * np_ + r];
    };
    for (int p = 0; p < np; ++p) {
      place(p, p, D[p]);
      if (p > 0) place(p, p - 1, L[p]);
      if (p + 1 < np) place(p, p + 1, U[p]);
    }
    if (!dense_inverse_rowmajor_par(nd, A.data())) ok = false;
    for (int q = 0; ok && q < np; ++q) {
      Op o{};
      o.out = ob[q];
      o.self = 0;
      const int nq = bs(ob[q]);
      for (int p = 0; p < np; ++p) {
        const int npp = bs(ob[p]);
        std::vector<double> blk((size_t)nq * npp);   // column-major nq x npp
        for (int c = 0; c < npp; ++c)
          for (int r = 0; r < nq; ++r) blk[(size_t)c * nq + r] = A[(size_t)(off0[q] + r) * nd + off0[p] + c];
        o.in[o.nterm] = ob[p];
        o.off[o.nterm] = put(blk);
        o.coef[o.nterm++] = 1.0;
      }
      top.push_back(o);
    }
  }
  if (!ok) {
    err = "singular block in block cyclic reduction";
    return;
  }
  auto emit = [&](const std::vector<Op>& ops) {
    for (const Op& o : ops) {
      f.op_out.push_back(o.out);
      f.op_self.push_back(o.self);
      f.op_nterm.push_back(o.nterm);
      for (int t = 0; t < NT; ++t) {
        f.op_in.push_back(t < o.nterm ? o.in[t] : 0);
        f.op_off.push_back(t < o.nterm ? o.off[t] : 0);
        f.op_coef.push_back(t < o.nterm ? o.coef[t] : 0.0);
      }
    }
    f.pass_begin.push_back((int)f.op_out.size());
  };
  f.pass_begin.push_back(0);
  for (const auto& ops : fwd) {
    emit(ops);
    f.pass_mode.push_back(0);
  }
  emit(top);
  f.pass_mode.push_back(2);
  for (int l = (int)bwd.size() - 1; l >= 0; --l) {
    emit(bwd[l]);
    f.pass_mode.push_back(1);
  }
  // Columns of a term matrix that are exactly zero at either end are left
  // out: the input rows they multiply are not read.  In the back
  // substitution D^-1 L couples only the neighbour's rows that the original
  // off-diagonal block touches (one node column of the slab).  A term whose
  // matrix is zero altogether is dropped.
  const size_t nops = f.op_out.size();
  f.op_k0.assign(nops * NT, 0);
  f.op_kn.assign(nops * NT, 0);
  for (size_t o = 0; o < nops; ++o) {
    const int bo = f.start[f.op_out[o] + 1] - f.start[f.op_out[o]];
    int w = 0;
    for (int t = 0; t < f.op_nterm[o]; ++t) {
      const size_t q = NT * o + t;
      const int ib = f.op_in[q], bi = f.start[ib + 1] - f.start[ib];
      const double* m = f.data.data() + f.op_off[q];
      auto zero_col = [&](int k) {
        for (int r = 0; r < bo; ++r)
          if (m[(size_t)k * bo + r] != 0.0) return false;
        return true;
      };
      int k0 = 0, k1 = bi;
      while (k0 < k1 && zero_col(k0)) ++k0;
      while (k1 > k0 && zero_col(k1 - 1)) --k1;
      if (k1 == k0) continue;
      const size_t qw = NT * o + w++;
      f.op_in[qw] = ib;
      f.op_off[qw] = f.op_off[q];
      f.op_coef[qw] = f.op_coef[q];
      f.op_k0[qw] = k0;
      f.op_kn[qw] = k1 - k0;
    }
    f.op_nterm[o] = w;
  }
  // An op whose terms are zero on whole row ranges of the output block is
  // split in two at the row where that saves most (when it saves at least a
  // tenth of the op's matrix data): each half keeps the terms that touch it.
  // In the forward passes U D^-1 is zero on the rows of the slab's first node
  // column.  A forward op left with nothing to add is dropped.
  BcrFactor g;
  g.op_out.reserve(nops);
  g.pass_begin.push_back(0);
  for (size_t p = 0; p + 1 < f.pass_begin.size(); ++p) {
    for (int o = f.pass_begin[p]; o < f.pass_begin[p + 1]; ++o) {
      const int bo = f.start[f.op_out[o] + 1] - f.start[f.op_out[o]];
      const int nt = f.op_nterm[o];
      std::vector<int> lo(nt), hi(nt);
      double total = 0.0;
      for (int t = 0; t < nt; ++t) {
        const size_t q = NT * o + t;
        const double* m = f.data.data() + f.op_off[q] + (size_t)f.op_k0[q] * bo;
        const int kn = f.op_kn[q];
        auto zero_row = [&](int r) {
          for (int k = 0; k < kn; ++k)
            if (m[(size_t)k * bo + r] != 0.0) return false;
          return true;
        };
        lo[t] = 0;
        hi[t] = bo;
        while (lo[t] < hi[t] && zero_row(lo[t])) ++lo[t];
        while (hi[t] > lo[t] && zero_row(hi[t] - 1)) --hi[t];
        total += (double)bo * kn;
      }
      int best = 0;
      double best_save = 0.0;
      for (int t = 0; t < nt; ++t)
        for (int rb : {lo[t], hi[t]}) {
          if (rb <= 0 || rb >= bo) continue;
          double save = 0.0;
          for (int u = 0; u < nt; ++u) {
            // rows [0, rb) need term u only if it starts there, [rb, bo) only
            // if it ends there
            if (lo[u] >= rb || lo[u] >= hi[u]) save += (double)rb * f.op_kn[NT * o + u];
            if (hi[u] <= rb || lo[u] >= hi[u]) save += (double)(bo - rb) * f.op_kn[NT * o + u];
          }
          if (save > best_save) {
            best_save = save;
            best = rb;
          }
        }
      const bool split = best > 0 && best_save >= 0.1 * total;
      for (int half = 0; half < (split ? 2 : 1); ++half) {
        const int a = split && half == 1 ? best : 0, b = split && half == 0 ? best : bo;
        std::vector<int> keep;
        for (int t = 0; t < nt; ++t)
          if (!split || (lo[t] < b && hi[t] > a)) keep.push_back(t);
        if (keep.empty() && f.pass_mode[p] == 0 && f.op_self[o]) continue;   // b stays as it is
        g.op_out.push_back(f.op_out[o]);
        g.op_self.push_back(f.op_self[o]);
        g.op_row0.push_back(a);
        g.op_rows.push_back(b - a);
        g.op_nterm.push_back((int)keep.size());
        for (int t = 0; t < NT; ++t) {
          const size_t q = t < (int)keep.size() ? NT * o + keep[t] : 0;
          const bool on = t < (int)keep.size();
          g.op_in.push_back(on ? f.op_in[q] : 0);
          g.op_off.push_back(on ? f.op_off[q] : 0);
          g.op_coef.push_back(on ? f.op_coef[q] : 0.0);
          g.op_k0.push_back(on ? f.op_k0[q] : 0);
          g.op_kn.push_back(on ? f.op_kn[q] : 0);
        }
      }
    }
    g.pass_begin.push_back((int)g.op_out.size());
  }
  f.op_out.swap(g.op_out);
  f.op_self.swap(g.op_self);
  f.op_row0.swap(g.op_row0);
  f.op_rows.swap(g.op_rows);
  f.op_nterm.swap(g.op_nterm);
  f.op_in.swap(g.op_in);
  f.op_off.swap(g.op_off);
  f.op_coef.swap(g.op_coef);
  f.op_k0.swap(g.op_k0);
  f.op_kn.swap(g.op_kn);
  f.pass_begin.swap(g.pass_begin);
}


void bcr_apply_host(const BcrFactor& f, int ncols, const double* b, double* x) {
  constexpr int NT = BcrFactor::NT;
  const size_t nv = (size_t)f.n * ncols;
  std::vector<double> B(b, b + nv), X(nv, 0.0);
  for (size_t p = 0; p + 1 < f.pass_begin.size(); ++p) {
    const int mode = f.pass_mode[p];
    std::vector<double>& out = mode != 0 ? X : B;
    std::vector<double> res = out;   // ops of a pass read the state before the pass
    parallel_for(f.pass_begin[p + 1] - f.pass_begin[p], [&](int q) {
      const int o = f.pass_begin[p] + q, ob = f.op_out[o];
      const int ld = f.start[ob + 1] - f.start[ob], row0 = f.op_row0[o], r0 = f.start[ob] + row0;
      for (int r = 0; r < f.op_rows[o]; ++r)
        for (int c = 0; c < ncols; ++c) {
          double acc = f.op_self[o] ? B[(size_t)(r0 + r) * ncols + c] : 0.0;
          for (int t = 0; t < f.op_nterm[o]; ++t) {
            const int ib = f.op_in[NT * o + t], k0 = f.op_k0[NT * o + t], kn = f.op_kn[NT * o + t];
            const int i0 = f.start[ib] + k0;
            const std::vector<double>& src = (mode == 1 && ib != ob) ? X : B;
            const double* m = f.data.data() + f.op_off[NT * o + t] + (size_t)k0 * ld + row0;
            double sum = 0.0;
            for (int k = 0; k < kn; ++k) sum += m[(size_t)k * ld + r] * src[(size_t)(i0 + k) * ncols + c];
            acc += f.op_coef[NT * o + t] * sum;
          }
          res[(size_t)(r0 + r) * ncols + c] = acc;
        }
    });
    out.swap(res);
  }
  std::copy(X.begin(), X.end(), x);
}

}  // namespace sgtt
