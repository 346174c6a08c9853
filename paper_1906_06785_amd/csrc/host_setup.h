// Host-side problem setup for the step-domain stochastic Galerkin system.
//
// Mesh and Q2-Q1 Taylor-Hood assembly (sec. 3.2, eq. 3.7-3.8; sec. 6.1),
// Legendre chaos matrices G_l, H_l (eq. 3.9), convection matrices N(w)
// (eq. 3.7) for given wind vectors, pressure-space LSC matrices
// B M*^-1 S M*^-1 B^T (eq. 5.19), and block-tridiagonal factorizations of
// the spatial matrices used by the mean-based preconditioner (eq. 5.19,
// eq. 5.23).  Plain C++; no device code here.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace sgtt {

struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int> rowptr, col;
  std::vector<double> val;           // one value array; extra value sets live elsewhere
  int nnz() const { return (int)col.size(); }
};

struct ProblemParams {
  double h = 0.25, L = 12.0;
  int m = 2, p = 2, nt = 10;
  double tau = 0.1, nu0 = 1.0 / 50, nu_coef = 0.1, ramp = 10.0;
  // 0: nu0 (1 + nu_coef sum_k xi_k / k^2), xi_k ~ U[-1,1]; 1: truncated KL
  // expansion of exp(-||x - y||_1 / corr_length) (sec. 6.1), sigma = nu_coef,
  // xi_k ~ U[-sqrt 3, sqrt 3]
  int visc_law = 0;
  double corr_length = 4.0;
};

struct Mesh {
  double h = 0, L = 0;
  int q = 0;                          // 1/h
  std::vector<int> I, J;              // lattice coordinates of velocity nodes (x = I*h/2)
  std::vector<int> pI, pJ;            // lattice coordinates of pressure nodes
  std::vector<std::array<int, 9>> conn;   // element -> velocity node (local a + 3 b)
  std::vector<std::array<int, 4>> pconn;  // element -> pressure node (local a + 2 b)
  std::vector<int> free_nodes, dir_nodes;  // sorted by (x1, x2)
  std::vector<int> free_id;           // node -> free index or -1
  std::vector<int> dir_id;            // node -> Dirichlet index or -1
  std::vector<double> g1;             // x1 inflow value at each node (0 if not inflow)
  int n_all() const { return (int)I.size(); }
  int n_s() const { return (int)free_nodes.size(); }
  int n_p() const { return (int)pI.size(); }
};


struct HostProblem {
  ProblemParams prm;
  Mesh mesh;
  int n_s = 0, n_u = 0, n_p = 0, n_all = 0, n_xi = 0, nt = 0;
  // scalar velocity pattern on free x free nodes with M and unit-viscosity A
  Csr Kff;                            // pattern; val unused
  std::vector<double> Mff, Aff;
  // scalar pattern free rows x all nodes (for residuals with the Dirichlet lift)
  Csr Kfa;
  std::vector<double> Mfa, Afa;
  // divergence: B (n_p x n_u, free dofs, columns [comp1 | comp2]) and B^T
  Csr B, Bt;
  // divergence against all velocity nodes: n_p x 2 n_all
  Csr Ball;
  // chaos
  std::vector<std::vector<int>> midx;
  std::vector<double> G;              // (m+1) x n_xi x n_xi
  std::vector<double> H;              // n_xi x n_xi x n_xi  (H[0] = I)
  std::vector<double> visc;           // c_0..c_m
  std::vector<double> Gnu;            // n_xi x n_xi
  // viscous terms sum_t Gv_t (x) A_t of eq. 3.6: nvisc chaos matrices
  // (n_xi x n_xi each) and stiffness value sets on Kff and Kfa.  Law 0: one
  // term G_nu (x) A (unit A); law 1: nu0 I (x) A and sqrt 3 G_l (x)
  // nu0 sigma sqrt(beta_l) A(a_l), l = 1..m.  Value set 0 is always the
  // unit-viscosity A (the mean operator uses nu0 times it).
  int nvisc = 1;
  std::vector<double> Gvisc;
  std::vector<std::vector<double>> Aff_visc, Afa_visc;
  // KL expansion (law 1): eigenvalues beta_l and modes a_l at the Q1
  // vertices (m x n_p, int a_l^2 = 1)
  std::vector<double> kl_beta, kl_modes;
  // time
  std::vector<double> ramp;           // a_k = 1 - exp(-ramp t_k), k = 1..nt
  // Dirichlet lift over all velocity nodes: g_all (2 n_all)
  std::vector<double> g_all;
  // M_* = diag(M) on free dofs (length n_s; both components share it)
  std::vector<double> Mstar;
  // pressure Laplacian X = B M*^-1 B^T and its pattern (n_p x n_p)
  Csr Xp;                             // pattern + values of X
  Csr Xmid;                           // pattern for B M*^-1 S M*^-1 B^T (S = M, A, N)
  std::vector<double> XM, XA;         // values on Xmid for S = M, S = A (unit)
  // Q1 pressure-space matrices of the PCD approximation (eq. 5.17): pattern,
  // mass M_p, unit-viscosity stiffness A_p (natural boundary conditions) and
  // diag(M_p)
  Csr Qp;
  std::vector<double> Mp, Ap, Mpstar;
  // slab partitions (block-tridiagonal orderings) of free velocity nodes and
  // pressure nodes
  std::vector<int> vel_blocks, p_blocks;
};

// Build everything that does not depend on a prior iterate.
void build_problem(const ProblemParams& prm, HostProblem& hp);

// Convection matrix values N(w) (eq. 3.7) for a wind given at all velocity
// nodes (w1, w2 of length n_all): values on Kff (free x free) and, if
// vals_fa != nullptr, on Kfa (free x all).
void convection_values(const HostProblem& hp, const double* w1, const double* w2,
                       double* vals_ff, double* vals_fa);

// Truncated Karhunen-Loeve expansion of exp(-||x - y||_1 / b) on the mesh
// (sec. 6.1): Galerkin on the Q1 vertex space, C a = beta M_p a with
// C_kl = int int c(x, y) psi_k(x) psi_l(y) by 3 x 3 Gauss quadrature in both
// integrals; the m largest eigenpairs by subspace iteration, modes
// M_p-orthonormal, signed so that the first vertex with |a| >= max|a| / 2
// has a > 0.  Throws when the quadrature would not fit (meshes finer than
// h = 1/8).
void kl_expansion(const HostProblem& hp, double b, int m, std::vector<double>& beta, std::vector<double>& modes);
// Values of the stiffness with coefficient field a (Q1 vertex values,
// interpolated to the Gauss points) on Kff and, if vals_fa != nullptr, Kfa.
void weighted_stiffness_values(const HostProblem& hp, const double* a_vertex, double* vals_ff, double* vals_fa);

// Q1 pressure-space convection values [N_p(w)]_kl = (w . grad psi_l, psi_k)
// on Qp for a Q2 wind given at all velocity nodes (sec. 5.1, F_p).
void pressure_convection_values(const HostProblem& hp, const double* w1, const double* w2, double* out);

// Q2 reference-element tables on the 3 x 3 Gauss points (the ones every
// assembly here uses): out[0..8] weights, then phi, d/dxi, d/deta as [g][k]
// (81 each, k = a + 3 b): 252 doubles.
void reference_tables(double* out);

// Values of B M*^-1 S M*^-1 B^T on the Xmid pattern for a scalar velocity
// matrix S given by values on Kff (applied to both components).
void lsc_middle_values(const HostProblem& hp, const double* Svals, double* out);

// Block cyclic reduction of a block-tridiagonal matrix: level l eliminates
// the odd positions of the level-l system (stride 2^l in the original block
// numbering).  The solve is a sequence of passes, each a set of independent
// block operations  out = [b_out] + sum_t coef_t M_t v_{in_t}  (M_t dense,
// col-major): forward passes (levels 0, 1, ...) update the even positions'
// right-hand sides b in place from their odd neighbours' b; then the top
// solve and the backward passes (top level down) write the solution x of the
// odd positions from their own b and their neighbours' x.  The reduction stops
// at 8 blocks or fewer; their system is solved with a dense inverse (one op
// per block, one term per block of the top system).
struct BcrFactor {
  int n = 0, nblk = 0, maxbs = 0;
  std::vector<int> start;              // nblk + 1
  std::vector<int> op_out, op_self;    // per op: output block, 1 = add v_out
  // per op: the rows [row0, row0 + rows) of the output block it writes; its
  // term matrices are stored for the whole block (rows of the block, column-
  // major) and the op uses their rows row0 ..
  std::vector<int> op_row0, op_rows;
  static constexpr int NT = 16;         // terms per op (at most)
  std::vector<int> op_nterm;           // per op: number of terms
  std::vector<int> op_in;              // NT per op
  std::vector<int64_t> op_off;         // NT per op: matrix offsets in data
  std::vector<double> op_coef;         // NT per op
  // NT per op: the term reads rows [k0, k0 + kn) of its input block and
  // multiplies them by columns [k0, k0 + kn) of its matrix (the others are
  // exactly zero)
  std::vector<int> op_k0, op_kn;
  std::vector<int> pass_begin;         // op ranges of the passes (npass + 1)
  // per pass: 0 reduce the right-hand side in place (inputs from b);
  // 2 solve the top system (inputs from b, output x); 1 back substitution
  // (own block from b, neighbours from x, output x)
  std::vector<int> pass_mode;
  std::vector<double> data;
};
void bcr_factor(const Csr& pat, const double* vals, const std::vector<int>& blocks, BcrFactor& f,
                std::string& err);
// The factor's op lists applied on the host (reference of the device
// passes): x = A^-1 b for ncols columns, row-major (row r at r * ncols).
void bcr_apply_host(const BcrFactor& f, int ncols, const double* b, double* x);




}  // namespace sgtt
