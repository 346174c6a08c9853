"""Oracle: the all-at-once stochastic Galerkin system of one Picard step.

Test infrastructure only (see oracle/__init__.py).

Operator (eq. 3.10-3.12 with eq. 3.14 and eq. 4.12-4.14):

    L = [[F + C, B^T], [B, 0]],
    F + C = tau^-1 (I - C_nt) (x) I (x) M  +  I (x) G_nu (x) A  +  N(w~),
    N(w~) = sum_{a,b} diag(w1_a) (x) (sum_l w2(a,l,b) H_l) (x) N(w3_b),
    B-blocks = I (x) I (x) B,

with bold M, A, N block-diagonal over the two velocity components,
C_nt = ones on the sub-diagonal, G_nu = sum_l c_l G_l for the viscosity
nu0 (1 + 0.1 sum_k xi_k / k^2) (eq. 3.6 with A_l = c_l A).

Right-hand side: Dirichlet data u_D = (1 - 4 x2^2)(1 - exp(-10 t)) e_1 on the
inflow (eq. 6.1), zero on walls, lifted to the right-hand side (sec. 3.2).
For a Picard step with prior iterate w the system is the residual equation
eq. 3.14 with r = f - L(w) [w; p_w] computed with the untruncated w (eq. 3.15,
sec. 4.3), while the operator uses w~ = T_eps_conv(w) (eq. 4.13-4.14).  The
convection field w is the full FE velocity: free TT plus the rank-1 Dirichlet
lift (a reading; the paper is silent).

Direct references (pins for the iterative solvers): a dense/sparse LU of the
explicit all-at-once matrix at tiny sizes and, at larger sizes, exact block
forward substitution in time (the system is block lower-bidiagonal in time).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import gpc, mesh as fem, tt


class Convection:
    """TT-operator form of N(w) (eq. 4.12) for a TT wind over ALL velocity
    nodes: w1 (n_t x k1), Hw[a,b] = sum_l w2(a,l,b) H_l, N_b = N(w3_b)."""

    def __init__(self, prob, w_all):
        G1, G2, G3 = w_all
        self.k1, self.k2 = G1.shape[1], G3.shape[0]
        self.w1 = G1
        self.w2 = G2
        # Hw[a, b] = sum_l G2[a, l, b] H_l   (H_l indexed from 0 = psi_1)
        self.Hw = np.einsum("alb,lij->abij", G2, prob.H)
        na = prob.mesh.n_all
        f = prob.mesh.free
        self.w3 = G3
        self.Nall = [fem.convection(prob.mesh, G3[b, :na], G3[b, na:]) for b in range(self.k2)]
        self.N_ff = [N[f][:, f].tocsr() for N in self.Nall]
        # bold (two-component) free-row restrictions
        self.Nb_ff = [sp.block_diag([N, N]).tocsr() for N in self.N_ff]
        self.Nb_fall = [sp.block_diag([N[f], N[f]]).tocsr() for N in self.Nall]
        # mean (psi_1 mode) convection: omega_b(t) = sum_a w1[t,a] w2[a,0,b]
        self.omega = G1 @ G2[:, 0, :]
        self.avg_coef = self.omega.mean(axis=0)

    def ttm_apply(self, x, which="ff", mean=False):
        """N(w) x (or the mean convection N_0 x of eq. 5.21) as an exact TT with
        ranks (k1 r1, k2 r2)."""
        G1, G2, G3 = x
        r1, n2, r2 = G2.shape
        O1 = (self.w1[:, :, None] * G1[:, None, :]).reshape(G1.shape[0], self.k1 * r1)
        if mean:
            Hw = np.einsum("ab,ij->abij", self.w2[:, 0, :], np.eye(n2))
        else:
            Hw = self.Hw
        O2 = np.einsum("abij,cjd->acibd", Hw, G2).reshape(self.k1 * r1, n2, self.k2 * r2)
        mats = self.Nb_ff if which == "ff" else self.Nb_fall
        O3 = np.concatenate([np.asarray(mats[b] @ G3.T).T for b in range(self.k2)], axis=0)
        return O1, O2, O3

    def full_apply(self, X, which="ff", mean=False):
        """Same operator applied to a full (n_t, n_xi, n_x) tensor."""
        nt, n2 = X.shape[0], X.shape[1]
        mats = self.Nb_fall if which == "fall" else self.Nb_ff
        Y = None
        for b in range(self.k2):
            Z = np.asarray(mats[b] @ X.reshape(nt * n2, -1).T).T.reshape(nt, n2, -1)
            if mean:
                Y_b = self.omega[:, b][:, None, None] * Z
            else:
                Y_b = np.einsum("ta,aij,tjx->tix", self.w1, self.Hw[:, b], Z, optimize=True)
            Y = Y_b if Y is None else Y + Y_b
        return Y


class Problem:
    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.mesh = fem.build_mesh(cfg["h"], cfg.get("L", 12.0))
        M, A, B1, B2, Mp = fem.assemble(self.mesh)
        self.M_all, self.A_all, self.Mp = M, A, Mp
        f, d = self.mesh.free, self.mesh.dirichlet
        self.n_s, self.n_u, self.n_p, self.n_all = self.mesh.n_s, self.mesh.n_u, self.mesh.n_p, self.mesh.n_all
        self.M = M[f][:, f].tocsr()
        self.A = A[f][:, f].tocsr()
        self.Mb = sp.block_diag([self.M, self.M]).tocsr()
        self.Ab = sp.block_diag([self.A, self.A]).tocsr()
        self.B = sp.hstack([B1[:, f], B2[:, f]]).tocsr()          # n_p x n_u
        self.Bt = self.B.T.tocsr()
        self.Mb_fall = sp.block_diag([M[f], M[f]]).tocsr()        # n_u x 2 n_all
        self.Ab_fall = sp.block_diag([A[f], A[f]]).tocsr()
        self.B_all = sp.hstack([B1, B2]).tocsr()                  # n_p x 2 n_all
        self.idx, self.G, self.H = gpc.gpc_matrices(cfg["m"], cfg["p"])
        self.n_xi = len(self.idx)
        self.c = gpc.viscosity_coefficients(cfg["m"], cfg["nu0"], cfg["nu_coef"])
        self.Gnu = np.einsum("l,lij->ij", self.c, self.G)
        # viscous terms sum_l G_l (x) A_l of eq. 3.6 as (chaos matrix, free x
        # free, free x all scalar stiffness): one term G_nu (x) A for the law
        # nu0 (1 + sigma sum xi_k / k^2) (A_l proportional to A); m + 1 terms
        # for the KL law of sec. 6.1, xi_k ~ U[-sqrt 3, sqrt 3] (G_l scaled by
        # sqrt 3) and A_l = nu0 sigma sqrt(beta_l) A(a_l)
        if cfg.get("viscosity", "power") == "kl":
            from . import kl
            self.kl_beta, self.kl_modes = kl.viscosity_fields(self.mesh, cfg["corr_length"], cfg["m"])
            terms = [(cfg["nu0"] * self.G[0], A)]
            for l in range(cfg["m"]):
                Al = fem.stiffness_weighted(self.mesh, self.kl_modes[l])
                terms.append((np.sqrt(3.0) * self.G[l + 1],
                              cfg["nu0"] * cfg["nu_coef"] * np.sqrt(self.kl_beta[l]) * Al))
        else:
            terms = [(self.Gnu, A)]
        self.visc = []
        for Gl, Al in terms:
            Af, Afa = Al[f][:, f].tocsr(), Al[f]
            self.visc.append((Gl, sp.block_diag([Af, Af]).tocsr(), sp.block_diag([Afa, Afa]).tocsr()))
        self.nt, self.tau = cfg["nt"], cfg["tau"]
        self.Ct = sp.diags([np.ones(self.nt - 1)], [-1], shape=(self.nt, self.nt)).tocsr()
        self.It = sp.identity(self.nt, format="csr")
        self.tk = self.tau * np.arange(1, self.nt + 1)
        self.ramp = 1.0 - np.exp(-cfg["ramp"] * self.tk)
        gall = np.zeros(2 * self.n_all)
        gall[d] = self.mesh.g1
        self.g_all = gall
        # mass-matrix diagonal M_* (sec. 5.1, "diagonal entries")
        self.Mstar = np.concatenate([self.M.diagonal(), self.M.diagonal()])

    # ---------- TT helpers ----------
    def embed(self, u):
        """Free-node velocity TT -> all-node velocity TT (zeros at Dirichlet nodes)."""
        G1, G2, G3 = u
        f, na, ns = self.mesh.free, self.n_all, self.n_s
        G3a = np.zeros((G3.shape[0], 2 * na))
        G3a[:, f] = G3[:, :ns]
        G3a[:, na + f] = G3[:, ns:]
        return G1, G2, G3a

    def lift(self):
        e1 = np.zeros(self.n_xi)
        e1[0] = 1.0
        return self.ramp[:, None], e1[None, :, None], self.g_all[None, :]

    def wind(self, prior):
        """All-node wind TT = embedded free velocity + Dirichlet lift."""
        if prior is None:
            return self.lift()
        return tt.concat([self.embed(prior[0]), self.lift()])

    def convection(self, prior, eps_conv):
        """N(w~) with w~ = T_eps_conv(w) (eq. 4.13); None for the Stokes system."""
        if prior is None:
            return None
        return Convection(self, tt.tt_round(self.wind(prior), eps_conv))

    # ---------- operator ----------
    def apply(self, x, conv=None):
        """L x as an exact TT pair (no truncation)."""
        u, p = x
        It_C = (self.It - self.Ct) / self.tau
        parts = [tt.mode_apply(u, It_C, None, self.Mb)]
        parts += [tt.mode_apply(u, None, Gl, Ab) for Gl, Ab, _ in self.visc]
        parts.append(tt.mode_apply(p, None, None, self.Bt))
        if conv is not None:
            parts.append(conv.ttm_apply(u))
        yu = tt.concat(parts)
        yp = tt.mode_apply(u, None, None, self.B)
        return yu, yp

    def apply_full(self, xu, xp, conv=None):
        """L applied to full tensors xu (n_t, n_xi, n_u), xp (n_t, n_xi, n_p)."""
        nt, nx = self.nt, self.n_xi
        U = xu.reshape(nt * nx, self.n_u)
        MU = np.asarray(self.Mb @ U.T).T.reshape(nt, nx, -1)
        yu = MU.copy()
        yu[1:] -= MU[:-1]
        yu /= self.tau
        for Gl, Ab, _ in self.visc:
            AU = np.asarray(Ab @ U.T).T.reshape(nt, nx, -1)
            yu += np.einsum("ij,tjx->tix", Gl, AU)
        yu += np.asarray(self.Bt @ xp.reshape(nt * nx, -1).T).T.reshape(nt, nx, -1)
        if conv is not None:
            yu += conv.full_apply(xu)
        yp = np.asarray(self.B @ U.T).T.reshape(nt, nx, -1)
        return yu, yp

    def residual_entries(self, b, x, which, t, i, j, conv=None):
        """Entries r[t_k, i_k, j_k] of r = b - L x (eq. 3.11-3.12), one by one
        from the TT cores: each sparse operator row touches only the core-3
        columns of its nonzeros.  which = "u" (velocity rows, free dofs) or
        "p" (pressure rows).  No full tensor is formed, so this works at any
        size.  With conv, the velocity rows include N(w~) u in the form of
        eq. 4.12: sum_{a,b} w1[t,a] sum_k Hw[a,b][i,k] (N_b u_{t,k})_j."""
        u, pp = x
        t = np.asarray(t, dtype=np.int64)
        i = np.asarray(i, dtype=np.int64)
        j = np.asarray(j, dtype=np.int64)
        # core1 x core2 contracted once per TT: G12[t] is the (n_xi x r2) slice
        g12 = {}

        def G12(G):
            key = id(G)
            if key not in g12:
                g12[key] = np.einsum("ta,aib->tib", G[0], G[1])
            return g12[key]

        def row_vals(G, mat, tk, row):
            # (mat @ X_t^T)[row] for all chaos indices: (n_xi,)  with X_t = G1[t] G2 G3
            lo, hi = mat.indptr[row], mat.indptr[row + 1]
            cols, vals = mat.indices[lo:hi], mat.data[lo:hi]
            return G12(G)[tk] @ (G[2][:, cols] @ vals)

        def entry_of(G, tk, ik, row, mat):
            return row_vals(G, mat, tk, row)[ik]

        out = np.empty(len(t))
        if which == "u":
            Iu = sp.identity(self.n_u, format="csr")
            for k in range(len(t)):
                tk, ik, jk = int(t[k]), int(i[k]), int(j[k])
                mu = row_vals(u, self.Mb, tk, jk)
                if tk > 0:
                    mu = mu - row_vals(u, self.Mb, tk - 1, jk)
                lx = mu[ik] / self.tau + entry_of(pp, tk, ik, jk, self.Bt)
                for Gl, Ab, _ in self.visc:
                    lx += Gl[ik] @ row_vals(u, Ab, tk, jk)
                if conv is not None:
                    for bb in range(conv.k2):
                        nv = row_vals(u, conv.Nb_ff[bb], tk, jk)          # over chaos index k
                        for a in range(conv.k1):
                            lx += conv.w1[tk, a] * (conv.Hw[a, bb][ik] @ nv)
                out[k] = entry_of(b[0], tk, ik, jk, Iu) - lx
        else:
            Ip = sp.identity(self.n_p, format="csr")
            for k in range(len(t)):
                tk, ik, jk = int(t[k]), int(i[k]), int(j[k])
                out[k] = entry_of(b[1], tk, ik, jk, Ip) - entry_of(u, tk, ik, jk, self.B)
        return out

    def explicit(self, conv=None):
        """Explicit sparse all-at-once matrix (scipy.sparse.kron), small sizes."""
        kron = sp.kron
        Kuu = kron(kron((self.It - self.Ct) / self.tau, sp.identity(self.n_xi)), self.Mb)
        for Gl, Ab, _ in self.visc:
            Kuu = Kuu + kron(kron(self.It, sp.csr_matrix(Gl)), Ab)
        if conv is not None:
            for a in range(conv.k1):
                for b in range(conv.k2):
                    Kuu = Kuu + kron(kron(sp.diags(conv.w1[:, a]), sp.csr_matrix(conv.Hw[a, b])),
                                     conv.Nb_ff[b])
        I2 = sp.identity(self.nt * self.n_xi)
        Kup = kron(I2, self.Bt)
        Kpu = kron(I2, self.B)
        return sp.bmat([[Kuu, Kup], [Kpu, None]]).tocsc()

    # ---------- right-hand side ----------
    def residual_tt(self, prior):
        """Exact TT of r = -(L_{free,all}(w) w_all + B^T p) for the prior iterate
        (Stokes: prior=None gives f).  Velocity rows are free rows only."""
        wall = self.wind(prior)
        It_C = (self.It - self.Ct) / self.tau
        parts = [tt.mode_apply(wall, It_C, None, self.Mb_fall)]
        parts += [tt.mode_apply(wall, None, Gl, Abfa) for Gl, _, Abfa in self.visc]
        if prior is not None:
            conv = Convection(self, wall)
            parts.append(conv.ttm_apply(wall, which="fall"))
            parts.append(tt.mode_apply(prior[1], None, None, self.Bt))
        ru = tt.scale(tt.concat(parts), -1.0)
        rp = tt.scale(tt.mode_apply(wall, None, None, self.B_all), -1.0)
        return ru, rp

    def rhs(self, prior=None, eps_rhs=1e-10):
        """Right-hand side TT pair of the Picard-step system: exact (ranks <= 2
        and 1) for Stokes; TT-SVD (Alg. 4.1) of the full residual otherwise."""
        r = self.residual_tt(prior)
        if prior is None:
            return r
        return tt.tt_svd(tt.full(r[0]), eps_rhs), tt.tt_svd(tt.full(r[1]), eps_rhs)

    # ---------- reference solutions ----------
    def solve_direct(self, bu, bp, conv=None):
        """Exact solution of L z = b by block forward substitution in time: at
        each step solve the SG saddle-point block with scipy's sparse LU."""
        nt, nx, nu, npp = self.nt, self.n_xi, self.n_u, self.n_p
        Ix = sp.identity(nx)
        base = sp.kron(Ix, self.Mb) / self.tau
        for Gl, Ab, _ in self.visc:
            base = base + sp.kron(sp.csr_matrix(Gl), Ab)
        Kup = sp.kron(Ix, self.Bt)
        Kpu = sp.kron(Ix, self.B)
        u = np.zeros((nt, nx, nu))
        p = np.zeros((nt, nx, npp))
        lu = None
        for k in range(nt):
            Kuu = base
            if conv is not None:
                for a in range(conv.k1):
                    for b in range(conv.k2):
                        if conv.w1[k, a] != 0.0:
                            Kuu = Kuu + conv.w1[k, a] * sp.kron(sp.csr_matrix(conv.Hw[a, b]), conv.Nb_ff[b])
            if lu is None or conv is not None:
                K = sp.bmat([[Kuu, Kup], [Kpu, None]]).tocsc()
                lu = spla.splu(K)
            rhs_u = bu[k].ravel().copy()
            if k > 0:
                rhs_u += (sp.kron(Ix, self.Mb) @ u[k - 1].ravel()) / self.tau
            sol = lu.solve(np.concatenate([rhs_u, bp[k].ravel()]))
            u[k] = sol[:nx * nu].reshape(nx, nu)
            p[k] = sol[nx * nu:].reshape(nx, npp)
        return u, p
