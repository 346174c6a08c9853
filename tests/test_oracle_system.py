"""Pins of the oracle's all-at-once operator, right-hand side and solvers:
explicit Kronecker matrices, dense direct solves, physics invariants, the
ideal preconditioner of eq. 5.3 and the full-tensor limit of the low-rank
solver."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import tt
from oracle.solver import lowrank_fgmres, FullOps, solve_tt, solve_full
from oracle.system import Problem
from synthetic_inputs import CONFIGS, random_tt_pair


@pytest.fixture(scope="module")
def tiny():
    return Problem(CONFIGS["tiny"])


def _prior(P, seed=3):
    # a smooth-ish prior velocity/pressure iterate (low rank, small amplitude)
    u, p = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 2), (1, 1), seed)
    return tt.scale(u, 0.3 / tt.tt_norm(u)), tt.scale(p, 0.1 / tt.tt_norm(p))


@pytest.mark.parametrize("name", ["tiny", "tinykl"])
def test_apply_matches_explicit_kron(name):
    P = Problem(CONFIGS[name])
    x = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 3), (2, 2), 0)
    K = P.explicit()
    ref = K @ tt.pair_full(x)
    assert np.abs(tt.pair_full(P.apply(x)) - ref).max() <= 1e-13 * np.abs(ref).max()
    yu, yp = P.apply_full(tt.full(x[0]), tt.full(x[1]))
    assert np.abs(np.concatenate([yu.ravel(), yp.ravel()]) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_apply_with_convection_matches_explicit(tiny):
    P = tiny
    conv = P.convection(_prior(P), 1e-3)
    x = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 3), (2, 2), 1)
    K = P.explicit(conv)
    ref = K @ tt.pair_full(x)
    got = tt.pair_full(P.apply(x, conv))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    yu, yp = P.apply_full(tt.full(x[0]), tt.full(x[1]), conv)
    assert np.abs(np.concatenate([yu.ravel(), yp.ravel()]) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["tiny", "tinykl"])
def test_time_stepping_equals_dense_solve(name):
    P = Problem(CONFIGS[name])
    b = P.rhs()
    K = P.explicit()
    zd = spla.spsolve(K, tt.pair_full(b))
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
    z = np.concatenate([u.ravel(), p.ravel()])
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)
    conv = P.convection(_prior(P), 1e-3)
    b2 = P.rhs(_prior(P))
    K2 = P.explicit(conv)
    zd2 = spla.spsolve(K2, tt.pair_full(b2))
    u2, p2 = P.solve_direct(tt.full(b2[0]), tt.full(b2[1]), conv)
    assert np.linalg.norm(np.concatenate([u2.ravel(), p2.ravel()]) - zd2) <= 1e-11 * np.linalg.norm(zd2)


def test_rhs_is_lifted_dirichlet_data(tiny):
    # f = -L_{free,Dirichlet} g a(t): check against the all-node operator applied
    # to the lift vector, assembled independently with scipy.sparse.kron.
    P = tiny
    b = P.rhs()
    assert tt.ranks(b[0]) == (2, 2) and tt.ranks(b[1]) == (1, 1)
    nt, nx = P.nt, P.n_xi
    e1 = np.zeros(nx)
    e1[0] = 1.0
    lift = np.kron(np.kron(P.ramp, e1), P.g_all)
    Kfa = sp.kron(sp.kron((P.It - P.Ct) / P.tau, sp.identity(nx)), P.Mb_fall) \
        + sp.kron(sp.kron(P.It, sp.csr_matrix(P.Gnu)), P.Ab_fall)
    Kpa = sp.kron(sp.identity(nt * nx), P.B_all)
    ref = -np.concatenate([Kfa @ lift, Kpa @ lift])
    assert np.abs(tt.pair_full(b) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_physics_divergence_free_and_outflow_flux():
    # With zero initial data the exact discrete solution is discretely
    # divergence-free (B u_full = 0 for each (t_k, psi_r)), and since q = 1 is in
    # the pressure space the net boundary flux is zero: outflow flux at x1 = L
    # equals the inflow flux (2/3)(1 - e^{-10 t_k}) in the psi_1 mode, 0 otherwise.
    cfg = dict(CONFIGS["tiny2"])
    P = Problem(cfg)
    b = P.rhs()
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
    nall = P.n_all
    f = P.mesh.free
    ufull = np.zeros((P.nt, P.n_xi, 2 * nall))
    ufull[:, :, f] = u[:, :, :P.n_s]
    ufull[:, :, nall + f] = u[:, :, P.n_s:]
    gall = P.g_all
    ufull += P.ramp[:, None, None] * np.eye(P.n_xi)[0][None, :, None] * gall[None, None, :]
    div = np.einsum("px,tkx->tkp", P.B_all.toarray(), ufull)
    assert np.abs(div).max() < 1e-10
    # flux through x1 = L: integrate u1 along the outflow edge with the Q2 trace
    x1, x2 = P.mesh.coords[:, 0], P.mesh.coords[:, 1]
    out = np.nonzero(np.abs(x1 - cfg["L"]) < 1e-12)[0]
    out = out[np.argsort(x2[out])]
    hh = cfg["h"]
    wts = np.zeros(out.size)      # Simpson weights per element edge (exact for Q2)
    for e in range(0, out.size - 1, 2):
        wts[e:e + 3] += np.array([1, 4, 1]) * hh / 6
    flux = np.einsum("tkx,x->tk", ufull[:, :, out], wts)
    assert np.abs(flux[:, 0] - (2.0 / 3.0) * P.ramp).max() < 1e-10
    assert np.abs(flux[:, 1:]).max() < 1e-10


def test_deterministic_limit():
    # nu_coef = 0: G_nu = nu0 I, so only the psi_1 mode is driven (G_0 = I).
    cfg = dict(CONFIGS["tiny"], nu_coef=0.0)
    P = Problem(cfg)
    b = P.rhs()
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
    assert np.abs(u[:, 1:]).max() < 1e-14 and np.abs(p[:, 1:]).max() < 1e-14
    assert np.abs(u[:, 0]).max() > 1e-2


def test_time_inverse_is_prefix_sum():
    P = Problem(CONFIGS["tiny"])
    IC = (P.It - P.Ct).toarray()
    assert np.allclose(np.linalg.inv(IC), np.tril(np.ones((P.nt, P.nt))))


def test_commutator_identity_eq_5_15(tiny):
    # M_p^-1 B M^-1 C - M_p^-1 C_p M_p^-1 B = 0 exactly (eq. 5.15)
    P = tiny
    nx = P.n_xi
    Mi = sp.kron(sp.kron(P.It, sp.identity(nx)), sp.linalg.inv(P.Mb.tocsc()))
    Mpi = sp.kron(sp.kron(P.It, sp.identity(nx)), sp.linalg.inv(P.Mp.tocsc()))
    Bb = sp.kron(sp.identity(P.nt * nx), P.B)
    Cb = -sp.kron(sp.kron(P.Ct, sp.identity(nx)), P.Mb) / P.tau
    Cp = -sp.kron(sp.kron(P.Ct, sp.identity(nx)), P.Mp) / P.tau
    D = Mpi @ Bb @ Mi @ Cb - Mpi @ Cp @ Mpi @ Bb
    assert abs(D).max() < 1e-10


def test_ideal_preconditioner_two_iterations(tiny):
    # eq. 5.2-5.3: with exact (F+C)^-1 and exact Schur complement, right
    # preconditioned GMRES converges in two iterations.
    P = tiny
    K = P.explicit().toarray()
    nu_tot = P.nt * P.n_xi * P.n_u
    F = K[:nu_tot, :nu_tot]
    Bt = K[:nu_tot, nu_tot:]
    Bm = K[nu_tot:, :nu_tot]
    Finv = np.linalg.inv(F)
    S = Bm @ Finv @ Bt
    Sinv = np.linalg.inv(S)

    def prec(y):
        ph = -Sinv @ y[nu_tot:]
        return np.concatenate([Finv @ (y[:nu_tot] - Bt @ ph), ph])

    ops = FullOps(P)
    b = tt.pair_full(P.rhs())
    z, k, res, bn = lowrank_fgmres(ops, lambda x: K @ x, prec, b, 1e-10, 0.0, 10)
    assert k == 2
    assert np.linalg.norm(K @ z - b) <= 1e-10 * bn


def test_tt_limit_reproduces_full_tensor_fgmres(tiny):
    # eps -> 0: the TT iterates reproduce the full-tensor flexible GMRES
    # (same Hessenberg entries, same iteration count).
    P = tiny
    b = P.rhs()
    rec_full, rec_tt = [], []
    solve_full(P, tt.full(b[0]), tt.full(b[1]), tol=1e-6, record=rec_full)
    from oracle.solver import TTOps, MeanLSC
    ops = TTOps(P)
    prec = MeanLSC(P, None, "tt", 1e-1, 1e-14, 20, 1e-14)
    lowrank_fgmres(ops, ops.apply, prec.apply_tt, b, 1e-6, 1e-14, 60, rec_tt)
    assert len(rec_full) == len(rec_tt)
    Hf, Ht = rec_full[-1]["H"], rec_tt[-1]["H"]
    assert np.abs(Hf - Ht).max() <= 1e-9 * np.abs(Hf).max()


def test_lowrank_solve_reaches_target_and_exact_solution(tiny):
    P = tiny
    b = P.rhs()
    z, st = solve_tt(P, b, tol=1e-10)
    assert st["rel"][-1] <= 1e-10
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
    zd = np.concatenate([u.ravel(), p.ravel()])
    assert np.linalg.norm(tt.pair_full(z) - zd) <= 1e-8 * np.linalg.norm(zd)


def test_lowrank_solve_with_convection(tiny):
    P = tiny
    prior = _prior(P)
    conv = P.convection(prior, 1e-3)
    b = P.rhs(prior)
    z, st = solve_tt(P, b, conv, tol=1e-10)
    assert st["rel"][-1] <= 1e-10
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]), conv)
    zd = np.concatenate([u.ravel(), p.ravel()])
    assert np.linalg.norm(tt.pair_full(z) - zd) <= 1e-8 * np.linalg.norm(zd)


def _steady_stokes(P, nu):
    """Steady Stokes with viscosity nu on the same mesh: nu A u + B^T p = -nu
    A_fD g, B u = -B_D g (the time-independent problem, built here directly)."""
    Kuu = nu * P.Ab
    K = sp.bmat([[Kuu, P.Bt], [P.B, None]]).tocsc()
    rhs = -np.concatenate([nu * (P.Ab_fall @ P.g_all), P.B_all @ P.g_all])
    sol = spla.spsolve(K, rhs)
    return sol[:P.n_u], sol[P.n_u:]


def test_long_time_limit_is_steady_stokes():
    # Backward Euler with a constant inflow converges to the steady problem:
    # pins the sign and scaling of the time shift C and of tau^-1 M.
    cfg = dict(CONFIGS["tiny"], nu0=1.0, nu_coef=0.0, ramp=1e9, tau=0.5, nt=60)
    P = Problem(cfg)
    b = P.rhs()
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
    us, ps = _steady_stokes(P, 1.0)
    assert np.linalg.norm(u[-1, 0] - us) <= 1e-10 * np.linalg.norm(us)
    assert np.linalg.norm(p[-1, 0] - ps) <= 1e-9 * np.linalg.norm(ps)


def test_stochastic_galerkin_mean_matches_quadrature():
    # One random variable, high chaos degree: the Galerkin mean of the final
    # time step equals the U[-1,1] expectation of deterministic solves with
    # nu(xi) = nu0 (1 + c xi), evaluated by Gauss-Legendre quadrature.
    from scipy.special import roots_legendre
    nu0, c = 0.5, 0.4
    cfg = dict(CONFIGS["tiny"], m=1, p=10, nu0=nu0, nu_coef=c, nt=3, tau=0.2)
    P = Problem(cfg)
    b = P.rhs()
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
    xq, wq = roots_legendre(16)
    mean = np.zeros(P.n_u)
    for x, w in zip(xq, wq):
        Pd = Problem(dict(cfg, m=1, p=0, nu0=nu0 * (1 + c * x), nu_coef=0.0))
        bd = Pd.rhs()
        ud, _ = Pd.solve_direct(tt.full(bd[0]), tt.full(bd[1]))
        mean += 0.5 * w * ud[-1, 0]
    assert np.linalg.norm(u[-1, 0] - mean) <= 1e-9 * np.linalg.norm(mean)


def test_kl_stochastic_galerkin_mean_matches_quadrature():
    # One KL mode, high chaos degree: the Galerkin mean of the final time step
    # equals the expectation over xi ~ U[-sqrt 3, sqrt 3] of deterministic
    # solves with nu(x, xi) = nu0 (1 + sigma sqrt(beta_1) a_1(x) xi)
    # (Gauss-Legendre quadrature in xi / sqrt 3).  Pins the sqrt 3 scaling of
    # G_1 and the assembly of A_1 = nu0 sigma sqrt(beta_1) A(a_1).
    from scipy.special import roots_legendre
    from oracle import mesh as fem
    nu0, sigma = 0.5, 0.2     # nu(x, xi) stays within about 30 % of nu0
    cfg = dict(CONFIGS["tinykl"], m=1, p=10, nu0=nu0, nu_coef=sigma, nt=3, tau=0.2)
    P = Problem(cfg)
    b = P.rhs()
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
    _, A, _, _, _ = fem.assemble(P.mesh)
    A1 = fem.stiffness_weighted(P.mesh, P.kl_modes[0])
    f = P.mesh.free
    xq, wq = roots_legendre(16)
    mean = np.zeros(P.n_u)
    for x, w in zip(xq, wq):
        xi = np.sqrt(3.0) * x
        Pd = Problem(dict(cfg, m=1, p=0, viscosity="power", nu_coef=0.0))
        Ad = nu0 * A + nu0 * sigma * np.sqrt(P.kl_beta[0]) * xi * A1
        Af, Afa = Ad[f][:, f].tocsr(), Ad[f]
        Pd.visc = [(np.eye(1), sp.block_diag([Af, Af]).tocsr(), sp.block_diag([Afa, Afa]).tocsr())]
        bd = Pd.rhs()
        ud, _ = Pd.solve_direct(tt.full(bd[0]), tt.full(bd[1]))
        mean += 0.5 * w * ud[-1, 0]
    assert np.linalg.norm(u[-1, 0] - mean) <= 1e-9 * np.linalg.norm(mean)


def test_residual_entries_match_full_residual():
    # the entry-by-entry residual (used at sizes where no full tensor fits
    # the oracle) equals the full-tensor residual b - L x at every entry
    P = Problem(CONFIGS["tiny"])
    x = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 4), (2, 3), 5)
    b = P.rhs()
    yu, yp = P.apply_full(tt.full(x[0]), tt.full(x[1]))
    ru, rp = tt.full(b[0]) - yu, tt.full(b[1]) - yp
    g = np.random.default_rng(0)
    for which, full, n in (("u", ru, P.n_u), ("p", rp, P.n_p)):
        t, i, j = g.integers(0, P.nt, 60), g.integers(0, P.n_xi, 60), g.integers(0, n, 60)
        e = P.residual_entries(b, x, which, t, i, j)
        assert np.abs(e - full[t, i, j]).max() <= 1e-13 * np.abs(full).max()
    # a Picard system: the convection term of eq. 4.12 entry by entry
    prior = _prior(P)
    conv = P.convection(prior, 1e-3)
    b2 = P.rhs(prior)
    yu, yp = P.apply_full(tt.full(x[0]), tt.full(x[1]), conv)
    ru, rp = tt.full(b2[0]) - yu, tt.full(b2[1]) - yp
    for which, full, n in (("u", ru, P.n_u), ("p", rp, P.n_p)):
        t, i, j = g.integers(0, P.nt, 60), g.integers(0, P.n_xi, 60), g.integers(0, n, 60)
        e = P.residual_entries(b2, x, which, t, i, j, conv=conv)
        assert np.abs(e - full[t, i, j]).max() <= 1e-13 * np.abs(full).max()


def test_picard_direct_contracts(tiny):
    # Picard's method (Alg. 3.1) at Reynolds ~100 converges linearly: the
    # nonlinear residual drops by a steady factor at every step
    from oracle.solver import picard_direct
    its, res = picard_direct(tiny, 3)
    assert len(its) == 4 and len(res) == 4
    assert all(res[i + 1] < 0.2 * res[i] for i in range(3))


def test_picard_direct_iterates_solve_the_frozen_wind_equations(tiny):
    # Alg. 3.1 in residual form (eq. 3.14-3.15) with exact solves is the
    # fixed-point iteration whose iterate i+1 solves the Oseen equations with
    # the wind of iterate i frozen: tau^-1 (I - C) M u + A u + N(w_i) u +
    # B^T p = 0 on the free velocity rows and B u = 0, for u the whole
    # velocity (Dirichlet lift included).  The nonlinear residual of iterate
    # i+1 plus N(w_{i+1}) w_{i+1} minus N(w_i) w_{i+1} is that Oseen residual
    # and must vanish; an update added with the wrong sign, a residual taken
    # at the wrong iterate or an update solved with the wrong wind fails it.
    from oracle.solver import picard_direct
    from oracle.system import Convection
    P = tiny
    its, res = picard_direct(P, 2)
    f = P.rhs(None)
    fn = np.sqrt(tt.tt_dot(f[0], f[0]) + tt.tt_dot(f[1], f[1]))
    priors = [(tt.tt_svd(U, 1e-15), tt.tt_svd(Pp, 1e-15)) for U, Pp in its]
    for i in range(2):
        wi, wj = P.wind(priors[i]), P.wind(priors[i + 1])
        ru, rp = P.residual_tt(priors[i + 1])
        oseen = (tt.full(ru) + tt.full(Convection(P, wj).ttm_apply(wj, which="fall"))
                 - tt.full(Convection(P, wi).ttm_apply(wj, which="fall")))
        assert np.linalg.norm(oseen) <= 1e-10 * fn
        assert np.linalg.norm(tt.full(rp)) <= 1e-10 * fn
        # the nonlinear residual itself does not vanish before convergence
        assert np.linalg.norm(tt.full(ru)) >= 1e-6 * fn


def test_exact_mean_solve_inverts_mean_matrix(tiny):
    # (F_0 + C) applied to the exact mean solve gives back the right-hand side
    from oracle.solver import MeanLSC
    P = tiny
    prec = MeanLSC(P, None, "full")
    g = np.random.default_rng(3)
    Y = g.standard_normal((P.nt, P.n_xi, P.n_u))
    V = prec.mean_solve_exact_full(Y)
    back = prec._mean_apply_full(V)
    assert np.linalg.norm(back - Y) <= 1e-12 * np.linalg.norm(Y)


def test_minv_inverts_the_mean_based_matrix(tiny):
    # eq. 5.23: M = (I - C) (x) I (x) F_avg with F_avg = tau^-1 M + nu_0 A +
    # N(w_avg) on both velocity components; the prefix-sum / spatial-solve
    # form of M^-1 must invert the explicit Kronecker matrix, with and
    # without convection (w_avg = time mean of the psi_1 mode of w~)
    from oracle.solver import MeanLSC
    P = tiny
    prior = _prior(P)
    for conv in (None, P.convection(prior, 1e-12)):
        Fs = P.M / P.tau + P.cfg["nu0"] * P.A
        if conv is not None:
            w_avg = (conv.w1 @ conv.w2[:, 0, :]).mean(axis=0)
            for b in range(conv.k2):
                Fs = Fs + w_avg[b] * conv.N_ff[b]
        Mexp = sp.kron(sp.kron(P.It - P.Ct, sp.identity(P.n_xi)), sp.block_diag([Fs, Fs])).tocsr()
        prec = MeanLSC(P, conv, "tt", velocity="minv")
        y = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 4), (1, 1), 9)[0]
        v = tt.full(prec._Minv_tt(y)).ravel()
        Y = tt.full(y).ravel()
        assert np.linalg.norm(Mexp @ v - Y) <= 1e-12 * np.linalg.norm(Y)


def test_minv_velocity_block_solves_to_target(tiny):
    # FGMRES with M^-1 applied once as the velocity block (a varying, inexact
    # preconditioner is admitted by the flexible method, sec. 4.2) still
    # reaches the exact solution through the refinement cycles
    P = tiny
    b = P.rhs()
    z, st = solve_tt(P, b, tol=1e-10, velocity="minv")
    assert st["rel"][-1] <= 1e-10
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
    zd = np.concatenate([u.ravel(), p.ravel()])
    assert np.linalg.norm(tt.pair_full(z) - zd) <= 1e-8 * np.linalg.norm(zd)


def test_pcd_pressure_operator_matches_explicit_kron(tiny):
    # eq. 5.17: F_p,0 + C_p = tau^-1 (I - C) (x) I (x) M_p + I (x) I (x) nu_0 A_p
    # + sum_b diag(omega_b) (x) I (x) N_p(w3_b), omega_b(t) the psi_1 mode of
    # the wind's time factor (the mean convection of sec. 5.1); the TT form
    # of the preconditioner must equal this Kronecker matrix
    from oracle import mesh as fem
    from oracle.solver import MeanLSC
    P = tiny
    prior = _prior(P)
    conv = P.convection(prior, 1e-12)
    prec = MeanLSC(P, conv, "tt", schur="pcd")
    na = P.mesh.n_all
    Ap = fem.pressure_stiffness(P.mesh)
    K = sp.kron(sp.kron((P.It - P.Ct) / P.tau, sp.identity(P.n_xi)), P.Mp) \
        + sp.kron(sp.identity(P.nt * P.n_xi), P.cfg["nu0"] * Ap)
    omega = conv.w1 @ conv.w2[:, 0, :]
    for b in range(conv.k2):
        Npb = fem.pressure_convection(P.mesh, conv.w3[b, :na], conv.w3[b, na:])
        K = K + sp.kron(sp.kron(sp.diags(omega[:, b]), sp.identity(P.n_xi)), Npb)
    q = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (1, 1), (2, 3), 4)[1]
    got = tt.full(prec._pressure_mean_apply_tt(q)).ravel()
    want = K @ tt.full(q).ravel()
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)
    # the full-tensor form is the same operator
    full = prec._pressure_mean_apply_full(tt.full(q)).ravel()
    assert np.linalg.norm(full - want) <= 1e-13 * np.linalg.norm(want)


def test_pcd_preconditioner_tt_equals_full_and_solves(tiny):
    # the TT form of the PCD preconditioner equals its full-tensor form
    # (eps -> 0), and FGMRES with it reaches the exact solution
    from oracle.solver import MeanLSC
    P = tiny
    prior = _prior(P)
    conv = P.convection(prior, 1e-3)
    y = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 3), (2, 2), 5)
    tt_prec = MeanLSC(P, conv, "tt", inner_tol=1e-13, inner_eps=1e-14, inner_maxit=60, eps=1e-14, schur="pcd")
    _, ph_tt = tt_prec.apply_tt(y)
    full_prec = MeanLSC(P, conv, "full", schur="pcd")
    ph_full = -full_prec.schur_inv_full(tt.full(y[1]))
    assert np.linalg.norm(tt.full(ph_tt) - ph_full) <= 1e-10 * np.linalg.norm(ph_full)
    b = P.rhs(prior)
    z, st = solve_tt(P, b, conv, tol=1e-10, schur="pcd")
    assert st["rel"][-1] <= 1e-10
    u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]), conv)
    zd = np.concatenate([u.ravel(), p.ravel()])
    assert np.linalg.norm(tt.pair_full(z) - zd) <= 1e-8 * np.linalg.norm(zd)


def _psi_multi(idx, xi):
    # orthonormal multivariate Legendre polynomial for U[-1,1]^m (scipy's
    # Legendre evaluation, independent of oracle.gpc)
    from scipy.special import eval_legendre
    v = 1.0
    for k, n in enumerate(idx):
        v = v * np.sqrt(2 * n + 1) * eval_legendre(n, xi[k])
    return v


def test_sg_convection_matches_quadrature():
    # eq. 4.12: the stochastic Galerkin convection of a wind w(t, xi, x) =
    # sum_l w_l(t, x) psi_l(xi) is the Galerkin projection
    #     out_r(t) = E[ psi_r(xi) N(w(t, xi)) u(t, xi) ],  u = sum_s u_s psi_s,
    # evaluated here by tensor Gauss-Legendre quadrature of deterministic
    # convection matrices assembled at each quadrature point (m = 2, p = 2).
    from scipy.special import roots_legendre
    from oracle import mesh as fem
    cfg = dict(CONFIGS["tiny"], m=2, p=2, nt=2)
    P = Problem(cfg)
    g = np.random.default_rng(21)
    na, f = P.n_all, P.mesh.free
    # an all-node wind TT of ranks (2, 3) and a free-dof velocity tensor
    W1 = g.standard_normal((P.nt, 2))
    W2 = g.standard_normal((2, P.n_xi, 3))
    W3 = g.standard_normal((3, 2 * na))
    conv = __import__("oracle.system", fromlist=["Convection"]).Convection(P, (W1, W2, W3))
    U = g.standard_normal((P.nt, P.n_xi, P.n_u))
    got = conv.full_apply(U)
    Wfull = np.einsum("ta,alb,bx->tlx", W1, W2, W3)          # (nt, n_xi, 2 n_all)
    xq, wq = roots_legendre(5)                               # exact for degree <= 9 per variable
    want = np.zeros_like(U)
    for q1, w1q in zip(xq, wq):
        for q2, w2q in zip(xq, wq):
            xi = (q1, q2)
            wt = 0.25 * w1q * w2q                            # U[-1,1]^2 density
            psi = np.array([_psi_multi(ix, xi) for ix in P.idx])
            for t in range(P.nt):
                w = psi @ Wfull[t]                           # wind at this xi
                N = fem.convection(P.mesh, w[:na], w[na:])[f][:, f]
                u = psi @ U[t]
                Nu = np.concatenate([N @ u[:P.n_s], N @ u[P.n_s:]])
                want[t] += wt * psi[:, None] * Nu[None, :]
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # the mean convection of eq. 5.21 (psi_1 mode of the wind, identity in
    # the chaos mode) is N(E[w]) applied to every chaos coefficient
    got0 = conv.full_apply(U, mean=True)
    want0 = np.zeros_like(U)
    for t in range(P.nt):
        N = fem.convection(P.mesh, Wfull[t, 0, :na], Wfull[t, 0, na:])[f][:, f]
        for r in range(P.n_xi):
            want0[t, r] = np.concatenate([N @ U[t, r, :P.n_s], N @ U[t, r, P.n_s:]])
    assert np.abs(got0 - want0).max() <= 1e-12 * np.abs(want0).max()


def test_meanlsc_block_code_with_exact_pieces_converges_in_two(tiny):
    # eq. 5.2-5.3 through MeanLSC's own block code: with the exact Schur
    # complement S = B (F + C)^-1 B^T and the exact (F + C)^-1 swapped in by
    # its hooks, flexible GMRES converges in two iterations.  A dropped
    # coupling B^T p^ or a transposed piece breaks this (S is not symmetric:
    # F + C is block lower-bidiagonal in time).  The sign and scale of the
    # Schur block are not fixed by it (block-triangular forms with +S or
    # -S both give two iterations).
    from oracle.solver import MeanLSC
    P = tiny
    K = P.explicit().toarray()
    nu_tot = P.nt * P.n_xi * P.n_u
    F, Bt, Bm = K[:nu_tot, :nu_tot], K[:nu_tot, nu_tot:], K[nu_tot:, :nu_tot]
    Finv = np.linalg.inv(F)
    Sinv = np.linalg.inv(Bm @ Finv @ Bt)
    shp_u, shp_p = (P.nt, P.n_xi, P.n_u), (P.nt, P.n_xi, P.n_p)
    prec = MeanLSC(P, None, "full", schur_inv=lambda Y: (Sinv @ Y.ravel()).reshape(shp_p),
                   velocity_inv=lambda Y: (Finv @ Y.ravel()).reshape(shp_u))
    ops = FullOps(P)

    def pc(v):
        u, p = ops.split(v)
        return ops.join(*prec.apply_full_exact(u, p))

    b = tt.pair_full(P.rhs())
    z, k, res, bn = lowrank_fgmres(ops, lambda x: K @ x, pc, b, 1e-10, 0.0, 10)
    assert k == 2
    assert np.linalg.norm(K @ z - b) <= 1e-10 * bn
    # a transposed Schur inverse loses the two-step convergence
    bad = MeanLSC(P, None, "full", schur_inv=lambda Y: (Sinv.T @ Y.ravel()).reshape(shp_p),
                  velocity_inv=lambda Y: (Finv @ Y.ravel()).reshape(shp_u))

    def pc_bad(v):
        u, p = ops.split(v)
        return ops.join(*bad.apply_full_exact(u, p))

    _, k_bad, _, _ = lowrank_fgmres(ops, lambda x: K @ x, pc_bad, b, 1e-10, 0.0, 10)
    assert k_bad > 2


def test_lsc_is_exact_for_a_diagonal_velocity_operator(tiny):
    # eq. 5.19: when the velocity operator is alpha M* (a multiple of the
    # diagonal mass used inside the LSC formula), X (B M*^-1 F M*^-1 B^T)^-1 X
    # with X = B M*^-1 B^T equals the exact Schur complement B F^-1 B^T =
    # X / alpha.  Pins the composition and placement of M*^-1 in MeanLSC.
    from oracle.solver import MeanLSC
    P = tiny
    alpha = 3.7
    Ms = P.Mstar
    prec = MeanLSC(P, None, "full", mean_apply=lambda U: alpha * Ms[None, None, :] * U)
    g = np.random.default_rng(5)
    Yp = g.standard_normal((P.nt, P.n_xi, P.n_p))
    got = prec.schur_inv_full(Yp)
    S = (P.B @ sp.diags(1.0 / (alpha * Ms)) @ P.Bt).toarray()
    want = np.linalg.solve(S, Yp.reshape(-1, P.n_p).T).T.reshape(Yp.shape)
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
