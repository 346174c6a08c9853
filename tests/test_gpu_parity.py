"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs.  Tolerances: FP64 kernels without truncation agree to
1e-12..1e-13 relative; truncated results are compared through what is unique
(full values, norms, residuals, exact solutions), never through cores."""
import numpy as np
import pytest

from oracle import tt
from oracle.solver import MeanLSC
from oracle.system import Problem
from synthetic_inputs import CONFIGS, random_tt_cores, random_tt_pair

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def sg():
    from paper_1906_06785_amd import sgtt
    return sgtt


@pytest.fixture(scope="module")
def ctx(sg):
    return sg.Context(0)


@pytest.fixture(scope="module")
def tiny(sg, ctx):
    P = Problem(CONFIGS["tiny"])
    S = sg.System(ctx, CONFIGS["tiny"])
    return P, S


@pytest.fixture(scope="module")
def c1(sg, ctx):
    P = Problem(CONFIGS["C1"])
    S = sg.System(ctx, CONFIGS["C1"])
    return P, S


def _pair_buf(S, pair, cap1=32, cap2=128):
    return S.pair(cap1, cap2).set(pair)


def test_dot_and_expand(sg, ctx, tiny):
    P, S = tiny
    _flush("dot/expand tiny")
    x = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 7), (2, 5), 1)
    y = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 9), (3, 4), 2)
    bx, by = _pair_buf(S, x), _pair_buf(S, y)
    ref = tt.pair_dot(x, y)
    got = ctx.dot(bx, by)
    assert abs(got - ref) <= 1e-12 * abs(ref)
    full = ctx.expand(bx.u).cpu().numpy()
    assert np.abs(full - tt.full(x[0])).max() <= 1e-13 * np.abs(full).max()


def test_axpby_is_the_exact_sum(sg, ctx, tiny):
    # sec. 4.1: a TT sum by core concatenation is exact and its ranks add
    P, S = tiny
    _flush("axpby tiny")
    x = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 7), (2, 5), 3)
    y = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 9), (3, 4), 4)
    bx, by = _pair_buf(S, x), _pair_buf(S, y)
    ctx.axpby(0.75, bx, -1.5, by)
    assert by.ranks == ((3 + 2, 7 + 9), (2 + 3, 5 + 4))
    for got, xc, yc in ((by.u, x[0], y[0]), (by.p, x[1], y[1])):
        want = 0.75 * tt.full(xc) - 1.5 * tt.full(yc)
        full = ctx.expand(got).cpu().numpy()
        assert np.abs(full - want).max() <= 1e-13 * np.abs(want).max()
    # a result above y's capacity is refused and y is left as it was
    small = S.pair(4, 12).set(y)
    before = [ctx.expand(t).cpu().numpy() for t in (small.u, small.p)]
    with pytest.raises(sg.SgttError) as ei:
        ctx.axpby(1.0, bx, 1.0, small)
    assert ei.value.code == -4
    assert small.ranks == ((2, 9), (3, 4))
    after = [ctx.expand(t).cpu().numpy() for t in (small.u, small.p)]
    assert all(np.array_equal(a, b) for a, b in zip(before, after))


def test_device_ranks_follow_every_output(sg, ctx, tiny):
    # sgtt_tt.d_ranks: every call that writes a TT also stores its live ranks
    # in device memory, ordered on the stream after the cores
    import ctypes
    P, S = tiny
    _flush("device ranks tiny")

    def dev(t):
        return tuple(t.d_ranks.cpu().tolist())

    x = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 7), (2, 5), 5)
    y = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 9), (3, 4), 6)
    bx, by = _pair_buf(S, x), _pair_buf(S, y)
    ctx.axpby(1.0, bx, 2.0, by)
    assert (dev(by.u), dev(by.p)) == ((5, 16), (5, 9)) == by.ranks
    ctx.round(by.u, 1e-3)
    assert dev(by.u) == (by.u.r1, by.u.r2)
    assert by.u.r2 < 16
    b = S.rhs()
    assert (dev(b.u), dev(b.p)) == b.ranks
    z, st, rc = S.solve(b, tol=1e-10)
    assert rc == 0 and st["rel_residual"] <= 1e-10
    assert (dev(z.u), dev(z.p)) == z.ranks
    # without a device copy (NULL) the output is written as before
    bz = _pair_buf(S, x)
    s = bz.struct()
    s.u.d_ranks = None
    s.p.d_ranks = None
    ctx.check(sg._lib.sgtt_axpby(ctx._c, 1.0, ctypes.byref(bx.struct()), 1.0, ctypes.byref(s)))
    assert (s.u.r1, s.u.r2, s.p.r1, s.p.r2) == (6, 14, 4, 10)
    assert dev(bz.u) == (0, 0)
    # a TT of another element type is refused and nothing is written
    s = by.struct()
    s.u.dtype = 1
    before = dev(by.u)
    with pytest.raises(sg.SgttError) as ei:
        ctx.check(sg._lib.sgtt_axpby(ctx._c, 1.0, ctypes.byref(bx.struct()), 1.0, ctypes.byref(s)))
    assert ei.value.code == -1
    assert (s.u.r1, s.u.r2) == (by.u.r1, by.u.r2) and dev(by.u) == before
    # an output pair whose pressure TT has another element type: neither TT
    # of the pair is written
    bo = S.pair(16, 128)
    s = bo.struct()
    s.p.dtype = 1
    with pytest.raises(sg.SgttError) as ei:
        ctx.check(sg._lib.sgtt_rhs(S._s, ctypes.byref(s)))
    assert ei.value.code == -1
    assert (s.u.r1, s.u.r2) == (1, 1) and dev(bo.u) == (0, 0)
    # a device copy of the ranks in plain host memory is refused before any
    # core is written
    host_ranks = (ctypes.c_int * 2)(-1, -1)
    s = by.struct()
    s.u.d_ranks = ctypes.cast(host_ranks, ctypes.c_void_p)
    r_before = (by.u.r1, by.u.r2)
    with pytest.raises(sg.SgttError) as ei:
        ctx.check(sg._lib.sgtt_axpby(ctx._c, 1.0, ctypes.byref(bx.struct()), 1.0, ctypes.byref(s)))
    assert ei.value.code == -1
    assert (s.u.r1, s.u.r2) == r_before and list(host_ranks) == [-1, -1]
    # so is a core in plain host memory, as an input and as an output
    host_core = np.zeros(by.p.n3 * by.p.cap2)
    for which in ("x", "y"):
        sx, sy = bx.struct(), by.struct()
        (sx if which == "x" else sy).p.core3 = host_core.ctypes.data
        with pytest.raises(sg.SgttError) as ei:
            ctx.check(sg._lib.sgtt_axpby(ctx._c, 1.0, ctypes.byref(sx), 1.0, ctypes.byref(sy)))
        assert ei.value.code == -1
    assert not host_core.any()


@pytest.mark.parametrize("n,ranks,eps", [((10, 6, 2992), (8, 24), 1e-3), ((10, 6, 2992), (8, 24), 1e-6),
                                         ((128, 35, 3000), (12, 40), 1e-6), ((7, 5, 137), (5, 9), 0.3)])
def test_round_error_bound_and_ranks(sg, ctx, n, ranks, eps):
    _flush(f"round n={n} ranks={ranks} eps={eps}")
    G = random_tt_cores(*n, *ranks, seed=11, decay=0.35)
    X = tt.full(G)
    buf = sg.TTBuf(*n, 96, 96).set_cores(*G)
    ctx.round(buf, eps)
    Y = ctx.expand(buf).cpu().numpy()
    nrm = np.linalg.norm(X)
    err = np.linalg.norm(Y - X)
    # eq. 4.6, up to the accuracy of FP64 Gram matrices (~1e-8 relative)
    assert err <= eps * nrm * (1 + 1e-6) + 1e-8 * nrm
    ref = tt.tt_round(G, eps)
    r_ref = tt.ranks(ref)
    assert abs(buf.r1 - r_ref[0]) <= 1 and abs(buf.r2 - r_ref[1]) <= 1
    # output is left-orthonormal: ||z|| = ||core3||
    G1, G2, G3 = buf.cores()
    assert np.abs(G1.T @ G1 - np.eye(buf.r1)).max() < 1e-10
    L = G2.reshape(-1, buf.r2)
    assert np.abs(L.T @ L - np.eye(buf.r2)).max() < 1e-10


@pytest.mark.parametrize("n1,r2,eps", [(12, 480, 1e-2), (12, 480, 1e-3), (20, 300, 1e-3)])
def test_round_large_rank_second_bond(sg, ctx, n1, r2, eps):
    # second-bond rank above 96: blocked pivoted Cholesky + skeleton path
    # (n1 = 20 makes the second Gram larger than 512, which takes that path
    # directly).  The error bound of eq. 4.6 still holds; the rank is close
    # to (and not below) the optimal one of the SVD truncation.
    _flush(f"round large rank n1={n1} r2={r2} eps={eps}")
    G = random_tt_cores(n1, 40, 3000, n1, r2, seed=12)
    G = (G[0], G[1], G[2] * np.exp(-0.03 * np.arange(r2))[:, None])
    X = tt.full(G)
    buf = sg.TTBuf(n1, 40, 3000, n1 + 4, r2).set_cores(*G)
    ctx.round(buf, eps)
    Y = ctx.expand(buf).cpu().numpy()
    nrm = np.linalg.norm(X)
    err = np.linalg.norm(Y - X)
    assert err <= eps * nrm * (1 + 1e-6) + 1e-8 * nrm
    r_ref = tt.ranks(tt.tt_round(G, eps))
    assert r_ref[1] > 96
    assert buf.r2 >= r_ref[1] - 1 and buf.r2 <= 1.5 * r_ref[1] + 4
    assert abs(buf.r1 - r_ref[0]) <= 1


@pytest.mark.parametrize("n1,r1", [(40, 40), (80, 80), (128, 128)])
def test_round_blocked_panel_sizes(sg, ctx, n1, r1):
    # second-bond Grams of order 35 r1 = 1400, 2800 and 4480: the register
    # panels of 16 and 8 pivots and, above order 4096, the 32-pivot panels in
    # global memory; the bound of eq. 4.6 holds on each
    _flush(f"round blocked panels n1={n1}")
    n2, n3, r2, eps = 35, 3000, 160, 1e-3
    G = random_tt_cores(n1, n2, n3, r1, r2, seed=13)
    G = (G[0], G[1], G[2] * np.exp(-0.03 * np.arange(r2))[:, None])
    X = tt.full(G)
    buf = sg.TTBuf(n1, n2, n3, r1 + 4, r2 + 8).set_cores(*G)
    ctx.round(buf, eps)
    Y = ctx.expand(buf).cpu().numpy()
    nrm = np.linalg.norm(X)
    assert np.linalg.norm(Y - X) <= eps * nrm * (1 + 1e-6) + 1e-8 * nrm
    assert 1 <= buf.r2 <= r2


def test_round_sum_cancellation(sg, ctx):
    # x + x - x rounds back to x's ranks and values
    _flush("round cancellation")
    G = random_tt_cores(10, 6, 500, 4, 6, 5)
    buf = sg.TTBuf(10, 6, 500, 32, 32).set_cores(*tt.concat([G, G, G], [1.0, 1.0, -1.0]))
    ctx.round(buf, 1e-10)
    assert (buf.r1, buf.r2) == (4, 6)
    Y = ctx.expand(buf).cpu().numpy()
    assert np.linalg.norm(Y - tt.full(G)) <= 1e-7 * np.linalg.norm(tt.full(G))


def test_round_zero_tt(sg, ctx):
    # the zero vector rounds to ranks (1, 1) and stays exactly zero
    _flush("round zero")
    G = [np.zeros_like(g) for g in random_tt_cores(10, 6, 500, 4, 6, 5)]
    buf = sg.TTBuf(10, 6, 500, 32, 32).set_cores(*G)
    ctx.round(buf, 1e-6)
    assert (buf.r1, buf.r2) == (1, 1)
    assert not np.any(ctx.expand(buf).cpu().numpy())


def test_round_difference_cancels(sg, ctx):
    # x - x: every direction cancels up to the rounding of the Gram matrices
    _flush("round x - x")
    G = random_tt_cores(10, 6, 500, 4, 6, 5)
    buf = sg.TTBuf(10, 6, 500, 32, 32).set_cores(*tt.concat([G, G], [1.0, -1.0]))
    ctx.round(buf, 1e-8)
    assert buf.r1 <= 8 and buf.r2 <= 12
    Y = ctx.expand(buf).cpu().numpy()
    assert np.linalg.norm(Y) <= 1e-6 * np.linalg.norm(tt.full(G))


def test_profiler_class_mask(sg, ctx, tiny):
    # events only for the selected kernel classes; all classes otherwise
    P, S = tiny
    _flush("profiler class mask")
    b = S.rhs()
    try:
        ctx.profile(True, classes=["k_bcr"])
        S.solve(b, restart=10, relax=1)
        got = ctx.profile_read()
        assert got["k_bcr"]["launches"] > 0 and got["k_bcr"]["seconds"] > 0
        assert all(v["launches"] == 0 and v["seconds"] == 0 for k, v in got.items() if k != "k_bcr")
        ctx.profile(True)
        S.solve(b, restart=10, relax=1)
        got = ctx.profile_read()
        assert got["k_bcr"]["launches"] > 0 and got["k_gemm"]["launches"] > 0
    finally:
        ctx.profile(False)


@pytest.mark.parametrize("which", ["tiny", "c1"])
def test_apply_matches_oracle(sg, ctx, tiny, c1, which):
    P, S = tiny if which == "tiny" else c1
    _flush(f"apply {which}")
    x = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 5), (2, 4), 3)
    bx = _pair_buf(S, x)
    out = S.apply(bx)
    ref = P.apply(x)
    assert out.ranks == (tt.ranks(ref[0]), tt.ranks(ref[1]))
    got = tt.pair_full(out.cores())
    want = tt.pair_full(ref)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_rhs_matches_oracle(sg, ctx, c1):
    P, S = c1
    _flush("rhs c1")
    b = S.rhs()
    ref = P.rhs()
    got = tt.pair_full(b.cores())
    want = tt.pair_full(ref)
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()


def test_hessenberg_lsq(sg, ctx):
    _flush("hessenberg lsq")
    g = np.random.default_rng(4)
    for k in (1, 3, 12, 30):
        H = np.triu(g.standard_normal((k + 1, k)), -1)
        beta = 1.7
        y, res = ctx.hessenberg_lsq(H, beta)
        e1 = np.zeros(k + 1)
        e1[0] = beta
        yr = np.linalg.lstsq(H, e1, rcond=None)[0]
        assert np.abs(y - yr).max() <= 1e-11 * max(1.0, np.abs(yr).max())
        assert abs(res - np.linalg.norm(H @ yr - e1)) <= 1e-11


@pytest.mark.parametrize("which", ["tiny", "c1"])
def test_preconditioner_matches_oracle(sg, ctx, tiny, c1, which):
    # with truncation switched (almost) off, P^-1 r of the library equals the
    # oracle's full-rank TT preconditioner, with the same inner iteration count
    P, S = tiny if which == "tiny" else c1
    _flush(f"precondition {which}")
    r = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 4), (2, 3), 9)
    br = _pair_buf(S, r, 32, 256)
    out, its = S.precondition(br, with_stats=True, eps_krylov=1e-13, inner_eps=1e-13, inner_tol=1e-1)
    prec = MeanLSC(P, None, "tt", 1e-1, 1e-13, 20, 1e-13)
    ref = prec.apply_tt(r)
    got = tt.pair_full(out.cores())
    want = tt.pair_full(ref)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    _flush(f"inner iterations gpu {its} oracle {prec.inner_iters[-1]}, rel difference {err:.2e}")
    assert its == prec.inner_iters[-1]
    # Gram-based rounding resolves singular values down to about sqrt(u)
    # relative, so the inner iterates agree to about 1e-8 per step
    assert err <= 1e-6


@pytest.mark.parametrize("which", ["tiny", "c1"])
def test_pcd_preconditioner_matches_oracle(sg, ctx, tiny, c1, which):
    # the mean-based PCD approximation (eq. 5.17) on the Stokes system
    P, S = tiny if which == "tiny" else c1
    _flush(f"pcd precondition {which}")
    r = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 4), (2, 3), 29)
    out = S.precondition(_pair_buf(S, r, 32, 256), eps_krylov=1e-13, inner_eps=1e-13, inner_tol=1e-1, schur=1)
    ref = MeanLSC(P, None, "tt", 1e-1, 1e-13, 20, 1e-13, schur="pcd").apply_tt(r)
    gp, wp = tt.full(out.cores()[1]), tt.full(ref[1])
    perr = np.linalg.norm(gp - wp) / np.linalg.norm(wp)
    err = np.linalg.norm(tt.pair_full(out.cores()) - tt.pair_full(ref)) / np.linalg.norm(tt.pair_full(ref))
    _flush(f"pressure block difference {perr:.2e}, pair difference {err:.2e}")
    assert perr <= 1e-10
    assert err <= 1e-7


def test_preconditioner_exact_inner_matches_oracle(sg, ctx, c1):
    # velocity block (F_0 + C)^-1 applied exactly (time stepping on the full
    # tensor, BCR spatial solves), compressed at 1e-13: equals the oracle's
    # exact mean-based preconditioner
    P, S = c1
    _flush("precondition exact inner c1")
    r = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 5), (2, 4), 19)
    out = S.precondition(_pair_buf(S, r, 32, 256), eps_krylov=1e-13, inner_eps=1e-13, inner_mode=1)
    ref_u, ref_p = MeanLSC(P, None, "full").apply_full_exact(tt.full(r[0]), tt.full(r[1]))
    want = np.concatenate([ref_u.ravel(), ref_p.ravel()])
    got = tt.pair_full(out.cores())
    # Gram-based TT-SVD of the full result: about sqrt(u) relative accuracy
    assert np.linalg.norm(got - want) <= 1e-8 * np.linalg.norm(want)


@pytest.mark.parametrize("precision", [0, 1])
def test_preconditioner_exact_inner_many_chaos_terms(sg, ctx, precision):
    # n_xi = 70 chaos columns per time step: the mass product of the time
    # stepping forms them in two column chunks (FP64: 64 + 6 with the group's
    # input rows staged once per chunk); FP64 and FP32 mean solves against the
    # oracle's exact preconditioner
    P = Problem(CONFIGS["tinyp4"])
    S = sg.System(ctx, CONFIGS["tinyp4"])
    assert P.n_xi == 70 and S.nxi == 70
    _flush(f"precondition exact inner tinyp4, precision {precision}")
    r = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 5), (2, 3), 29)
    out = S.precondition(_pair_buf(S, r, 32, 512), eps_krylov=1e-13, inner_eps=1e-13, inner_mode=1,
                         precision=precision)
    ref_u, ref_p = MeanLSC(P, None, "full").apply_full_exact(tt.full(r[0]), tt.full(r[1]))
    want = np.concatenate([ref_u.ravel(), ref_p.ravel()])
    got = tt.pair_full(out.cores())
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    _flush(f"error {err:.2e}")
    assert err <= (1e-8 if precision == 0 else 1e-5)


def test_preconditioner_exact_inner_long_horizon(sg, ctx):
    # the same at 32 time steps (C1b), twice: the first call chooses the
    # spatial solve's kernel variants, the second reuses the choice
    P = Problem(CONFIGS["C1b"])
    S = sg.System(ctx, CONFIGS["C1b"])
    r = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 9), (2, 4), 23)
    ref_u, ref_p = MeanLSC(P, None, "full").apply_full_exact(tt.full(r[0]), tt.full(r[1]))
    want = np.concatenate([ref_u.ravel(), ref_p.ravel()])
    for call in range(2):
        _flush(f"precondition exact inner c1b, call {call}")
        out = S.precondition(_pair_buf(S, r, 32, 256), eps_krylov=1e-13, inner_eps=1e-13, inner_mode=1)
        got = tt.pair_full(out.cores())
        # Gram-based TT-SVD of the full result: about sqrt(u) = 1.5e-8 relative
        assert np.linalg.norm(got - want) <= 3e-8 * np.linalg.norm(want)


# Solution-error checks refine past the 1e-8 residual target (exact residual
# 1e-10), so that the error against the exact solution is measured rather than
# bounded by cond(L) * 1e-8, and then require ||x - x*|| <= 1e-8 ||x*||.
TIGHT = dict(tol=1e-10, max_cycles=12)


def _solution_error(P, x, conv=None, b=None):
    bo = P.rhs() if b is None else b
    u, p = P.solve_direct(tt.full(bo[0]), tt.full(bo[1]), conv)
    zd = np.concatenate([u.ravel(), p.ravel()])
    return np.linalg.norm(tt.pair_full(x.cores()) - zd) / np.linalg.norm(zd)


def test_solve_c1_stokes_to_1e8(sg, ctx, c1):
    P, S = c1
    _flush("solve C1 Stokes")
    b = S.rhs()
    x, st, rc = S.solve(b)
    _flush(f"stats {st}")
    assert rc == 0
    assert st["rel_residual"] <= 1e-8
    # the oracle evaluates the residual of the GPU solution independently
    bu, bp = [tt.full(c) for c in b.cores()]
    xu, xp = [tt.full(c) for c in x.cores()]
    yu, yp = P.apply_full(xu, xp)
    rel = np.sqrt(np.sum((bu - yu) ** 2) + np.sum((bp - yp) ** 2)) / np.sqrt(np.sum(bu ** 2) + np.sum(bp ** 2))
    assert rel <= 1e-8
    assert abs(S.residual(b, x) - rel) <= 1e-3 * rel + 1e-14
    # refined past the target: the error against the exact (time-stepping)
    # solution of the oracle
    x2, st2, rc2 = S.solve(b, S.pair(96, 1024), **TIGHT)
    err = _solution_error(P, x2)
    _flush(f"refined: rel residual {st2['rel_residual']:.2e}, solution error {err:.2e}")
    assert rc2 == 0 and st2["rel_residual"] <= 1e-10
    assert err <= 1e-8


def test_solve_c1_outer_iterations_match_oracle(sg, ctx, c1):
    # the same method on both sides (Alg. 4.2 cycles with the mean-based LSC
    # preconditioner and the inner GMRES of eq. 5.22-5.23, restart 30, fixed
    # truncation 1e-6, refinement right-hand sides compressed at 1e-6): the
    # outer iteration counts agree within 2 (ranks may differ by one at a
    # threshold, which can shift an iteration)
    from oracle.solver import solve_tt
    P, S = c1
    _flush("solve c1: outer iterations against the oracle")
    b = S.rhs()
    x, st, rc = S.solve(b, S.pair(96, 1024), restart=30, relax=0, outer_explicit=1, inner_mode=0,
                        cycle_rhs_factor=1e-30)
    _, ost = solve_tt(P, P.rhs())
    _flush(f"outer iterations gpu {st['outer_iters']} ({st['cycles']} cycles), oracle {ost['outer']} "
           f"({ost['cycles']} cycles); inner gpu {st['inner_iters']} oracle {sum(ost['inner'])}")
    assert rc == 0 and st["rel_residual"] <= 1e-8 and ost["rel"][-1] <= 1e-8
    assert abs(st["outer_iters"] - ost["outer"]) <= 2


def test_solve_c1_exact_inner_to_1e8(sg, ctx, c1):
    P, S = c1
    _flush("solve c1 exact inner")
    x, st, rc = S.solve(S.rhs(), S.pair(64, 1024), restart=20, relax=1, inner_mode=1, **TIGHT)
    err = _solution_error(P, x)
    _flush(f"rel residual {st['rel_residual']:.2e}, solution error {err:.2e}")
    assert rc == 0 and st["rel_residual"] <= 1e-10
    assert err <= 1e-8


@pytest.mark.parametrize("precision", [1, 2])
def test_solve_c1_mixed_precision_to_1e8(sg, ctx, c1, precision):
    # FP32 / BF16 matrix-core products inside the preconditioner's inner
    # solve; the FP64 outer refinement still reaches the exact solution
    P, S = c1
    _flush(f"solve c1 precision={precision}")
    b = S.rhs()
    x, st, rc = S.solve(b, S.pair(64, 1024), restart=20, relax=1, precision=precision, **TIGHT)
    err = _solution_error(P, x)
    _flush(f"rel residual {st['rel_residual']:.2e}, solution error {err:.2e}")
    assert rc == 0 and st["rel_residual"] <= 1e-10
    assert err <= 1e-8


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_preconditioner_reduced_precision_meets_inner_tolerance(sg, ctx, c1, precision):
    # In every precision the preconditioner does what eq. 5.2 with eq. 5.22
    # asks, checked with the oracle's operators on full tensors: the pressure
    # part is p^ = -S_LSC^-1 y_p (FP64 in every mode), and the velocity part
    # solves (F_0 + C) v = y_u - B^T p^ to the inner tolerance 1e-1 (plus the
    # inner truncation 1e-3).  Reduced precision only changes which
    # approximate solution the inner GMRES returns.
    P, S = c1
    _flush(f"precondition c1 precision={precision}")
    r = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 4), (2, 3), 9)
    out = S.precondition(_pair_buf(S, r, 32, 256), inner_eps=1e-3, precision=precision)
    zu, zp = [tt.full(c) for c in out.cores()]
    prec = MeanLSC(P, None, "full")
    ph = -prec.schur_inv_full(tt.full(r[1]))
    assert np.linalg.norm(zp - ph) <= 1e-5 * np.linalg.norm(ph)
    sh = (P.nt * P.n_xi, -1)
    rhs = tt.full(r[0]) - np.asarray(P.Bt @ ph.reshape(sh).T).T.reshape(zu.shape)
    res = np.linalg.norm(prec._mean_apply_full(zu) - rhs) / np.linalg.norm(rhs)
    _flush(f"inner relative residual {res:.3e}")
    assert res <= 0.15


def test_reserved_context_solves_without_allocating(sg):
    # with an arena reserved up front, a solve whose working set fits makes
    # no device allocation (after a first solve has tuned the spatial-solve
    # kernels for its column counts); the answer is the same
    ctx = sg.Context(0)
    _flush("reserved context: C1 solves")
    ctx.reserve(8 << 30)
    S = sg.System(ctx, CONFIGS["C1"])
    b = S.rhs()
    x1, st1, rc1 = S.solve(b, S.pair(96, 1024), restart=20, relax=1, inner_mode=1)
    x2, st2, rc2 = S.solve(b, S.pair(96, 1024), restart=20, relax=1, inner_mode=1)
    mem = ctx.memory()
    _flush(f"allocations: first solve {st1['device_allocs']}, second {st2['device_allocs']}; memory {mem}")
    assert rc1 == 0 and rc2 == 0 and st2["rel_residual"] <= 1e-8
    assert st2["device_allocs"] == 0
    assert 0 < mem["arena_peak_bytes"] <= mem["arena_bytes"] == 8 << 30
    d = tt.pair_full(x1.cores()) - tt.pair_full(x2.cores())
    assert np.linalg.norm(d) <= 1e-12 * np.linalg.norm(tt.pair_full(x1.cores()))


def test_preconditioner_fp32_mean_solve_matches_oracle(sg, ctx, c1):
    # the time-stepped mean solve in FP32 (precision 1) against the oracle's
    # FP64 full-format preconditioner: agreement to FP32 rounding, far below
    # the 1e-3 truncation the mean solve is compressed with
    P, S = c1
    _flush("precondition c1, FP32 time-stepped mean solve")
    r = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 4), (2, 3), 31)
    out = S.precondition(_pair_buf(S, r, 32, 256), eps_krylov=1e-13, inner_eps=1e-13, inner_mode=1, precision=1)
    prec = MeanLSC(P, None, "full")
    yu, yp = tt.full(r[0]), tt.full(r[1])
    vu, vp = prec.apply_full_exact(yu, yp)
    want = np.concatenate([vu.ravel(), vp.ravel()])
    got = tt.pair_full(out.cores())
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    _flush(f"FP32 mean solve vs oracle: {err:.2e}")
    assert err <= 1e-5


def test_solve_c1_fp32_mean_solve_to_1e8(sg, ctx, c1):
    # the flexible outer solve with the FP32 mean solve in the preconditioner
    # still reaches the oracle's exact solution (FP64 outer iteration and
    # refinement, sec. 4.2)
    P, S = c1
    _flush("solve c1 with the FP32 mean solve")
    b = S.rhs()
    x, st, rc = S.solve(b, S.pair(96, 1024), restart=20, relax=1, inner_mode=1, precision=1, **TIGHT)
    err = _solution_error(P, x)
    _flush(f"outer {st['outer_iters']} residual {st['rel_residual']:.2e} solution error {err:.2e}")
    assert rc == 0 and st["rel_residual"] <= 1e-10
    assert err <= 1e-8


def test_solve_c1_relaxed_precision_to_1e8(sg, ctx, c1):
    # precision 3: the FP32 mean solve only once the residual of the whole
    # solve is below 0.05 tol / 1e-5; the solve still reaches the oracle's
    # exact solution, with the same outer iterations as in FP64 and some
    # preconditioner applications in FP32
    P, S = c1
    _flush("solve c1 with relaxed precision")
    b = S.rhs()
    x64, st64, rc64 = S.solve(b, S.pair(96, 1024), restart=20, relax=1, inner_mode=1, precision=0, **TIGHT)
    x, st, rc = S.solve(b, S.pair(96, 1024), restart=20, relax=1, inner_mode=1, precision=3, **TIGHT)
    err = _solution_error(P, x)
    _flush(f"outer {st['outer_iters']} (FP64 {st64['outer_iters']}) residual {st['rel_residual']:.2e} "
           f"solution error {err:.2e} FP32 applications {st['f32_applications']}")
    assert rc == 0 and st["rel_residual"] <= 1e-10
    assert err <= 1e-8
    assert st["f32_applications"] > 0
    assert st["outer_iters"] <= st64["outer_iters"] + 2
    assert st64["f32_applications"] == 0


@pytest.fixture(scope="module")
def kl_systems(sg, ctx):
    out = {}
    for name in ("tinykl", "C1kl"):
        out[name] = (Problem(CONFIGS[name]), sg.System(ctx, CONFIGS[name]))
    return out


@pytest.mark.parametrize("name", ["tinykl", "C1kl"])
def test_kl_apply_and_rhs_match_oracle(sg, ctx, kl_systems, name):
    # the paper's KL viscosity (sec. 6.1): m + 1 viscous terms
    # sum_l G_l (x) A_l in the operator (eq. 3.6, 3.11-3.12) and in the
    # right-hand side, each side with its own KL expansion
    P, S = kl_systems[name]
    _flush(f"KL apply and rhs {name}")
    x = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 5), (2, 4), 41)
    out = S.apply(_pair_buf(S, x, 32, 128))
    want = tt.pair_full(P.apply(x))
    got = tt.pair_full(out.cores())
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    b = S.rhs()
    bo = tt.pair_full(P.rhs())
    assert np.abs(tt.pair_full(b.cores()) - bo).max() <= 1e-12 * np.abs(bo).max()


def test_kl_solve_c1_reaches_oracle_solution(sg, ctx, kl_systems):
    P, S = kl_systems["C1kl"]
    _flush("KL solve C1")
    b = S.rhs()
    x, st, rc = S.solve(b, S.pair(96, 1024), restart=20, relax=1, inner_mode=1, **TIGHT)
    err = _solution_error(P, x)
    _flush(f"outer {st['outer_iters']} residual {st['rel_residual']:.2e} solution error {err:.2e}")
    assert rc == 0 and st["rel_residual"] <= 1e-10
    assert err <= 1e-8
