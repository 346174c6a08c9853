"""GPU parity at the benchmark's full size: the 64 x 192 step grid (h = 1/16),
m = 4, p = 3 (n_xi = 35), n_t = 128, tau = 0.05 -- 255.4 M unknowns -- solved
with exactly the options bench.py times.  The oracle cannot hold the system,
so it checks the GPU's full-format residual tensor on sampled entries that it
computes one by one from the solution's TT cores and its own right-hand side,
and the residual norm is recomputed from that tensor."""
import math

import numpy as np
import pytest

from oracle import tt
from oracle.system import Problem
from synthetic_inputs import CONFIGS

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.mark.timeout(600)
def test_c2_bench_solve_residual_on_sampled_entries():
    import torch
    from paper_1906_06785_amd import sgtt
    from bench import OUT_CAPS, solve_options

    print("full-size C2 Stokes solve (bench options)", flush=True)
    ctx = sgtt.Context(0)
    S = sgtt.System(ctx, CONFIGS["C2"])
    b = S.rhs()
    x, st, rc = S.solve(b, S.pair(*OUT_CAPS), **solve_options())
    print("solve stats", st, flush=True)
    assert rc == 0 and st["rel_residual"] <= 1e-8
    ru, rp, rel = S.residual_tensor(b, x)
    assert rel <= 1e-8
    assert abs(rel - st["rel_residual"]) <= 1e-3 * st["rel_residual"]

    P = Problem(CONFIGS["C2"])
    bo = P.rhs()
    bnorm = math.sqrt(tt.tt_dot(bo[0], bo[0]) + tt.tt_dot(bo[1], bo[1]))
    rnorm = math.sqrt(float((ru * ru).sum()) + float((rp * rp).sum()))
    # the GPU's residual norm is the norm of its residual tensor, over the oracle's ||b||
    assert abs(rnorm / bnorm - rel) <= 1e-6 * rel
    xc = x.cores()
    g = np.random.default_rng(2024)
    for which, R, n, cnt in (("u", ru, P.n_u, 3000), ("p", rp, P.n_p, 1000)):
        t, i, j = g.integers(0, P.nt, cnt), g.integers(0, P.n_xi, cnt), g.integers(0, n, cnt)
        want = P.residual_entries(bo, xc, which, t, i, j)
        got = R[torch.as_tensor(t), torch.as_tensor(i), torch.as_tensor(j)].cpu().numpy()
        err = np.abs(got - want).max()
        print(which, "max entry difference", err, "max |r| sampled", np.abs(want).max(), flush=True)
        assert err <= 1e-13 * bnorm


def _entries(cores, t, i, j):
    # z[t, i, j] of a TT in the paper's convention, entry by entry
    G1, G2, G3 = cores
    return np.einsum("ka,akb,bk->k", G1[t], G2[:, i, :], G3[:, j])


@pytest.mark.timeout(900)
def test_c2_picard_step1_operator_and_residual_on_sampled_entries():
    """Picard step-1 system at the full size (Alg. 3.1, eq. 3.14-3.15 with the
    convection of eq. 4.12) around a seeded smooth deterministic prior
    iterate whose wind has exact TT ranks (4, 4) (the Stokes iterate's wind truncated at 1e-3
    has ranks (5, 5) at this size): with eps_conv = 1e-12 both sides keep the
    wind unchanged, so N(w~) is the same operator on both.  (Winds with more
    spatial columns than one pass of the sparse product takes are checked at
    C1 in test_gpu_picard.py.)
    Checked: the right-hand side against the oracle's exact residual of the
    prior (within the truncation eps_rhs), the operator L(w~) x on sampled
    entries (the GPU's b - r against the oracle's L x), and the exact
    relative residual <= 1e-8."""
    import torch
    from paper_1906_06785_amd import sgtt
    from bench import OUT_CAPS, solve_options
    from synthetic_inputs import smooth_prior

    cfg = CONFIGS["C2"]
    P = Problem(cfg)
    prior = smooth_prior(P.nt, P.n_xi, cfg["tau"], P.mesh.coords[P.mesh.free], P.n_p, ranks_u=(3, 6),
                         ranks_p=(2, 3), seed=11, mean_only=True)
    print("full-size C2 Picard step-1 system around a smooth prior (bench options)", flush=True)
    ctx = sgtt.Context(0)
    pb = sgtt.PairBuf(P.nt, P.n_xi, P.n_u, P.n_p, 8, 32).set(prior)
    eps_rhs = 1e-6
    S = sgtt.System(ctx, cfg, prior=pb, eps_conv=1e-12, eps_rhs=eps_rhs)
    assert (S.info.conv_r1, S.info.conv_r2) == (4, 4)
    b = S.rhs(S.pair(128, 1024))
    print("rhs ranks", b.ranks, flush=True)
    # verbose: one line per outer iteration on stderr (progress of a long solve)
    x, st, rc = S.solve(b, S.pair(*OUT_CAPS), **dict(solve_options(), verbose=1))
    print("solve stats", st, flush=True)
    assert rc == 0 and st["rel_residual"] <= 1e-8
    ru, rp, rel = S.residual_tensor(b, x)
    assert rel <= 1e-8

    conv = P.convection(prior, 1e-12)
    assert (conv.k1, conv.k2) == (4, 4)
    bo = P.residual_tt(prior)     # exact (untruncated) right-hand side, eq. 3.15
    bnorm = math.sqrt(tt.tt_dot(bo[0], bo[0]) + tt.tt_dot(bo[1], bo[1]))
    xc, bc = x.cores(), b.cores()
    g = np.random.default_rng(2025)
    for which, R, n, cnt, q in (("u", ru, P.n_u, 2000, 0), ("p", rp, P.n_p, 1000, 1)):
        t, i, j = g.integers(0, P.nt, cnt), g.integers(0, P.n_xi, cnt), g.integers(0, n, cnt)
        b_gpu = _entries(bc[q], t, i, j)
        b_or = _entries(bo[q], t, i, j)
        db = np.abs(b_gpu - b_or).max()
        r_gpu = R[torch.as_tensor(t), torch.as_tensor(i), torch.as_tensor(j)].cpu().numpy()
        Lx_gpu = b_gpu - r_gpu
        Lx_or = b_or - P.residual_entries(bo, xc, which, t, i, j, conv)
        dL = np.abs(Lx_gpu - Lx_or).max()
        print(which, "rhs entry difference", db, "operator entry difference", dL, "max |Lx| sampled",
              np.abs(Lx_or).max(), "||b||", bnorm, flush=True)
        # the right-hand side is the exact residual truncated at eps_rhs
        # (up to the FP64 Gram accuracy of the truncation, ~1e-8)
        assert db <= (eps_rhs + 1e-8) * bnorm
        # the same operator on the same vector
        assert dL <= 1e-11 * bnorm
