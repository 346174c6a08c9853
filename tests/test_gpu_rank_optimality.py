"""Ranks of the device's Gram-based rounding against the optimal ranks of
SVD truncation (the oracle's tt_round, eq. 4.5-4.7) on the C2 solve's own
vectors: the velocity and pressure TTs of L x for the C2 Stokes solution x
(ranks before rounding up to about 200, second-bond Grams of order above 512,
which take the blocked pivoted Cholesky and skeleton route), at the Krylov
truncation tolerance and around it.  The error bound of eq. 4.6 holds on
every one; the ranks are reported and bounded against the optimal ones."""
import numpy as np
import pytest

from oracle import tt
from synthetic_inputs import CONFIGS

pytestmark = pytest.mark.gpu


def test_rounding_ranks_near_optimal_on_c2_vectors():
    from paper_1906_06785_amd import sgtt as sg
    print("rank optimality c2", flush=True)
    ctx = sg.Context(0)
    S = sg.System(ctx, CONFIGS["C2"])
    b = S.rhs()
    x, st, rc = S.solve(b, S.pair(512, 8192), restart=20, relax=1, inner_mode=1)
    assert rc == 0
    # a partial solve, its exact residual b - L x5 (the right-hand side of a
    # refinement cycle), and that residual preconditioned (a Krylov direction)
    x5, _, _ = S.solve(b, S.pair(512, 8192), restart=5, max_cycles=1, relax=1, inner_mode=1)
    r = S.apply(x5, S.pair(1024, 8192))
    r = ctx.axpby(1.0, b, -1.0, r)
    rr = S.pair(1024, 8192)
    rr.set(r.cores())
    for comp in (rr.u, rr.p):
        ctx.round(comp, 1e-6)
    z = S.precondition(rr, S.pair(512, 8192), inner_mode=1)
    vectors = {"solution": x, "residual": r, "preconditioned": z}
    rows = []
    for (name, v), comp, G in [((nm, v), c, G) for nm, v in vectors.items() for c, G in zip(("u", "p"), v.cores())]:
        n1, n2, n3 = G[0].shape[0], G[1].shape[1], G[2].shape[1]
        nrm = tt.tt_norm(G)
        for eps in (1e-4, 1e-6, 1e-8):
            ref = tt.tt_round(G, eps)
            r_ref = tt.ranks(ref)
            buf = sg.TTBuf(n1, n2, n3, G[0].shape[1], G[2].shape[0]).set_cores(*G)
            ctx.round(buf, eps)
            got = buf.cores()
            err = tt.tt_norm(tt.concat([got, G], [1.0, -1.0]))
            rows.append((name, comp, eps, G[0].shape[1], G[2].shape[0], r_ref, (buf.r1, buf.r2), err / nrm))
            print(f"{name} {comp} eps {eps:.0e}: ranks in ({G[0].shape[1]}, {G[2].shape[0]}), optimal {r_ref}, "
                  f"device ({buf.r1}, {buf.r2}), error {err / nrm:.2e}", flush=True)
            if eps >= 1e-6:
                # eq. 4.6 up to the accuracy of FP64 Grams, and ranks at or
                # just above the optimal ones
                assert err <= eps * nrm * (1 + 1e-6) + 2e-8 * nrm
                assert abs(buf.r1 - r_ref[0]) <= 1
                assert r_ref[1] - 1 <= buf.r2 <= 1.25 * r_ref[1] + 4
            else:
                # below the Gram floor: products of Gram matrices of cores
                # that cancel in the sum resolve singular values only to a
                # few 1e-8 of the norm to a few 1e-7; the rank found is then
                # at most the optimal one and the error is that floor
                assert err <= 1e-6 * nrm
                assert buf.r1 <= r_ref[0] + 1 and buf.r2 <= r_ref[1] + 1
