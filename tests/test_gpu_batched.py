"""Batched solves of independent problems (different grids, chaos sizes,
horizons and mean viscosities) on several contexts at once: every result,
refined past the target, matches the oracle's exact (time-stepping) solution
of its problem to 1e-8, and takes within one outer iteration of the same
problem solved alone (the spatial-solve kernel variant is tuned per factor by
timing, and the variants add their partial products in different orders)."""
import numpy as np
import pytest

from oracle import tt
from oracle.system import Problem
from synthetic_inputs import batch_configs

pytestmark = pytest.mark.gpu


def test_batched_equals_sequential():
    from paper_1906_06785_amd import sgtt
    cfgs = batch_configs(6, seed=5, small=True)
    print("batch", cfgs, flush=True)
    ctxs = [sgtt.Context(0) for _ in range(3)]
    systems = [sgtt.System(ctxs[i % 3], c) for i, c in enumerate(cfgs)]
    bs = [S.rhs() for S in systems]
    xs = [S.pair(64, 1024) for S in systems]
    stats, status = sgtt.solve_batched(systems, bs, xs, restart=20, relax=1, tol=1e-10, max_cycles=12)
    assert all(s == 0 for s in status)
    assert all(st["rel_residual"] <= 1e-10 for st in stats)
    solo = sgtt.Context(0)
    for c, x, st in zip(cfgs, xs, stats):
        P = Problem(c)
        b = P.rhs()
        u, p = P.solve_direct(tt.full(b[0]), tt.full(b[1]))
        want = np.concatenate([u.ravel(), p.ravel()])
        err = np.linalg.norm(tt.pair_full(x.cores()) - want) / np.linalg.norm(want)
        S = sgtt.System(solo, c)
        y, st1, rc = S.solve(S.rhs(), S.pair(64, 1024), restart=20, relax=1, tol=1e-10, max_cycles=12)
        print(c, "error vs oracle", err, "outer", st["outer_iters"], st1["outer_iters"], flush=True)
        assert rc == 0
        assert err <= 1e-8
        assert abs(st["outer_iters"] - st1["outer_iters"]) <= 1
