"""The time loop of the exact mean solve as one captured HIP graph (solve
option graph = 1): every replay gives what the plain launches give, with
other work of the program and synchronizations between the replays, in FP64
and FP32, on two systems of one context; a solve with it takes the same
iterations as without and meets the oracle's solution."""
import numpy as np
import pytest

from oracle import tt
from oracle.system import Problem
from synthetic_inputs import CONFIGS, random_tt_pair

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
def c1(sg, ctx):
    return Problem(CONFIGS["C1"]), sg.System(ctx, CONFIGS["C1"])


@pytest.fixture(scope="module")
def tiny(sg, ctx):
    return Problem(CONFIGS["tiny"]), sg.System(ctx, CONFIGS["tiny"])


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_match_plain_launches(sg, ctx, c1, tiny, precision):
    import torch
    opts = dict(eps_krylov=1e-13, inner_eps=1e-13, inner_mode=1, precision=precision)
    for name, (P, S) in (("C1", c1), ("tiny", tiny)):
        _flush(f"graph replays {name} precision {precision}")
        rs = [random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (3, 5), (2, 4), 40 + i) for i in range(3)]
        bufs = [S.pair(32, 256).set(r) for r in rs]
        # plain launches first: they also tune the spatial solve's kernels,
        # which the graph is captured after
        plain = [tt.pair_full(S.precondition(b, **opts).cores()) for b in bufs]
        for rep in range(3):
            for i, b in enumerate(bufs):
                got = tt.pair_full(S.precondition(b, graph=1, **opts).cores())
                d = _rel(got, plain[i])
                _flush(f"  replay {rep} input {i}: max rel difference {d:.1e}, identical {np.array_equal(got, plain[i])}")
                assert d <= 1e-14
                # the program's own work and a synchronization between replays
                S.apply(b)
                again = tt.pair_full(S.precondition(b, **opts).cores())
                torch.cuda.synchronize()
                assert _rel(again, plain[i]) <= 1e-14


def test_solve_with_graph_matches_plain_and_oracle(sg, ctx, c1):
    P, S = c1
    _flush("solve c1 with the graph form of the mean solve")
    b = S.rhs()
    tight = dict(tol=1e-10, inner_mode=1, restart=20, eps_krylov=1e-10, inner_eps=1e-10)
    x0, st0, rc0 = S.solve(b, **tight)
    x1, st1, rc1 = S.solve(b, **tight, graph=1)
    _flush(f"plain: {st0['outer_iters']} outer, {st0['rel_residual']:.2e}; graph: {st1['outer_iters']} outer, "
           f"{st1['rel_residual']:.2e}, {st1['graph_launches']} graph launches")
    assert rc0 == 0 and rc1 == 0
    assert st1["outer_iters"] == st0["outer_iters"]
    assert st1["rel_residual"] <= 1e-10
    assert st1["graph_launches"] >= 1 and st0["graph_launches"] == 0
    f0, f1 = tt.pair_full(x0.cores()), tt.pair_full(x1.cores())
    assert np.linalg.norm(f1 - f0) <= 1e-12 * np.linalg.norm(f0)
    # the oracle's exact solution of the same system
    bo = P.rhs()
    u, p = P.solve_direct(tt.full(bo[0]), tt.full(bo[1]))
    want = np.concatenate([u.ravel(), p.ravel()])
    err = np.linalg.norm(f1 - want) / np.linalg.norm(want)
    _flush(f"solution error against the oracle {err:.2e}")
    assert err <= 1e-8


def test_graph_option_is_checked(sg, ctx, tiny):
    P, S = tiny
    r = random_tt_pair(P.nt, P.n_xi, P.n_u, P.n_p, (2, 3), (2, 3), 47)
    with pytest.raises(sg.SgttError) as ei:
        S.precondition(S.pair(32, 256).set(r), inner_mode=1, graph=2)
    assert ei.value.code == -1
