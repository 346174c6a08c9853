"""Failure handling forced from the host, every kernel exiting normally:
the iteration limit (Alg. 4.2's maxit; status SGTT_W_NOT_CONVERGED with the
best iterate), a non-finite right-hand side (refused before any rounding,
the context usable afterwards), a network whose corrections do not help
(the learned mean solve falls back to the exact one), and a context
destroyed before the system and network made on it."""
import numpy as np
import pytest

from synthetic_inputs import CONFIGS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    from paper_1906_06785_amd import sgtt
    return sgtt


@pytest.fixture(scope="module")
def ctx(sg):
    return sg.Context(0)


def test_iteration_limit_returns_best_iterate(sg, ctx):
    print("iteration limit c1", flush=True)
    S = sg.System(ctx, CONFIGS["C1"])
    b = S.rhs()
    x, st, rc = S.solve(b, S.pair(64, 1024), restart=2, max_cycles=1)
    assert rc == 1 and st["cycles"] == 1 and st["outer_iters"] == 2
    assert 0.0 < st["rel_residual"] < 1.0
    assert S.residual(b, x) == pytest.approx(st["rel_residual"], rel=1e-10, abs=1e-14)


def test_non_finite_right_hand_side_is_refused(sg, ctx):
    print("non-finite right-hand side tiny", flush=True)
    S = sg.System(ctx, CONFIGS["tiny"])
    b = S.rhs()
    b.u.c3[0] = float("nan")
    with pytest.raises(sg.SgttError) as e:
        S.solve(b, S.pair(16, 64))
    assert e.value.code == -5
    # the context and the system still work
    x, st, rc = S.solve(S.rhs(), S.pair(16, 64))
    assert rc == 0 and st["rel_residual"] <= 1e-8


def test_useless_network_falls_back_to_exact_mean_solve(sg, ctx):
    print("learned fallback c1", flush=True)
    S = sg.System(ctx, CONFIGS["C1"])
    net = sg.Mlp(ctx, S.info.n_s, 64, 0, 11)
    g = np.random.default_rng(5)
    net.set_params({k: 30.0 * g.standard_normal(v.shape).astype(np.float32) for k, v in net.get_params().items()})
    net.attach(S)
    x, st, rc = S.solve(S.rhs(), S.pair(64, 1024), restart=20, relax=1, inner_mode=0)
    net.attach(S, False)
    print(st, flush=True)
    assert rc == 0 and st["rel_residual"] <= 1e-8
    assert st["learned_calls"] > 0 and st["learned_fallback"] == 1


def test_context_destroyed_before_its_system_and_network(sg):
    """A garbage-collected cycle finalizes its objects in any order: a
    context destroyed while a system and a network still use it stays
    alive until the last of them is destroyed (then it is released)."""
    print("context destroyed first tiny", flush=True)
    c2 = sg.Context(0)
    S = sg.System(c2, CONFIGS["tiny"])
    net = sg.Mlp(c2, S.info.n_s, 64, 0, 3)
    x, st, rc = S.solve(S.rhs(), S.pair(16, 64))
    assert rc == 0 and st["rel_residual"] <= 1e-8
    c2.__del__()   # context first
    assert c2._c is None
    S.__del__()    # the system's TTs go back to the closing context's pool
    net.__del__()  # the last child: the context is released here
    assert S._s is None and net._m is None
