"""GPU parity of the learned correction of the mean spatial solve: the
hand-written forward and backward kernels against the FP64 oracle (same
FP16-rounded weights), training on pairs the solver records from its own
exact mean solves, and solves with the network in the preconditioner (which
must still reach the exact-residual target; iteration counts are reported
against the plain preconditioner)."""
import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import tt
from oracle.system import Problem
from synthetic_inputs import CONFIGS

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


def _params(n, w, seed):
    p = omlp.init_params(n, w, seed)
    g = np.random.default_rng(seed + 7)
    p["b1"] = (0.1 * g.standard_normal(w)).astype(np.float32).astype(np.float64)
    p["b2"] = (0.1 * g.standard_normal(w)).astype(np.float32).astype(np.float64)
    p["b3"] = (0.1 * g.standard_normal(n)).astype(np.float32).astype(np.float64)
    return p


@pytest.mark.parametrize("n,w,B", [(40, 16, 7), (70, 48, 37), (130, 96, 65)])
def test_mlp_forward_and_gradients_match_oracle(sg, ctx, n, w, B):
    _flush(f"mlp n={n} w={w} B={B}")
    p = _params(n, w, n)
    net = sg.Mlp(ctx, n, w, 0, 0)
    net.set_params(p)
    g = np.random.default_rng(n + 1)
    X = g.standard_normal((n, B)).astype(np.float32).astype(np.float64)
    T = g.standard_normal((n, B)).astype(np.float32).astype(np.float64)
    Y = net.forward(X)
    Yo, _ = omlp.forward(p, X)
    assert np.linalg.norm(Y - Yo) <= 1e-5 * np.linalg.norm(Yo)
    # the preconditioner's form on the FP16 matrix cores: against the oracle
    # with the same operand rounding (a rounding to FP16 taken from FP32
    # values that differ in the last bit can land one FP16 step apart, so
    # the bound is a few FP16 steps of one activation), and against the
    # exact forward by the FP16 rounding of the operands
    Y16 = net.forward(X, f16=True)
    Yo16 = omlp.forward_f16(p, X)
    e16 = np.linalg.norm(Y16 - Yo16) / np.linalg.norm(Yo16)
    e64 = np.linalg.norm(Y16 - Yo) / np.linalg.norm(Yo)
    _flush(f"fp16 operands: vs oracle with fp16 operands {e16:.2e}, vs exact forward {e64:.2e}")
    assert e16 <= 2e-4
    assert e64 <= 5e-3
    L, gr = net.loss_grad(X, T)
    Lo, go = omlp.grads(p, X, T)
    assert abs(L - Lo) <= 1e-5 * Lo
    for k in go:
        assert np.linalg.norm(gr[k] - go[k]) <= 1e-4 * np.linalg.norm(go[k]), k


def test_mlp_adam_steps_match_oracle(sg, ctx):
    # full-batch Adam from zero state, three steps, against the oracle's
    # update on its own FP64 gradients of the FP16-rounded working weights
    _flush("mlp adam")
    n, w, B, lr = 40, 16, 9, 1e-3
    p = _params(n, w, 3)
    net = sg.Mlp(ctx, n, w, B, 0)
    net.set_params(p)
    g = np.random.default_rng(4)
    X = g.standard_normal((n, B)).astype(np.float32).astype(np.float64)
    T = g.standard_normal((n, B)).astype(np.float32).astype(np.float64)
    assert net.add_pairs(X, T) == B
    losses = net.train(3, batch=B, lr=lr)
    master = {k: v.copy() for k, v in p.items()}
    work = {k: v.copy() for k, v in p.items()}
    state = {k: [np.zeros_like(v), np.zeros_like(v)] for k, v in p.items()}
    for t in range(1, 4):
        L, gr = omlp.grads(work, X, T)
        assert abs(losses[t - 1] - L) <= 1e-5 * L
        for k in p:
            master[k], w16 = omlp.adam_step(master[k], gr[k], state[k], lr, t)
            work[k] = w16 if k.startswith("W") else master[k]
    got = net.get_params()
    for k in p:
        # FP32 masters vs FP64: agreement to FP32 resolution of the weights
        # (each step moves a parameter by about lr, so a wrong update rule
        # shows at that scale); gradients near Adam's eps may flip
        d = np.abs(got[k] - master[k])
        assert np.mean(d <= 1e-4 * lr + 4e-7 * np.abs(master[k])) >= 0.98, k
        assert d.max() <= 6 * lr + 1e-6, k


def test_mlp_save_and_load(sg, ctx, tmp_path):
    # a trained network written to a file and read into another network of
    # the same shape gives the same parameters and the same forward, on both
    # matrix-core forms; a network of another shape refuses the file and
    # keeps its own parameters
    _flush("mlp save/load")
    n, w, B = 40, 16, 9
    net = sg.Mlp(ctx, n, w, B, 0)
    net.set_params(_params(n, w, 7))
    g = np.random.default_rng(8)
    X = g.standard_normal((n, B)).astype(np.float32)
    T = g.standard_normal((n, B)).astype(np.float32)
    net.add_pairs(X, T)
    net.train(2, batch=B, lr=1e-3)
    f = str(tmp_path / "net.sgmlp")
    net.save(f)
    assert sg.mlp_file_info(f) == (n, w, net.size()[0])
    other = sg.Mlp(ctx, n, w, 0, 11)
    other.load(f)
    a, b = net.get_params(), other.get_params()
    assert all(np.array_equal(a[k], b[k]) for k in a)
    assert np.array_equal(sg.read_mlp_host(f, n, w), net.flatten(a))
    for f16 in (False, True):
        assert np.array_equal(net.forward(X, f16), other.forward(X, f16))
    wrong = sg.Mlp(ctx, n, w + 1, 0, 12)
    before = wrong.get_params()
    with pytest.raises(sg.SgttError) as e:
        wrong.load(f)
    assert e.value.code == -1
    after = wrong.get_params()
    assert all(np.array_equal(before[k], after[k]) for k in before)


def test_learned_mean_solve_c1(sg, ctx):
    _flush("learned mean solve c1")
    cfg = CONFIGS["C1"]
    S = sg.System(ctx, cfg)
    b = S.rhs()
    ns = S.info.n_s
    x0, st0, rc0 = S.solve(b, S.pair(64, 1024), restart=20, relax=1)
    assert rc0 == 0
    net = sg.Mlp(ctx, ns, 256, 20000, 1)
    net.collect(S)
    S.solve(b, S.pair(64, 1024), restart=20, relax=1)
    net.collect(S, False)
    npar, npairs = net.size()
    assert npairs > 1000
    losses = net.train(600, batch=128, lr=1e-3, seed=2)
    print("pairs", npairs, "loss first", losses[:5].mean(), "last", losses[-20:].mean(), flush=True)
    # an output of zero is the plain Jacobi step: relative error 1
    assert losses[-20:].mean() < 0.5
    net.attach(S)
    x1, st1, rc1 = S.solve(b, S.pair(64, 1024), restart=20, relax=1)
    print("plain", st0, flush=True)
    print("learned", st1, flush=True)
    assert rc1 == 0 and st1["rel_residual"] <= 1e-8
    assert st1["learned_calls"] > 0
    # refined past the target, the learned solve reaches the oracle's exact
    # solution: the network changes only the preconditioner
    x2, st2, rc2 = S.solve(b, S.pair(64, 1024), restart=20, relax=1, tol=1e-10, max_cycles=12)
    P = Problem(cfg)
    bo = P.rhs()
    u, p = P.solve_direct(tt.full(bo[0]), tt.full(bo[1]))
    want = np.concatenate([u.ravel(), p.ravel()])
    err = np.linalg.norm(tt.pair_full(x2.cores()) - want) / np.linalg.norm(want)
    print("learned solve refined: error vs oracle", err, flush=True)
    assert rc2 == 0 and err <= 1e-8


def test_learned_gain_on_held_out_viscosity(sg, ctx):
    """What the trained network gains, on a system it has not seen.  Pairs
    come from exact mean solves of C1-shaped systems with mean viscosities
    1/30, 1/45 and 1/80; the held-out system has nu0 = 1/60.  The same solve
    (inner GMRES velocity block, eq. 5.22-5.23) runs with F_avg^-1 inside M
    taken three ways: the exact spatial solve (the plain preconditioner), the
    Jacobi step D^-1 alone (a network with zero weights: what the network
    corrects), and D^-1 plus the trained correction.  The trained network
    must need fewer inner iterations than the Jacobi step and no fallback;
    the plain preconditioner is reported beside them."""
    import time
    _flush("learned gain on a held-out viscosity")
    base = CONFIGS["C1"]
    opts = dict(restart=20, relax=1, inner_mode=0)
    ns = None
    net = None
    for nu0 in (1 / 30, 1 / 45, 1 / 80):
        S = sg.System(ctx, dict(base, nu0=nu0))
        ns = S.info.n_s
        if net is None:
            net = sg.Mlp(ctx, ns, 256, 30000, 1)
        net.collect(S)
        S.solve(S.rhs(), S.pair(64, 1024), **opts)
        net.collect(S, False)
        del S
    npar, npairs = net.size()
    losses = net.train(800, batch=128, lr=1e-3, seed=3)
    _flush(f"pairs {npairs}, training loss first {losses[:5].mean():.3f} last {losses[-20:].mean():.3f}")
    S = sg.System(ctx, dict(base, nu0=1 / 60))
    b = S.rhs()
    zero = sg.Mlp(ctx, ns, 256, 0, 5)
    zero.set_params({k: np.zeros_like(v) for k, v in zero.get_params().items()})
    runs = {}
    for name, m in (("plain", None), ("jacobi", zero), ("learned", net)):
        if m is not None:
            m.attach(S)
        t0 = time.perf_counter()
        x, st, rc = S.solve(b, S.pair(64, 1024), **opts)
        dt = time.perf_counter() - t0
        if m is not None:
            m.attach(S, False)
        runs[name] = (st, rc, dt)
        _flush(f"{name}: outer {st['outer_iters']} inner {st['inner_iters']} residual {st['rel_residual']:.2e} "
               f"fallback {st['learned_fallback']} learned calls {st['learned_calls']} time {dt:.2f} s")
        assert rc == 0 and st["rel_residual"] <= 1e-8
    st_l, st_j = runs["learned"][0], runs["jacobi"][0]
    assert st_l["learned_calls"] > 0 and not st_l["learned_fallback"]
    assert st_j["learned_fallback"] or st_l["inner_iters"] < st_j["inner_iters"]
