"""GPU parity of the block cyclic reduction spatial solves (the F_avg solve of
eq. 5.23 and the X = B M*^-1 B^T solve of eq. 5.19) against sparse direct
solves of the oracle's own assembly, for every kernel variant of the passes
(forced for all passes) and for the tuned choice."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

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


_systems = {}


def _system(sg, ctx, name):
    if name not in _systems:
        cfg = CONFIGS[name]
        P = Problem(cfg)
        S = sg.System(ctx, cfg)
        F = (P.M / cfg["tau"] + cfg["nu0"] * P.A).tocsc()
        X = (P.B @ sp.diags(1.0 / P.Mstar) @ P.Bt).tocsc()
        _systems[name] = (P, S, spl.splu(F), spl.splu(X))
    return _systems[name]


@pytest.mark.parametrize("name", ["C1", "C1b", "C2"])
@pytest.mark.parametrize("ncols", [35, 7])
def test_bcr_every_variant_matches_direct_solve(sg, ctx, name, ncols):
    import torch
    P, S, Flu, Xlu = _system(sg, ctx, name)
    rng = np.random.default_rng(ncols)
    ran = 0
    for which, lu, ncomp in ((0, Flu, 2), (1, Xlu, 1)):
        n = lu.shape[0]
        b = rng.standard_normal((ncomp * n, ncols))
        ref = np.concatenate([lu.solve(b[z * n:(z + 1) * n]) for z in range(ncomp)])
        bd = torch.from_numpy(b).cuda()
        for v in range(-1, sg.bcr_variant_count()):
            _flush(f"bcr {name} which={which} ncols={ncols} variant={v}")
            try:
                x = S.bcr_apply(which, bd, v).cpu().numpy()
            except sg.SgttError as e:
                assert "too large" in str(e)
                continue
            ran += 1
            assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max(), (which, v)
        # the right-hand side is left as it was
        assert torch.equal(bd.cpu(), torch.from_numpy(b))
    assert ran >= 2 * 12


def test_bcr_rejects_bad_arguments(sg, ctx):
    import torch
    P, S, Flu, Xlu = _system(sg, ctx, "C1")
    b = torch.zeros((P.n_p, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(sg.SgttError):
        S.bcr_apply(1, b, sg.bcr_variant_count())
    with pytest.raises(ValueError):
        S.bcr_apply(0, b, -1)


def test_bcr_choice_follows_its_factor_across_systems(sg, ctx):
    # the tuned kernel choice belongs to the factor it was timed on: systems
    # destroyed and assembled again (a C1 factor, then the larger C1b and C2
    # factors, then C1 again) each solve correctly with the tuned choice,
    # whatever device addresses the allocator hands out
    import gc
    import torch
    rng = np.random.default_rng(77)
    for name in ("C1", "C1b", "C2", "C1"):
        cfg = CONFIGS[name]
        P = Problem(cfg)
        F = (P.M / cfg["tau"] + cfg["nu0"] * P.A).tocsc()
        lu = spl.splu(F)
        for rep in range(2):
            S = sg.System(ctx, cfg)
            n = lu.shape[0]
            b = rng.standard_normal((2 * n, 35))
            ref = np.concatenate([lu.solve(b[z * n:(z + 1) * n]) for z in range(2)])
            _flush(f"bcr tuned choice {name} rep {rep}")
            x = S.bcr_apply(0, torch.from_numpy(b).cuda(), -1).cpu().numpy()
            assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max(), name
            del S
            gc.collect()
