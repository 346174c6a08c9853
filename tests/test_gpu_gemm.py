"""The library's FP64 product kernels (64 x 64 tiles, split-K for long
reductions, 128 x 128 tiles for large outputs) through sgtt_gemm, against
FP64 products on the host, at shapes that span several tiles with ragged
edges on every side."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    from paper_1906_06785_amd import sgtt
    return sgtt


@pytest.fixture(scope="module")
def ctx(sg):
    return sg.Context(0)


@pytest.mark.parametrize("m,n,k,beta", [(10, 7, 5, 0.0), (130, 70, 33, 0.5), (64, 64, 5000, 0.0),
                                        (300, 260, 37, 0.0), (517, 389, 150, -1.0), (256, 1000, 16, 0.0),
                                        (2049, 300, 201, 0.0), (300, 300, 0, 2.0)])
def test_gemm_matches_host_product(sg, ctx, m, n, k, beta):
    import torch
    print(f"gemm {m}x{n}x{k}", flush=True)
    g = np.random.default_rng(m + 3 * n + 7 * k)
    A = g.standard_normal((m, k))
    B = g.standard_normal((k, n))
    C0 = g.standard_normal((m, n))
    dev = torch.device("cuda", 0)
    tA, tB, tC = (torch.from_numpy(x).to(dev) for x in (A, B, C0))
    got = ctx.gemm(tA, tB, tC, alpha=1.5, beta=beta).cpu().numpy()
    want = 1.5 * (A @ B) + beta * C0
    scale = 1.5 * np.abs(A) @ np.abs(B) + abs(beta) * np.abs(C0)
    assert np.all(np.abs(got - want) <= 1e-14 * max(k, 1) * scale + 1e-300)
