"""Pins of the oracle's chaos matrices: closed forms and brute-force tensor
quadrature with scipy's Legendre polynomials (independent of oracle.gpc's
numpy evaluation)."""
from math import comb

import numpy as np
import pytest
from scipy.special import eval_legendre, roots_legendre

from oracle import gpc


@pytest.mark.parametrize("m,p", [(2, 2), (3, 3), (4, 3), (2, 1)])
def test_sizes_and_identities(m, p):
    idx, G, H = gpc.gpc_matrices(m, p)
    assert len(idx) == comb(m + p, p)          # n_xi = (m+p)!/(m!p!), sec. 6.1
    assert idx[0] == (0,) * m                  # psi_1 = 1 first
    n = len(idx)
    assert np.allclose(G[0], np.eye(n), atol=1e-14)     # G_0 = I (sec. 5.2)
    assert np.allclose(H[0], np.eye(n), atol=1e-14)     # H_1 = I (sec. 5.2)
    for l in range(m + 1):
        assert np.allclose(G[l], G[l].T, atol=1e-15)
    for l in range(n):
        assert np.allclose(H[l], H[l].T, atol=1e-14)


def _psi(n, x):
    return np.sqrt(2 * n + 1) * eval_legendre(n, x)


@pytest.mark.parametrize("m,p", [(2, 2), (3, 2)])
def test_brute_force_tensor_quadrature(m, p):
    idx, G, H = gpc.gpc_matrices(m, p)
    x, w = roots_legendre(p + 3)
    w = w / 2.0
    grids = np.meshgrid(*([x] * m), indexing="ij")
    W = np.ones_like(grids[0])
    for k, wk in enumerate(np.meshgrid(*([w] * m), indexing="ij")):
        W = W * wk
    Psi = []
    for a in idx:
        v = np.ones_like(grids[0])
        for k in range(m):
            v = v * _psi(a[k], grids[k])
        Psi.append(v)
    n = len(idx)
    for l in range(1, m + 1):
        ref = np.array([[np.sum(W * grids[l - 1] * Psi[r] * Psi[s]) for s in range(n)] for r in range(n)])
        assert np.abs(ref - G[l]).max() < 1e-13
    for l in range(n):
        ref = np.array([[np.sum(W * Psi[l] * Psi[r] * Psi[s]) for s in range(n)] for r in range(n)])
        assert np.abs(ref - H[l]).max() < 1e-13


def test_recurrence_closed_form():
    # <xi psi_j psi_{j-1}> = j / sqrt(4 j^2 - 1) for orthonormal Legendre
    X = gpc.xi1d(5)
    for j in range(1, 6):
        assert abs(X[j, j - 1] - j / np.sqrt(4 * j * j - 1)) < 1e-14
    assert np.abs(np.diag(X)).max() < 1e-15
