"""Pins of the oracle's tensor-train algebra against library SVDs, the
explicit Kronecker product and the error bounds of sec. 4.1."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import tt
from synthetic_inputs import random_tt_cores

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_vec_order_is_c_order():
    # eq. 4.1: vec index i3 + (i2-1) n3 + (i1-1) n2 n3  (1-based)
    G = random_tt_cores(4, 3, 5, 2, 2, 1)
    X = tt.full(G)
    v = X.ravel()
    i1, i2, i3 = 2, 1, 3
    assert v[i3 + i2 * 5 + i1 * 3 * 5] == X[i1, i2, i3]


@pytest.mark.parametrize("eps", [1e-1, 1e-3, 1e-6])
def test_round_equals_ttsvd_of_full(eps):
    G = random_tt_cores(7, 5, 40, 6, 9, 3, decay=0.6)
    X = tt.full(G)
    a = tt.tt_round(G, eps)
    b = tt.tt_svd(X, eps)
    assert tt.ranks(a) == tt.ranks(b)
    assert np.linalg.norm(tt.full(a) - tt.full(b)) <= 1e-10 * np.linalg.norm(X)
    err = np.linalg.norm(tt.full(a) - X)
    assert err <= eps * np.linalg.norm(X) * (1 + 1e-12)        # eq. 4.6


def test_truncation_error_is_discarded_singular_values():
    # Eckart-Young on the first unfolding: TT-SVD keeps r1 leading singular
    # triplets; the error of that step is the discarded tail.
    G = random_tt_cores(9, 4, 30, 7, 8, 5, decay=0.5)
    X = tt.full(G)
    s = np.linalg.svd(X.reshape(9, -1), compute_uv=False)
    eps = 1e-2
    delta = eps * np.linalg.norm(X) / np.sqrt(2)
    r1 = tt.rank_cut(s, delta)
    assert np.sqrt(np.sum(s[r1:] ** 2)) <= delta < np.sqrt(np.sum(s[r1 - 1:] ** 2))
    a = tt.tt_svd(X, eps)
    assert tt.ranks(a)[0] == r1
    # total error <= sqrt(delta1^2 + delta2^2) (eq. 4.7)
    assert np.linalg.norm(tt.full(a) - X) <= np.sqrt(2) * delta * (1 + 1e-12)


def test_round_of_sum_and_exact_cases():
    G = random_tt_cores(5, 4, 20, 3, 4, 7)
    s = tt.concat([G, G], [1.0, 1.0])
    assert tt.ranks(s) == (6, 8)
    r = tt.tt_round(s, 1e-12)
    assert tt.ranks(r) == (3, 4)
    assert np.allclose(tt.full(r), 2 * tt.full(G), atol=1e-12)
    z = tt.tt_round(tt.concat([G, G], [0.0, 0.0]), 1e-8)       # exact zero -> rank 1
    assert tt.ranks(z) == (1, 1) and np.abs(tt.full(z)).max() < 1e-12


def test_dot_and_norm():
    x = random_tt_cores(6, 5, 17, 3, 4, 11)
    y = random_tt_cores(6, 5, 17, 2, 5, 12)
    assert abs(tt.tt_dot(x, y) - tt.full(x).ravel() @ tt.full(y).ravel()) < 1e-9
    assert abs(tt.tt_norm(x) - np.linalg.norm(tt.full(x))) < 1e-10


def test_kron_apply_matches_explicit_kron():
    # eq. 4.4
    n1, n2, n3 = 4, 3, 10
    x = random_tt_cores(n1, n2, n3, 2, 3, 21)
    g = np.random.default_rng(5)
    X1 = g.standard_normal((n1, n1))
    X2 = g.standard_normal((n2, n2))
    X3 = sp.random(n3, n3, density=0.4, random_state=3, format="csr")
    y = tt.kron_apply([(X1, X2, X3), (None, X2, None)], x)
    K = sp.kron(sp.kron(X1, X2), X3) + sp.kron(sp.kron(np.eye(n1), X2), np.eye(n3))
    assert np.allclose(K @ tt.full(x).ravel(), tt.full(y).ravel(), atol=1e-11)


def test_storage_ratio_eq_6_6():
    g = GOLD["storage_ratio"]
    n_t, n_xi, n_u = 64, 20, 2992
    k1, k2 = g["kappa1"], g["kappa2"]
    num = n_t * k1 + n_xi * k1 * k2 + n_u * k2
    den = n_t * n_xi * n_u
    assert num == g["numerator"] and den == g["denominator"]
    assert round(100 * num / den, 1) == g["percent"]
