"""Oracle: generalized polynomial chaos (Legendre) and the stochastic Galerkin
matrices G_l, H_l.

Test infrastructure only (see oracle/__init__.py).

The paper (sec. 3.2, eq. 3.9, sec. 5.2) fixes: orthonormal m-variate
polynomials with <psi_r psi_s> = delta_rs, psi_1 = 1, total degree <= p,
n_xi = (m+p)!/(m!p!) (sec. 6.1), [G_l]_rs = <xi_l psi_r psi_s> with xi_0 = 1,
[H_l]_rs = <psi_l psi_r psi_s>, so G_0 = H_1 = I.

Here xi_k ~ U[-1,1] iid; the 1-D orthonormal family is sqrt(2n+1) P_n.
Ordering of multi-indices (a convention shared with the GPU library by
definition): graded by total degree, and within one degree in descending
lexicographic order, e.g. m=2: (0,0), (1,0), (0,1), (2,0), (1,1), (0,2).

Triple products are evaluated by Gauss-Legendre quadrature of the 1-D
polynomials, which is exact at the point count used.  Pins
(tests/test_oracle_gpc.py): n_xi formula, G_0 = H_1 = I, symmetry, and a brute
force m-dimensional tensor quadrature of <xi_l psi_r psi_s>.
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np
from numpy.polynomial import legendre as npleg


def multi_indices(m: int, p: int):
    out = []
    for deg in range(p + 1):
        level = [a for a in itertools.product(range(deg + 1), repeat=m) if sum(a) == deg]
        level.sort(reverse=True)
        out.extend(level)
    assert len(out) == comb(m + p, p)
    return out


def psi1d(n: int, x: np.ndarray) -> np.ndarray:
    """sqrt(2n+1) P_n(x): orthonormal for the uniform density 1/2 on [-1,1]."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return np.sqrt(2 * n + 1) * npleg.legval(x, c)


def _gauss(npts):
    x, w = npleg.leggauss(npts)
    return x, w / 2.0   # expectation under U[-1,1]


def triple1d(p: int):
    """T[a,b,c] = <psi_a psi_b psi_c> for a,b,c <= p (1-D)."""
    x, w = _gauss(2 * p + 2)
    P = np.array([psi1d(n, x) for n in range(p + 1)])
    return np.einsum("q,aq,bq,cq->abc", w, P, P, P)


def xi1d(p: int):
    """X[a,b] = <xi psi_a psi_b> (1-D)."""
    x, w = _gauss(p + 2)
    P = np.array([psi1d(n, x) for n in range(p + 1)])
    return np.einsum("q,q,aq,bq->ab", w, x, P, P)


def gpc_matrices(m: int, p: int):
    """Returns (idx, G, H): G[l] for l = 0..m, H[l] for l = 0..n_xi-1
    (H[0] is the paper's H_1 = I)."""
    idx = multi_indices(m, p)
    n = len(idx)
    X = xi1d(p)
    T = triple1d(p)
    I = np.array(idx)
    G = np.zeros((m + 1, n, n))
    G[0] = np.eye(n)
    for l in range(m):
        for r in range(n):
            for s in range(n):
                others = np.all(np.delete(I[r], l) == np.delete(I[s], l))
                if others:
                    G[l + 1, r, s] = X[I[r, l], I[s, l]]
    H = np.zeros((n, n, n))
    for l in range(n):
        for r in range(n):
            for s in range(n):
                v = 1.0
                for k in range(m):
                    v *= T[I[l, k], I[r, k], I[s, k]]
                H[l, r, s] = v
    return idx, G, H


def viscosity_coefficients(m: int, nu0: float, nu_coef: float):
    """nu(xi) = nu0 (1 + nu_coef * sum_k xi_k / k^2): c_0 = nu0,
    c_k = nu_coef * nu0 / k^2, so that sum_l G_l (x) A_l = G_nu (x) A with
    G_nu = sum_l c_l G_l and A the unit-viscosity stiffness (eq. 3.6-3.7)."""
    return np.array([nu0] + [nu_coef * nu0 / k ** 2 for k in range(1, m + 1)])
