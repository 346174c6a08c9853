"""Oracle: truncated Karhunen-Loeve expansion of the random viscosity
(sec. 6.1): nu(x, xi) = nu0 (1 + sigma sum_{l=1}^m sqrt(beta_l) a_l(x) xi_l)
with the exponential covariance c(x, y) = exp(-||x - y||_1 / b) and
(beta_l, a_l) its m largest eigenpairs, int_D c(x, y) a_l(y) dy = beta_l a_l(x),
computed with a standard finite element method as the paper does.

Test infrastructure only (see oracle/__init__.py).

Discretization (a reading: the paper does not say which elements): Galerkin
on the bilinear (Q1) space of the mesh vertices, C a = beta M_p a with
C_kl = int int c(x, y) psi_k(x) psi_l(y) dx dy by 3 x 3 Gauss quadrature in
both integrals and M_p the Q1 mass matrix; eigenvectors M_p-orthonormal
(int a_l^2 = 1).  Sign convention (both sides use it): the first vertex, in
vertex order, where |a_l| >= max|a_l| / 2 has a_l > 0.

The stiffness matrices of the expansion (eq. 3.6-3.7 with nu_l(x) =
nu0 sigma sqrt(beta_l) a_l(x)) weight the Q2 gradients by the Q1 field a_l at
the Gauss points (mesh.stiffness_weighted).

Pins (tests/test_oracle_kl.py): on a rectangle the separable kernel's
eigenvalues are products of the 1-D exponential kernel's, known in closed form
through transcendental equations; the weighted stiffness reproduces the unit
stiffness for a = 1 and the domain's first moment for a = x1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import mesh as fem


def _q1_quadrature(pcoords, pconn, h):
    """Gauss points (ng, 2), weights (ng,) and the sparse Q1 basis values at
    them (ng x n_vertices) for square elements of side h."""
    _, _, psi, wq = fem._ref_tables()
    ne = pconn.shape[0]
    gp = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
    # reference point g = ia + 3 jb at (gp[ia], gp[jb]); element corner 0 is
    # its lower-left vertex, the square spans [x0, x0 + h] x [y0, y0 + h]
    xi = np.array([gp[g % 3] for g in range(9)])
    eta = np.array([gp[g // 3] for g in range(9)])
    x0 = pcoords[pconn[:, 0]]
    X = np.empty((ne, 9, 2))
    X[:, :, 0] = x0[:, None, 0] + (xi[None, :] + 1.0) * h / 2.0
    X[:, :, 1] = x0[:, None, 1] + (eta[None, :] + 1.0) * h / 2.0
    W = np.broadcast_to(wq * (h / 2.0) ** 2, (ne, 9))
    rows = np.repeat(np.arange(ne * 9), 4)
    cols = np.broadcast_to(pconn[:, None, :], (ne, 9, 4)).reshape(-1)
    vals = np.broadcast_to(psi[None, :, :], (ne, 9, 4)).reshape(-1)
    Psi = sp.csr_matrix((vals, (rows, cols)), shape=(ne * 9, pcoords.shape[0]))
    return X.reshape(-1, 2), W.reshape(-1), Psi


def q1_mass(pcoords, pconn, h):
    X, W, Psi = _q1_quadrature(pcoords, pconn, h)
    return (Psi.T @ sp.diags(W) @ Psi).tocsr()


def covariance_matrix(pcoords, pconn, h, b):
    """C_kl = int int exp(-||x - y||_1 / b) psi_k(x) psi_l(y) dx dy."""
    X, W, Psi = _q1_quadrature(pcoords, pconn, h)
    D = np.abs(X[:, None, 0] - X[None, :, 0]) + np.abs(X[:, None, 1] - X[None, :, 1])
    K = np.exp(-D / b) * W[:, None] * W[None, :]
    return np.asarray(Psi.T @ (Psi.T @ K.T).T)


def kl_modes(pcoords, pconn, h, b, m):
    """The m largest eigenpairs (beta descending, a: m x n_vertices)."""
    C = covariance_matrix(pcoords, pconn, h, b)
    Mp = q1_mass(pcoords, pconn, h).toarray()
    n = C.shape[0]
    beta, V = sla.eigh(C, Mp, subset_by_index=[n - m, n - 1])
    beta, V = beta[::-1], V[:, ::-1]
    for l in range(m):
        v = V[:, l]
        first = np.nonzero(np.abs(v) >= 0.5 * np.abs(v).max())[0][0]
        if v[first] < 0:
            V[:, l] = -v
    return beta, V.T.copy()


def viscosity_fields(mesh, b, m):
    """KL modes on the pressure (Q1 vertex) lattice of the step mesh."""
    return kl_modes(mesh.pcoords, mesh.pconn, mesh.h, b, m)
