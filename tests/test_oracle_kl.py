"""Pins of the oracle's Karhunen-Loeve expansion (sec. 6.1) and of the
weighted stiffness matrices it feeds (eq. 3.6-3.7), against closed forms."""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import kl
from oracle import mesh as fem


def _exp_kernel_1d(a, b, count):
    """Eigenvalues of exp(-|x - y| / b) on an interval of length 2a, largest
    first: lambda = 2 b / (1 + b^2 w^2) with w from 1/b = w tan(w a) (even
    eigenfunctions) or w = -tan(w a) / b (odd ones), one root per branch of
    the tangent."""
    vals = []
    for k in range(count + 2):
        lo, hi = k * np.pi / a + 1e-12, (k + 0.5) * np.pi / a - 1e-12
        vals.append(brentq(lambda w: 1.0 / b - w * np.tan(w * a), lo, hi))
        lo, hi = (k + 0.5) * np.pi / a + 1e-12, (k + 1) * np.pi / a - 1e-12
        vals.append(brentq(lambda w: w + np.tan(w * a) / b, lo, hi))
    lam = sorted((2 * b / (1 + b * b * w * w) for w in vals), reverse=True)
    return np.array(lam[:count])


def _rectangle(nx, ny, h):
    # Q1 vertices of an nx x ny grid of squares of side h, vertex order
    # sorted by (x1, x2) like the step mesh's
    verts = [(i, j) for i in range(nx + 1) for j in range(ny + 1)]
    vid = {v: k for k, v in enumerate(verts)}
    pconn = np.array([[vid[(i + a, j + bb)] for bb in range(2) for a in range(2)]
                      for i in range(nx) for j in range(ny)])
    pcoords = np.array(verts, dtype=float) * h
    return pcoords, pconn


def test_kl_eigenvalues_on_a_rectangle_match_the_separable_closed_form():
    # c(x, y) = exp(-|x1-y1|/b) exp(-|x2-y2|/b) on [0, 2] x [0, 1]: the
    # eigenvalues are products of the 1-D ones (interval lengths 2 and 1)
    h, b = 1.0 / 16, 1.5
    pcoords, pconn = _rectangle(32, 16, h)
    beta, a = kl.kl_modes(pcoords, pconn, h, b, 4)
    l1 = _exp_kernel_1d(1.0, b, 4)
    l2 = _exp_kernel_1d(0.5, b, 4)
    want = np.sort(np.outer(l1, l2).ravel())[::-1][:4]
    assert np.allclose(beta, want, rtol=2e-3), (beta, want)
    # M_p-orthonormal modes and the sign convention
    Mp = kl.q1_mass(pcoords, pconn, h)
    G = a @ (Mp @ a.T)
    assert np.abs(G - np.eye(4)).max() < 1e-10
    for v in a:
        first = np.nonzero(np.abs(v) >= 0.5 * np.abs(v).max())[0][0]
        assert v[first] > 0


def test_weighted_stiffness_constant_and_linear_coefficient():
    m = fem.build_mesh(0.25, 12.0)
    _, A, _, _, _ = fem.assemble(m)
    one = np.ones(m.n_p)
    assert abs(fem.stiffness_weighted(m, one) - A).max() < 1e-13
    # a = x1 and u = x2 (exact in Q2): (a grad u, grad u) = int x1 dx over the
    # domain = 2 * 12^2 / 2 (channel) - 1 * 1 / 2 (inlet) = 143.5
    Ax = fem.stiffness_weighted(m, m.pcoords[:, 0])
    u = m.coords[:, 1]
    assert abs(u @ Ax @ u - 143.5) < 1e-10
