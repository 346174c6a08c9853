"""Pins of the oracle's mesh and Q2-Q1 assembly against facts the paper and
the mathematics fix (not against the oracle itself)."""
import json
import os

import numpy as np
import pytest

from oracle import mesh as fem

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_dof_counts_printed_in_paper():
    # sec. 6.1: h = 2^-2 gives n_u = 2992, n_p = 461
    m = fem.build_mesh(0.25, 12.0)
    assert m.n_u == GOLD["dofs_h_quarter"]["n_u"]
    assert m.n_p == GOLD["dofs_h_quarter"]["n_p"]


def test_all_at_once_size_printed_in_paper():
    from math import comb
    g = GOLD["all_at_once_size"]
    m = fem.build_mesh(0.25, 12.0)
    n_xi = comb(g["m"] + g["d_psi"], g["d_psi"])
    assert n_xi == g["n_xi"]
    assert g["n_t"] * n_xi * (m.n_u + m.n_p) == g["unknowns"]


@pytest.mark.parametrize("h,L,nu,npp", [(0.5, 2.0, 136, 31), (0.25, 2.0, 592, 101),
                                        (1.0 / 16, 12.0, 50368, 6641)])
def test_lattice_counts(h, L, nu, npp):
    # counts from enumerating the Q2 / Q1 node lattice by hand:
    # h=1/2,L=2: 20 elements; h=1/16: 64x192 grid
    m = fem.build_mesh(h, L)
    assert (m.n_u, m.n_p) == (nu, npp)


def test_mass_integrates_area():
    m = fem.build_mesh(0.25, 12.0)
    M, A, B1, B2, Mp = fem.assemble(m)
    one = np.ones(m.n_all)
    # |inlet| + |channel| = 1 * 1 + 12 * 2 = 25
    assert abs(one @ (M @ one) - 25.0) < 1e-12
    assert abs(np.ones(m.n_p) @ (Mp @ np.ones(m.n_p)) - 25.0) < 1e-12


def test_stiffness_kills_constants_and_divergence_of_fields():
    m = fem.build_mesh(0.25, 12.0)
    M, A, B1, B2, Mp = fem.assemble(m)
    one = np.ones(m.n_all)
    assert np.abs(A @ one).max() < 1e-13
    # div of a constant field is 0; div of (x1, 0) is 1, so B1 x1 = -(psi_i, 1)
    assert np.abs(B1 @ one).max() < 1e-14 and np.abs(B2 @ one).max() < 1e-14
    rowsum = Mp @ np.ones(m.n_p)
    assert np.abs(B1 @ m.coords[:, 0] + rowsum).max() < 1e-13
    assert np.abs(B2 @ m.coords[:, 1] + rowsum).max() < 1e-13
    # Laplacian of x1^2 is 2: (grad x1^2, grad phi_i) = -(2, phi_i) + boundary;
    # check on interior nodes only (natural boundary terms vanish there)
    x = m.coords[:, 0]
    interior = np.ones(m.n_all, bool)
    interior[m.dirichlet] = False
    interior &= (np.abs(m.coords[:, 0] - 12.0) > 1e-12) & (np.abs(m.coords[:, 0] + 1.0) > 1e-12)
    lhs = A @ (x * x)
    rhs = -2.0 * (M @ one)
    assert np.abs((lhs - rhs)[interior]).max() < 1e-12


def test_convection_skew_up_to_boundary():
    # (w.grad phi_j, phi_i) + (w.grad phi_i, phi_j) = boundary integral of
    # (w.n) phi_i phi_j for a constant (divergence-free) w: zero whenever one of
    # the two nodes is off the boundary.
    m = fem.build_mesh(0.5, 2.0)
    w1 = np.full(m.n_all, 1.0)
    w2 = np.full(m.n_all, 0.3)
    N = fem.convection(m, w1, w2).toarray()
    S = N + N.T
    x1, x2 = m.coords[:, 0], m.coords[:, 1]
    on_bd = np.zeros(m.n_all, bool)
    on_bd[m.dirichlet] = True
    on_bd |= np.abs(x1 - 2.0) < 1e-12
    off = ~on_bd
    assert np.abs(S[off, :]).max() < 1e-14
    assert np.abs(S[:, off]).max() < 1e-14
    # outflow boundary x1 = L: w.n = 1 -> S restricted to outflow nodes = Q2
    # boundary mass on that edge, whose total is the edge length 2
    out = np.abs(x1 - 2.0) < 1e-12
    assert abs(S[np.ix_(out, out)].sum() - 2.0) < 1e-12


def test_convection_orientation_constant_wind():
    # eq. 3.7: [N(w)]_ij = (w . grad phi_j, phi_i), so N(w) applied to the
    # nodal values of a Q2 function v gives the moments (w . grad v, phi_i).
    # For constant w and v = x1 (or x2) that is w1 (1, phi_i) = w1 (M 1)_i on
    # EVERY row; the transposed matrix gives (w . grad phi_i, x1) instead,
    # which differs on every row.
    m = fem.build_mesh(0.5, 2.0)
    M, A, B1, B2, Mp = fem.assemble(m)
    one = np.ones(m.n_all)
    x1, x2 = m.coords[:, 0], m.coords[:, 1]
    w1, w2 = 0.7, -0.4
    N = fem.convection(m, np.full(m.n_all, w1), np.full(m.n_all, w2))
    assert np.abs(N @ x1 - w1 * (M @ one)).max() < 1e-14
    assert np.abs(N @ x2 - w2 * (M @ one)).max() < 1e-14
    assert np.abs(N.T @ x1 - w1 * (M @ one)).max() > 1e-3
    # quadratic v = x1^2: w . grad v = 2 w1 x1, a Q2 function
    assert np.abs(N @ (x1 * x1) - 2 * w1 * (M @ x1)).max() < 1e-13


def test_convection_orientation_solenoidal_wind():
    # non-constant divergence-free wind w = (x2, x1): w . grad x1 = x2 and
    # w . grad x2 = x1, so N x1 = M x2 and N x2 = M x1 row by row; the Q2
    # wind is exact and 3x3 Gauss integrates the products exactly.
    m = fem.build_mesh(0.25, 2.0)
    M, A, B1, B2, Mp = fem.assemble(m)
    x1, x2 = m.coords[:, 0], m.coords[:, 1]
    N = fem.convection(m, x2.copy(), x1.copy())
    assert np.abs(N @ x1 - M @ x2).max() < 1e-13
    assert np.abs(N @ x2 - M @ x1).max() < 1e-13
    # and for v = x1 x2: w . grad v = x2^2 + x1^2
    assert np.abs(N @ (x1 * x2) - M @ (x1 * x1 + x2 * x2)).max() < 1e-13


def test_pressure_stiffness_kills_constants_and_integrates_gradients():
    # Q1 stiffness on the pressure space (sec. 5.1): A_p 1 = 0, and for the Q1
    # fields x1 and x2, (grad x_k, grad x_k) = area = 25 and the cross term 0
    m = fem.build_mesh(0.25, 12.0)
    Ap = fem.pressure_stiffness(m)
    assert np.abs(Ap @ np.ones(m.n_p)).max() < 1e-13
    x1, x2 = m.pcoords[:, 0], m.pcoords[:, 1]
    assert abs(x1 @ Ap @ x1 - 25.0) < 1e-11
    assert abs(x2 @ Ap @ x2 - 25.0) < 1e-11
    assert abs(x1 @ Ap @ x2) < 1e-11


def test_pressure_convection_orientation_and_skew():
    # [N_p(w)]_ij = (w . grad psi_j, psi_i): for w = (1, 0) the pressure field
    # x1 has w . grad x1 = 1, so N_p(w) x1 = M_p 1 on every row (a transposed
    # N_p fails this); and N_p + N_p^T = boundary terms of the divergence-free
    # w, zero on rows of nodes off the faces where w . n != 0 (inflow x1 = -1,
    # outflow x1 = 12 and the step faces x1 = 0, |x2| >= 1/2)
    m = fem.build_mesh(0.25, 12.0)
    _, _, _, _, Mp = fem.assemble(m)
    one = np.ones(m.n_all)
    Np = fem.pressure_convection(m, one, 0.0 * one)
    x1 = m.pcoords[:, 0]
    assert np.abs(Np @ x1 - Mp @ np.ones(m.n_p)).max() < 1e-13
    S = (Np + Np.T).tocsr()
    px1, px2 = m.pcoords[:, 0], m.pcoords[:, 1]
    step_face = (np.abs(px1) < 1e-12) & (np.abs(px2) >= 0.5 - 1e-12)
    interior = (np.abs(px1 + 1.0) > 1e-12) & (np.abs(px1 - 12.0) > 1e-12) & ~step_face
    assert np.abs(S[interior].toarray()).max() < 1e-13
    # a wind (0, 1): w . grad x2 = 1
    Np2 = fem.pressure_convection(m, 0.0 * one, one)
    assert np.abs(Np2 @ m.pcoords[:, 1] - Mp @ np.ones(m.n_p)).max() < 1e-13
