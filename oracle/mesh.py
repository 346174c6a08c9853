"""Oracle: symmetric-step mesh and Q2-Q1 (Taylor-Hood) finite elements.

Test infrastructure only (see oracle/__init__.py).

Follows sec. 3.2 (basis ordering {(phi_i,0)},{(0,phi_i)}, eq. 3.7 for M, A, N,
eq. 3.8 for B) and sec. 6.1 (domain, boundary conditions, uniform squares of
size h).  Element integrals use 3x3 Gauss quadrature on every element.

Node numbering convention (shared with the GPU library by definition, not by
code): Q2 nodes live on the lattice x = (I, J) * h/2; free velocity nodes and
Q1 pressure nodes are each sorted by (x1, x2) lexicographically.  Velocity
dofs are [component x1 on free nodes; component x2 on free nodes].

Pins (tests/test_oracle_fem.py): the paper prints n_u = 2992, n_p = 461 at
h = 1/4; 1^T M 1 = area = 25; A 1 = 0; B applied to a constant field = 0;
B applied to u = (x1, 0) equals minus the row sums of the pressure mass matrix.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

_GP = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_GW = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def _q2_1d(t):
    return np.array([t * (t - 1) / 2, 1 - t * t, t * (t + 1) / 2])


def _q2_1d_d(t):
    return np.array([t - 0.5, -2 * t, t + 0.5])


def _q1_1d(t):
    return np.array([(1 - t) / 2, (1 + t) / 2])


@dataclass
class StepMesh:
    h: float
    L: float
    coords: np.ndarray      # (n_all, 2) velocity-node coordinates
    conn: np.ndarray        # (ne, 9) element -> velocity node, local k = a + 3 b
    pcoords: np.ndarray     # (n_p, 2)
    pconn: np.ndarray       # (ne, 4) element -> pressure node, local k = a + 2 b
    free: np.ndarray        # indices of free velocity nodes (sorted by x1, x2)
    dirichlet: np.ndarray   # indices of Dirichlet velocity nodes
    g1: np.ndarray          # x1-velocity Dirichlet values at `dirichlet` nodes (no ramp)

    @property
    def n_all(self):
        return self.coords.shape[0]

    @property
    def n_s(self):
        return self.free.size

    @property
    def n_u(self):
        return 2 * self.free.size

    @property
    def n_p(self):
        return self.pcoords.shape[0]


def build_mesh(h: float, L: float = 12.0) -> StepMesh:
    """Uniform-square mesh of the symmetric step (sec. 6.1, Fig. 6.1)."""
    q = int(round(1.0 / h))
    assert abs(q * h - 1.0) < 1e-12 and q % 2 == 0, "1/h must be an even integer"
    nL = int(round(q * L))
    assert abs(nL - q * L) < 1e-9
    elems = [(ec, er) for ec in range(-q, 0) for er in range(-q // 2, q // 2)]
    elems += [(ec, er) for ec in range(0, nL) for er in range(-q, q)]
    nodes = set()
    pnodes = set()
    for ec, er in elems:
        for b in range(3):
            for a in range(3):
                nodes.add((2 * ec + a, 2 * er + b))
        for b in range(2):
            for a in range(2):
                pnodes.add((2 * ec + 2 * a, 2 * er + 2 * b))
    nodes = sorted(nodes)
    pnodes = sorted(pnodes)
    nid = {n: i for i, n in enumerate(nodes)}
    pid = {n: i for i, n in enumerate(pnodes)}
    conn = np.array([[nid[(2 * ec + a, 2 * er + b)] for b in range(3) for a in range(3)]
                     for ec, er in elems], dtype=np.int64)
    pconn = np.array([[pid[(2 * ec + 2 * a, 2 * er + 2 * b)] for b in range(2) for a in range(2)]
                      for ec, er in elems], dtype=np.int64)
    IJ = np.array(nodes, dtype=np.int64)
    s = h / 2.0
    coords = IJ.astype(float) * s
    pcoords = np.array(pnodes, dtype=float) * s
    I, J = IJ[:, 0], IJ[:, 1]
    inflow = I == -2 * q
    inlet_wall = (np.abs(J) == q) & (I <= 0)
    channel_wall = np.abs(J) == 2 * q
    step_face = (I == 0) & (np.abs(J) >= q)
    is_dir = inflow | inlet_wall | channel_wall | step_face
    free = np.nonzero(~is_dir)[0]
    dirichlet = np.nonzero(is_dir)[0]
    x2 = coords[dirichlet, 1]
    g1 = np.where(inflow[dirichlet], 1.0 - 4.0 * x2 * x2, 0.0)
    return StepMesh(h, L, coords, conn, pcoords, pconn, free, dirichlet, g1)


def _q1_1d_d(t):
    return np.array([-0.5, 0.5])


def _ref_tables_q1():
    """Q1 basis derivatives at the 9 Gauss points: dpsi[g, k, d]."""
    dpsi = np.zeros((9, 4, 2))
    g = 0
    for jb in range(3):
        for ia in range(3):
            xi, eta = _GP[ia], _GP[jb]
            px, py = _q1_1d(xi), _q1_1d(eta)
            dx, dy = _q1_1d_d(xi), _q1_1d_d(eta)
            for b in range(2):
                for a in range(2):
                    dpsi[g, a + 2 * b, 0] = dx[a] * py[b]
                    dpsi[g, a + 2 * b, 1] = px[a] * dy[b]
            g += 1
    return dpsi


def _ref_tables():
    """Basis values / derivatives at the 9 Gauss points of the reference square."""
    phi = np.zeros((9, 9))      # [gauss point g, local node k]
    dphi = np.zeros((9, 9, 2))  # d/dxi, d/deta
    psi = np.zeros((9, 4))      # Q1
    wq = np.zeros(9)
    g = 0
    for jb in range(3):
        for ia in range(3):
            xi, eta = _GP[ia], _GP[jb]
            wq[g] = _GW[ia] * _GW[jb]
            lx, ly = _q2_1d(xi), _q2_1d(eta)
            dx, dy = _q2_1d_d(xi), _q2_1d_d(eta)
            for b in range(3):
                for a in range(3):
                    k = a + 3 * b
                    phi[g, k] = lx[a] * ly[b]
                    dphi[g, k, 0] = dx[a] * ly[b]
                    dphi[g, k, 1] = lx[a] * dy[b]
            px, py = _q1_1d(xi), _q1_1d(eta)
            for b in range(2):
                for a in range(2):
                    psi[g, a + 2 * b] = px[a] * py[b]
            g += 1
    return phi, dphi, psi, wq


def _assemble(conn_r, conn_c, Ke, nr, nc):
    ne, kr = conn_r.shape
    kc = conn_c.shape[1]
    rows = np.repeat(conn_r, kc, axis=1).ravel()
    cols = np.tile(conn_c, (1, kr)).ravel()
    vals = np.broadcast_to(Ke, (ne, kr, kc)).reshape(ne, kr * kc).ravel() if Ke.ndim == 2 \
        else Ke.reshape(ne, kr * kc).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(nr, nc))


def assemble(mesh: StepMesh):
    """Scalar Q2 mass M, unit-viscosity stiffness A, divergence blocks B1, B2
    (eq. 3.7-3.8, over ALL velocity nodes) and the Q1 pressure mass Mp."""
    phi, dphi, psi, wq = _ref_tables()
    h = mesh.h
    jac = (h / 2.0) ** 2
    Me = np.einsum("g,gi,gj->ij", wq, phi, phi) * jac
    Ae = np.einsum("g,gid,gjd->ij", wq, dphi, dphi)          # (2/h)^2 * jac = 1
    # [B_xk]_ij = -(psi_i, d phi_j / d x_k); d/dx = (2/h) d/dxi
    B1e = -np.einsum("g,gi,gj->ij", wq, psi, dphi[:, :, 0]) * jac * (2.0 / h)
    B2e = -np.einsum("g,gi,gj->ij", wq, psi, dphi[:, :, 1]) * jac * (2.0 / h)
    Mpe = np.einsum("g,gi,gj->ij", wq, psi, psi) * jac
    n, npp = mesh.n_all, mesh.n_p
    M = _assemble(mesh.conn, mesh.conn, Me, n, n)
    A = _assemble(mesh.conn, mesh.conn, Ae, n, n)
    B1 = _assemble(mesh.pconn, mesh.conn, B1e, npp, n)
    B2 = _assemble(mesh.pconn, mesh.conn, B2e, npp, n)
    Mp = _assemble(mesh.pconn, mesh.pconn, Mpe, npp, npp)
    return M, A, B1, B2, Mp


def convection(mesh: StepMesh, w1: np.ndarray, w2: np.ndarray):
    """[N(w)]_ij = (w . grad phi_j, phi_i) for a Q2 wind w = (w1, w2) given at
    all velocity nodes (eq. 3.7), assembled over all nodes."""
    phi, dphi, _, wq = _ref_tables()
    h = mesh.h
    W1 = w1[mesh.conn] @ phi.T   # (ne, 9 gauss) wind at quadrature points
    W2 = w2[mesh.conn] @ phi.T
    # jac * (2/h) = h/2
    Ne = np.einsum("g,eg,gi,gj->eij", wq, W1, phi, dphi[:, :, 0]) \
        + np.einsum("g,eg,gi,gj->eij", wq, W2, phi, dphi[:, :, 1])
    Ne *= h / 2.0
    return _assemble(mesh.conn, mesh.conn, Ne, mesh.n_all, mesh.n_all)


def pressure_stiffness(mesh: StepMesh):
    """Unit-viscosity Q1 stiffness on the pressure space, [A_p]_ij =
    (grad psi_j, grad psi_i) over the whole domain with no boundary condition
    imposed (the pressure convection-diffusion operator of sec. 5.1 is only
    multiplied with, never inverted, so its boundary treatment is a reading:
    natural conditions everywhere)."""
    _, _, _, wq = _ref_tables()
    dpsi = _ref_tables_q1()
    Ape = np.einsum("g,gid,gjd->ij", wq, dpsi, dpsi)   # (2/h)^2 * jac = 1
    return _assemble(mesh.pconn, mesh.pconn, Ape, mesh.n_p, mesh.n_p)


def pressure_convection(mesh: StepMesh, w1: np.ndarray, w2: np.ndarray):
    """[N_p(w)]_ij = (w . grad psi_j, psi_i) on the Q1 pressure space for a Q2
    wind (w1, w2) given at all velocity nodes (sec. 5.1, F_p)."""
    phi, _, psi, wq = _ref_tables()
    dpsi = _ref_tables_q1()
    h = mesh.h
    W1 = w1[mesh.conn] @ phi.T
    W2 = w2[mesh.conn] @ phi.T
    Ne = np.einsum("g,eg,gi,gj->eij", wq, W1, psi, dpsi[:, :, 0]) \
        + np.einsum("g,eg,gi,gj->eij", wq, W2, psi, dpsi[:, :, 1])
    Ne *= h / 2.0
    return _assemble(mesh.pconn, mesh.pconn, Ne, mesh.n_p, mesh.n_p)


def stiffness_weighted(mesh: StepMesh, a_vertex: np.ndarray):
    """[A(a)]_ij = (a grad phi_j, grad phi_i) over all velocity nodes for a
    coefficient field a given by its values at the Q1 (pressure) vertices
    and interpolated bilinearly to the Gauss points (eq. 3.7 with a
    spatially varying viscosity)."""
    phi, dphi, psi, wq = _ref_tables()
    Ag = a_vertex[mesh.pconn] @ psi.T                 # (ne, 9) coefficient at the Gauss points
    Ae = np.einsum("g,eg,gid,gjd->eij", wq, Ag, dphi, dphi)   # (2/h)^2 * jac = 1
    return _assemble(mesh.conn, mesh.conn, Ae, mesh.n_all, mesh.n_all)
