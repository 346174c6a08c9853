"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds problem descriptions (plain numbers) and seeded random
generators only.  It contains none of the method's arithmetic: no mesh, no
finite elements, no chaos matrices, no tensor-train algebra.  Both sides of the
parity tests draw their inputs from here and nowhere else.

Problem family (Elman & Su, sec. 6.1, Table 6.1): flow over a symmetric step,
inlet [-1,0]x[-1/2,1/2], channel [0,L]x[-1,1], uniform squares of size h,
Q2-Q1 elements, backward Euler with n_t steps of size tau, viscosity
nu(xi) = nu0 * (1 + nu_coef * sum_k xi_k / k^2) with xi_k iid U[-1,1],
Legendre chaos of total degree <= p in m variables.
"""
from __future__ import annotations

import numpy as np

# Grid labels such as "16x48" and "64x192" read as (4/h) x (12/h), i.e. the
# Q2 node lattice across the channel height by the element count along the
# channel: h = 1/4 and h = 1/16 respectively (pinned by the paper's dof counts
# n_u = 2992, n_p = 461 at h = 1/4).
CONFIGS = {
    # smallest sizes: the dense all-at-once matrix is formed and solved directly
    "tiny": dict(h=0.5, L=2.0, m=2, p=1, nt=3, tau=0.1, nu0=1.0 / 50, nu_coef=0.1,
                 ramp=10.0),
    "tiny2": dict(h=0.25, L=2.0, m=2, p=2, nt=4, tau=0.1, nu0=1.0 / 50, nu_coef=0.1,
                  ramp=10.0),
    # 16x48 grid (h=1/4), m=2, p=2 (6 chaos terms), nt=10, tau=0.1: Stokes system
    "C1": dict(h=0.25, L=12.0, m=2, p=2, nt=10, tau=0.1, nu0=1.0 / 50, nu_coef=0.1,
               ramp=10.0),
    # 64x192 grid (h=1/16), m=4, p=3 (35 chaos terms), nt=128, tau=0.05
    "C2": dict(h=1.0 / 16, L=12.0, m=4, p=3, nt=128, tau=0.05, nu0=1.0 / 50,
               nu_coef=0.1, ramp=10.0),
    # sizes of the paper's Table 6.1 (h = 2^-2, m = 3, degree 3 (n_xi = 20),
    # t_f = 1 with tau = 2^-6 (nt = 64), nu0 = 1/50), with this build's
    # viscosity law (relative amplitude nu_coef = sigma = 0.01)
    "paper": dict(h=0.25, L=12.0, m=3, p=3, nt=64, tau=1.0 / 64, nu0=1.0 / 50, nu_coef=0.01,
                  ramp=10.0),
    # the Table 6.1 problem with the paper's own viscosity: truncated KL
    # expansion of an exponential covariance (correlation length b = 4,
    # sigma = 0.01, m = 3 modes), xi_k ~ U[-sqrt 3, sqrt 3]
    "paper_kl": dict(h=0.25, L=12.0, m=3, p=3, nt=64, tau=1.0 / 64, nu0=1.0 / 50, nu_coef=0.01,
                     ramp=10.0, viscosity="kl", corr_length=4.0),
    # small KL problem for the oracle's pins and GPU parity (sigma raised so
    # that the random part is visible at FP64 tolerances)
    "tinykl": dict(h=0.5, L=2.0, m=2, p=2, nt=3, tau=0.1, nu0=1.0 / 50, nu_coef=0.3,
                   ramp=10.0, viscosity="kl", corr_length=4.0),
    "C1kl": dict(h=0.25, L=12.0, m=2, p=2, nt=10, tau=0.1, nu0=1.0 / 50, nu_coef=0.3,
                 ramp=10.0, viscosity="kl", corr_length=4.0),
    # intermediate size used by parity tests at a shape between C1 and C2
    "C1b": dict(h=0.125, L=12.0, m=3, p=2, nt=32, tau=0.05, nu0=1.0 / 50,
                nu_coef=0.1, ramp=10.0),
    # many chaos terms on a small mesh: m = 4, p = 4 gives n_xi = 70, more
    # columns per time step than one 64-wide pass of the mass product takes
    "tinyp4": dict(h=0.5, L=2.0, m=4, p=4, nt=3, tau=0.1, nu0=1.0 / 50, nu_coef=0.1,
                   ramp=10.0),
}

# Solver defaults (readings of the paper):
SOLVER_DEFAULTS = dict(
    tol=1e-8,            # exact relative residual target of one Picard-step solve
    eps_krylov=1e-6,     # TT truncation of Krylov / preconditioned vectors
    tol_cycle=1e-4,      # relative tolerance of one flexible-GMRES cycle
    restart=30,          # iterations per cycle
    max_cycles=8,
    inner_tol=1e-1,      # mean-matrix inner solve (paper: 1e-1 suffices)
    inner_eps=1e-3,      # truncation inside the inner solve
    inner_maxit=20,
    eps_conv=1e-3,       # truncation of the convection field (Table 6.2)
)


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_tt_cores(n1: int, n2: int, n3: int, r1: int, r2: int, seed: int,
                    decay: float = 0.0):
    """Random TT cores (paper convention): G1 (n1 x r1), G2 (r1 x n2 x r2),
    G3 (r2 x n3), entries N(0,1).  With decay>0 the rank columns are scaled by
    exp(-decay*index) so that the tensor has a decaying spectrum."""
    g = rng(seed)
    G1 = g.standard_normal((n1, r1))
    G2 = g.standard_normal((r1, n2, r2))
    G3 = g.standard_normal((r2, n3))
    if decay > 0.0:
        G1 = G1 * np.exp(-decay * np.arange(r1))[None, :]
        G3 = G3 * np.exp(-decay * np.arange(r2))[:, None]
    return G1, G2, G3


def random_tt_pair(nt: int, nxi: int, nu: int, np_: int, ranks_u, ranks_p,
                   seed: int, decay: float = 0.0):
    """A (velocity, pressure) pair of random TTs with the given ranks."""
    u = random_tt_cores(nt, nxi, nu, ranks_u[0], ranks_u[1], seed, decay)
    p = random_tt_cores(nt, nxi, np_, ranks_p[0], ranks_p[1], seed + 7919, decay)
    return u, p


def batch_configs(n: int = 64, seed: int = 0, small: bool = False):
    """Independent problems for batched solves, drawn in a fixed order by
    default_rng(seed): grid h, number of random variables m, chaos degree p,
    time steps n_t (tau = 0.05) and a mean viscosity nu0 log-uniform in
    [1/200, 1/20]; the viscosity law and inflow are those of CONFIGS.  small
    selects coarse grids and short horizons (for tests)."""
    g = rng(seed)
    hs = (0.25, 0.125) if small else (0.125, 1.0 / 12.0, 0.0625)
    ms = (2, 3) if small else (2, 3, 4)
    ps = (1, 2) if small else (2, 3)
    nts = (8, 16) if small else (32, 64, 128)
    out = []
    for _ in range(n):
        out.append(dict(h=float(g.choice(hs)), L=12.0, m=int(g.choice(ms)), p=int(g.choice(ps)),
                        nt=int(g.choice(nts)), tau=0.05,
                        nu0=float(np.exp(g.uniform(np.log(1 / 200), np.log(1 / 20)))), nu_coef=0.1,
                        ramp=10.0))
    return out


def smooth_prior(nt: int, nxi: int, tau: float, coords_free, n_p: int, ranks_u=(4, 17), ranks_p=(2, 3),
                 seed: int = 0, amplitude: float = 0.4, mean_only: bool = False):
    """A prior iterate (velocity TT over free nodes, pressure TT) shaped like
    a flow solution, with exact TT ranks: time columns ramp up like the
    inflow, (1 - exp(-10 t)) sin((a + 1) pi t / (2 T)); chaos slices decay
    with the chaos index (mean_only: only the first chaos mode, a
    deterministic prior); each spatial column is the velocity of a stream
    function sin(alpha (x1 + 1)) sin(beta (x2 + 1)) sampled at the free
    nodes (component 1 rows, then component 2 rows).  coords_free: (n_s, 2)
    free node coordinates.  Returns ((G1, G2, G3), (P1, P2, P3)) in the
    paper's core convention (G3: r2 x n)."""
    g = rng(seed)
    k1, k2 = ranks_u
    t = tau * np.arange(1, nt + 1)
    T = t[-1]
    ramp = 1.0 - np.exp(-10.0 * t)
    G1 = np.stack([amplitude * ramp * np.sin((a + 1) * np.pi * t / (2 * T)) for a in range(k1)], axis=1)
    decay = np.exp(-0.5 * np.arange(nxi))
    G2 = g.standard_normal((k1, nxi, k2)) * decay[None, :, None] / np.sqrt(k1 * k2)
    G2[:, 0, :] += 1.0 / np.sqrt(k1 * k2)
    if mean_only:
        G2[:, 1:, :] = 0.0
    x1, x2 = coords_free[:, 0], coords_free[:, 1]
    cols = []
    for b in range(k2):
        al = np.pi * (1 + b // 3) / 13.0
        be = np.pi * (1 + b % 3) / 2.0
        u1 = be * np.sin(al * (x1 + 1)) * np.cos(be * (x2 + 1))
        u2 = -al * np.cos(al * (x1 + 1)) * np.sin(be * (x2 + 1))
        v = np.concatenate([u1, u2])
        cols.append(v / np.abs(v).max())
    G3 = np.stack(cols, axis=0)
    j1, j2 = ranks_p
    P1 = np.stack([0.1 * ramp * np.cos(a * np.pi * t / T) for a in range(j1)], axis=1)
    P2 = g.standard_normal((j1, nxi, j2)) * decay[None, :, None]
    if mean_only:
        P2[:, 1:, :] = 0.0
    P3 = g.standard_normal((j2, n_p))
    return (G1, G2, G3), (P1, P2, P3)
