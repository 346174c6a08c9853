"""CPU checks of the native library without a GPU: it loads, exports every
symbol include/sgtt.h declares, and its host-side setup (mesh, Q2-Q1 CSR
matrices, chaos matrices, LSC pressure matrices) equals the oracle's
independent numpy assembly entry by entry."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.system import Problem
from synthetic_inputs import CONFIGS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1906_06785_amd import sgtt
    return sgtt


def test_library_exports_every_declared_symbol():
    sg = _lib()
    header = open(os.path.join(ROOT, "include", "sgtt.h")).read()
    declared = set(re.findall(r"\b(sgtt_[a-z_0-9]+)\s*\(", header))
    assert declared, "no declarations parsed"
    import ctypes
    lib = ctypes.CDLL(sg.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(sg.EXPORTED) == declared


def test_binding_structs_match_the_compiled_layout():
    # every ctypes mirror of a public struct has the size the library was
    # compiled with (a field added on one side only shows here)
    import ctypes
    sg = _lib()
    sizes = sg.abi_sizes()
    assert set(sizes) == set(sg.ABI_STRUCTS)
    for name, n in sizes.items():
        assert ctypes.sizeof(getattr(sg, name)) == n, name


def _rel(a, b):
    a = sp.csr_matrix(a)
    b = sp.csr_matrix(b)
    d = abs(a - b).max()
    return d / max(abs(b).max(), 1e-300)


@pytest.mark.parametrize("name", ["tiny", "tiny2", "C1"])
def test_host_matrices_match_oracle(name):
    sg = _lib()
    cfg = CONFIGS[name]
    hp = sg.HostProblem(cfg)
    P = Problem(cfg)
    assert (hp.n_s, hp.n_u, hp.n_p, hp.n_xi, hp.nt) == (P.n_s, P.n_u, P.n_p, P.n_xi, P.nt)
    assert _rel(hp.csr(0), P.M) < 1e-14
    assert _rel(hp.csr(1), P.A) < 1e-14
    assert _rel(hp.csr(2), P.B) < 1e-14
    Msi = sp.diags(1.0 / P.Mstar)
    assert _rel(hp.csr(3), P.B @ Msi @ P.Bt) < 1e-13
    assert _rel(hp.csr(4), P.B @ Msi @ P.Mb @ Msi @ P.Bt) < 1e-13
    assert _rel(hp.csr(5), P.B @ Msi @ P.Ab @ Msi @ P.Bt) < 1e-13
    # the PCD pressure-space matrices (eq. 5.17)
    from oracle import mesh as fem
    assert _rel(hp.csr(6), P.Mp) < 1e-14
    assert _rel(hp.csr(7), fem.pressure_stiffness(P.mesh)) < 1e-14
    G = hp.gpc(0)
    H = hp.gpc(1)
    assert np.abs(G - P.G).max() < 1e-14
    assert np.abs(H - P.H).max() < 1e-14
    assert np.abs(hp.gpc(2) - P.Gnu).max() < 1e-16
    coords, free, g = hp.mesh()
    assert np.abs(coords - P.mesh.coords).max() == 0.0
    assert np.array_equal(free, P.mesh.free)
    assert np.abs(g - P.g_all).max() == 0.0


def test_host_setup_full_size_counts():
    # 64x192 grid (h = 1/16), m = 4, p = 3
    sg = _lib()
    hp = sg.HostProblem(CONFIGS["C2"])
    assert (hp.n_u, hp.n_p, hp.n_xi, hp.nt) == (50368, 6641, 35, 128)


@pytest.mark.parametrize("name", ["tiny", "C1", "C2"])
def test_host_block_cyclic_reduction_solves_spatial_systems(name):
    """The op lists of the block cyclic reduction (the device passes' program)
    applied on the host solve the velocity matrix M/tau + nu A (eq. 5.23) and
    the pressure Laplacian B M*^-1 B^T (eq. 5.19) as a sparse direct solve of
    the oracle's own assembly does."""
    import scipy.sparse.linalg as spl
    sg = _lib()
    cfg = CONFIGS[name]
    hp = sg.HostProblem(cfg)
    P = Problem(cfg)
    rng = np.random.default_rng(7)
    tau, nu = 0.1, 1.0 / 50
    Msi = sp.diags(1.0 / P.Mstar)
    for which, A in ((0, (P.M / tau + nu * P.A).tocsc()), (1, (P.B @ Msi @ P.Bt).tocsc())):
        b = rng.standard_normal((A.shape[0], 5))
        x, npass = hp.bcr_solve(which, b, tau, nu)
        assert npass >= 1
        ref = spl.splu(A).solve(b)
        assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
        assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_host_block_cyclic_reduction_rejects_bad_arguments():
    sg = _lib()
    hp = sg.HostProblem(CONFIGS["tiny"])
    with pytest.raises(sg.SgttError):
        hp.bcr_solve(2, np.ones((hp.n_p, 1)))
    with pytest.raises(sg.SgttError):
        hp.bcr_solve(0, np.ones((hp.n_s, 1)), tau=0.0)


def test_host_kl_expansion_and_viscous_terms_match_oracle():
    # KL law (sec. 6.1): eigenpairs of the covariance, the sqrt 3 scaled chaos
    # matrices and the m + 1 stiffness matrices against the oracle's
    # independent assembly
    sg = _lib()
    from synthetic_inputs import CONFIGS
    cfg = CONFIGS["paper_kl"]
    hp = sg.HostProblem(cfg)
    P = Problem(cfg)
    beta, modes, nv = hp.kl()
    assert nv == cfg["m"] + 1 and len(beta) == cfg["m"]
    assert np.allclose(beta, P.kl_beta, rtol=1e-10)
    assert np.abs(modes - P.kl_modes).max() <= 1e-8 * np.abs(P.kl_modes).max()
    Gv = hp.gpc(3)
    for t, (Gl, Ab, _) in enumerate(P.visc):
        assert np.abs(Gv[t] - Gl).max() < 1e-14
        n = P.n_s
        assert _rel(hp.csr(8 + t), Ab[:n, :n]) < 1e-12
    # the other law has one viscous term, G_nu (x) A
    hp0 = sg.HostProblem(CONFIGS["C1"])
    assert hp0.kl()[2] == 1
    assert np.abs(hp0.gpc(3)[0] - hp0.gpc(2)).max() == 0.0
