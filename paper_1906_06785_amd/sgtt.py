"""Python binding of the sgtt C ABI (include/sgtt.h).

Argument marshalling only: every step of the solver runs in the HIP library
(libsgtt.so).  PyTorch provides device memory and the stream.  If the
library is missing, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgtt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"sgtt native library not built: {LIB_PATH} (run paper_1906_06785_amd.build)")
# PyTorch owns device memory and streams; load its HIP runtime first so that
# libsgtt.so binds to the same libamdhip64.so.7 (one HIP runtime per process).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

SGTT_OK = 0
SGTT_W_NOT_CONVERGED = 1
SGTT_E_RANK_CAP = -4


class SgttTT(C.Structure):
    _fields_ = [("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int), ("r1", C.c_int), ("r2", C.c_int),
                ("cap1", C.c_int), ("cap2", C.c_int), ("core1", C.c_void_p), ("core2", C.c_void_p),
                ("core3", C.c_void_p), ("dtype", C.c_int), ("d_ranks", C.c_void_p)]


SGTT_DTYPE_F64 = 0


class SgttPair(C.Structure):
    _fields_ = [("u", SgttTT), ("p", SgttTT)]


class ProblemDesc(C.Structure):
    _fields_ = [("h", C.c_double), ("L", C.c_double), ("m", C.c_int), ("p", C.c_int), ("nt", C.c_int),
                ("tau", C.c_double), ("nu0", C.c_double), ("nu_coef", C.c_double), ("ramp", C.c_double),
                ("eps_conv", C.c_double), ("eps_rhs", C.c_double), ("viscosity_law", C.c_int),
                ("corr_length", C.c_double)]


class SystemInfo(C.Structure):
    _fields_ = [("n_s", C.c_int), ("n_u", C.c_int), ("n_p", C.c_int), ("n_xi", C.c_int), ("nt", C.c_int),
                ("n_all", C.c_int), ("conv_r1", C.c_int), ("conv_r2", C.c_int), ("rhs_r1u", C.c_int),
                ("rhs_r2u", C.c_int), ("rhs_r1p", C.c_int), ("rhs_r2p", C.c_int), ("setup_seconds", C.c_double),
                ("rhs_norm", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("eps_krylov", C.c_double), ("tol_cycle", C.c_double),
                ("restart", C.c_int), ("max_cycles", C.c_int), ("inner_tol", C.c_double),
                ("inner_eps", C.c_double), ("inner_maxit", C.c_int), ("verbose", C.c_int),
                ("outer_explicit", C.c_int), ("inner_explicit", C.c_int), ("relax", C.c_int),
                ("precision", C.c_int), ("inner_rhs_eps", C.c_double), ("cycle_rhs_factor", C.c_double),
                ("inner_mode", C.c_int), ("schur", C.c_int), ("graph", C.c_int)]


PICARD_MAX_STEPS = 16


class PicardOpts(C.Structure):
    _fields_ = [("max_steps", C.c_int), ("tol_picard", C.c_double), ("eps_soln", C.c_double),
                ("solve", SolveOpts), ("update_mode", C.c_int)]


class PicardStats(C.Structure):
    _n = PICARD_MAX_STEPS + 1
    _fields_ = [("steps", C.c_int), ("nonlinear_residual", C.c_double * _n), ("linear_residual", C.c_double * _n),
                ("outer_iters", C.c_int * _n), ("inner_iters", C.c_int * _n), ("solve_seconds", C.c_double * _n),
                ("assemble_seconds", C.c_double * (_n + 1)), ("rank_u", (C.c_int * 2) * _n),
                ("rank_p", (C.c_int * 2) * _n), ("seconds", C.c_double),
                ("stored_rank_u", (C.c_int * 2) * _n), ("stored_rank_p", (C.c_int * 2) * _n)]

    def as_dict(self):
        n = self.steps + 1
        return {"steps": self.steps, "nonlinear_residual": list(self.nonlinear_residual[:n]),
                "linear_residual": list(self.linear_residual[:n]), "outer_iters": list(self.outer_iters[:n]),
                "inner_iters": list(self.inner_iters[:n]), "solve_seconds": list(self.solve_seconds[:n]),
                "assemble_seconds": list(self.assemble_seconds[:n + 1]),
                "rank_u": [tuple(r) for r in self.rank_u[:n]], "rank_p": [tuple(r) for r in self.rank_p[:n]],
                "stored_rank_u": [tuple(r) for r in self.stored_rank_u[:n]],
                "stored_rank_p": [tuple(r) for r in self.stored_rank_p[:n]],
                "seconds": self.seconds}


class IterRecord(C.Structure):
    _fields_ = [("cycle", C.c_int), ("iter", C.c_int), ("rel", C.c_double), ("rank_v_u", C.c_int * 2),
                ("rank_v_p", C.c_int * 2), ("rank_z_u", C.c_int * 2), ("rank_z_p", C.c_int * 2),
                ("seconds", C.c_double)]

    def as_dict(self):
        return {"cycle": self.cycle, "iter": self.iter, "rel": self.rel, "rank_v_u": tuple(self.rank_v_u),
                "rank_v_p": tuple(self.rank_v_p), "rank_z_u": tuple(self.rank_z_u),
                "rank_z_p": tuple(self.rank_z_p), "seconds": self.seconds}


class MemoryInfo(C.Structure):
    _fields_ = [("arena_bytes", C.c_size_t), ("arena_peak_bytes", C.c_size_t), ("cached_bytes", C.c_size_t),
                ("device_allocs", C.c_long)]


class SolveStats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("outer_iters", C.c_int), ("inner_iters", C.c_int),
                ("rel_residual", C.c_double), ("seconds", C.c_double), ("max_rank_krylov_u", C.c_int),
                ("max_rank_krylov_p", C.c_int), ("roundings", C.c_int), ("t_apply", C.c_double),
                ("t_round", C.c_double), ("t_precond", C.c_double), ("t_residual", C.c_double),
                ("learned_calls", C.c_int), ("learned_fallback", C.c_int), ("device_allocs", C.c_long),
                ("f32_applications", C.c_int), ("graph_launches", C.c_long)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_sig = {
    "sgtt_version": (C.c_char_p, []),
    "sgtt_context_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "sgtt_context_destroy": (C.c_int, [_P]),
    "sgtt_context_reserve": (C.c_int, [_P, C.c_size_t]),
    "sgtt_context_memory": (C.c_int, [_P, C.POINTER(MemoryInfo)]),
    "sgtt_last_error": (C.c_char_p, [_P]),
    "sgtt_assemble": (C.c_int, [_P, C.POINTER(ProblemDesc), C.POINTER(SgttPair), C.POINTER(_P)]),
    "sgtt_system_destroy": (C.c_int, [_P]),
    "sgtt_system_info_get": (C.c_int, [_P, C.POINTER(SystemInfo)]),
    "sgtt_rhs": (C.c_int, [_P, C.POINTER(SgttPair)]),
    "sgtt_apply": (C.c_int, [_P, C.POINTER(SgttPair), C.POINTER(SgttPair), C.c_double]),
    "sgtt_precondition": (C.c_int, [_P, C.POINTER(SgttPair), C.POINTER(SgttPair), C.POINTER(SolveOpts),
                                    C.POINTER(SolveStats)]),
    "sgtt_round": (C.c_int, [_P, C.POINTER(SgttTT), C.c_double, C.c_int]),
    "sgtt_dot": (C.c_int, [_P, C.POINTER(SgttPair), C.POINTER(SgttPair), C.POINTER(C.c_double)]),
    "sgtt_axpby": (C.c_int, [_P, C.c_double, C.POINTER(SgttPair), C.c_double, C.POINTER(SgttPair)]),
    "sgtt_solve": (C.c_int, [_P, C.POINTER(SgttPair), C.POINTER(SgttPair), C.POINTER(SolveOpts),
                             C.POINTER(SolveStats)]),
    "sgtt_residual": (C.c_int, [_P, C.POINTER(SgttPair), C.POINTER(SgttPair), C.POINTER(C.c_double)]),
    "sgtt_solve_history": (C.c_int, [_P, C.c_int, C.POINTER(IterRecord), C.POINTER(C.c_int)]),
    "sgtt_gemm": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_double, _P, C.c_long, _P, C.c_long, C.c_double,
                            _P, C.c_long]),
    "sgtt_pair_save": (C.c_int, [_P, C.POINTER(SgttPair), C.c_char_p]),
    "sgtt_pair_load": (C.c_int, [_P, C.c_char_p, C.POINTER(SgttPair)]),
    "sgtt_pair_file_write_host": (C.c_int, [C.c_char_p, C.POINTER(C.c_int), C.POINTER(C.c_void_p)]),
    "sgtt_pair_file_info": (C.c_int, [C.c_char_p, C.POINTER(C.c_int)]),
    "sgtt_mlp_save": (C.c_int, [_P, C.c_char_p]),
    "sgtt_mlp_load": (C.c_int, [_P, C.c_char_p]),
    "sgtt_mlp_file_write_host": (C.c_int, [C.c_char_p, C.c_int, C.c_int, _P]),
    "sgtt_mlp_file_info": (C.c_int, [C.c_char_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_long)]),
    "sgtt_mlp_file_read_host": (C.c_int, [C.c_char_p, C.c_int, C.c_int, _P]),
    "sgtt_pair_file_read_host": (C.c_int, [C.c_char_p, C.POINTER(C.c_int), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_int)]),
    "sgtt_expand": (C.c_int, [_P, C.POINTER(SgttTT), _P]),
    "sgtt_hessenberg_lsq": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int, C.c_double, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
    "sgtt_profile_enable": (C.c_int, [_P, C.c_int]),
    "sgtt_profile_enable_classes": (C.c_int, [_P, C.c_uint]),
    "sgtt_profile_sample": (C.c_int, [_P, C.c_int]),
    "sgtt_abi_sizes": (C.c_int, [C.POINTER(C.c_long), C.c_int]),
    "sgtt_profile_read": (C.c_int, [_P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_long), C.POINTER(C.c_int)]),
    "sgtt_profile_class_name": (C.c_char_p, [C.c_int]),
    "sgtt_picard": (C.c_int, [_P, C.POINTER(ProblemDesc), C.POINTER(PicardOpts), C.POINTER(SgttPair),
                              C.POINTER(PicardStats)]),
    "sgtt_solve_batched": (C.c_int, [C.POINTER(_P), C.c_int, C.POINTER(C.POINTER(SgttPair)),
                                     C.POINTER(C.POINTER(SgttPair)), C.POINTER(SolveOpts), C.POINTER(SolveStats),
                                     C.POINTER(C.c_int)]),
    "sgtt_mlp_create": (C.c_int, [_P, C.c_int, C.c_int, C.c_long, C.c_uint, C.POINTER(_P)]),
    "sgtt_mlp_destroy": (C.c_int, [_P]),
    "sgtt_mlp_size": (C.c_int, [_P, C.POINTER(C.c_long), C.POINTER(C.c_long)]),
    "sgtt_mlp_set_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "sgtt_mlp_get_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "sgtt_mlp_forward": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_float)]),
    "sgtt_mlp_forward_f16": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_float)]),
    "sgtt_mlp_loss_grad": (C.c_int, [_P, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int,
                                     C.POINTER(C.c_double), C.POINTER(C.c_float)]),
    "sgtt_mlp_train": (C.c_int, [_P, C.c_int, C.c_int, C.c_double, C.c_uint, C.POINTER(C.c_double)]),
    "sgtt_mlp_add_pairs": (C.c_int, [_P, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_long,
                                     C.POINTER(C.c_long)]),
    "sgtt_mlp_collect": (C.c_int, [_P, _P]),
    "sgtt_mlp_attach": (C.c_int, [_P, _P]),
    "sgtt_residual_tensor": (C.c_int, [_P, C.POINTER(SgttPair), C.POINTER(SgttPair), _P, _P,
                                       C.POINTER(C.c_double)]),
    "sgtt_profile_read_regions": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "sgtt_profile_region_name": (C.c_char_p, [C.c_int]),
    "sgtt_host_problem_create": (C.c_int, [C.POINTER(ProblemDesc), C.POINTER(_P)]),
    "sgtt_host_problem_destroy": (C.c_int, [_P]),
    "sgtt_host_sizes": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "sgtt_host_csr": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "sgtt_host_gpc": (C.c_int, [_P, C.c_int, C.POINTER(C.c_double)]),
    "sgtt_host_kl": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]),
    "sgtt_host_mesh": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "sgtt_bcr_apply": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "sgtt_bcr_variant_count": (C.c_int, []),
    "sgtt_bcr_apply_noalloc": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "sgtt_host_bcr_solve": (C.c_int, [_P, C.c_int, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig.keys())


class SgttError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sgtt error {code}: {msg}")
        self.code = code


def make_desc(cfg: dict, eps_conv=1e-3, eps_rhs=1e-6) -> ProblemDesc:
    return ProblemDesc(float(cfg["h"]), float(cfg.get("L", 12.0)), int(cfg["m"]), int(cfg["p"]), int(cfg["nt"]),
                       float(cfg["tau"]), float(cfg["nu0"]), float(cfg["nu_coef"]), float(cfg.get("ramp", 10.0)),
                       float(cfg.get("eps_conv", eps_conv)), float(cfg.get("eps_rhs", eps_rhs)),
                       1 if cfg.get("viscosity", "power") == "kl" else 0, float(cfg.get("corr_length", 4.0)))


def make_opts(**kw) -> SolveOpts:
    d = dict(tol=1e-8, eps_krylov=1e-6, tol_cycle=1e-4, restart=30, max_cycles=8, inner_tol=1e-1,
             inner_eps=1e-3, inner_maxit=20, verbose=0, outer_explicit=1, inner_explicit=0, relax=0, precision=0,
             inner_rhs_eps=0.0, cycle_rhs_factor=0.0, inner_mode=0, schur=0, graph=0)
    d.update(kw)
    return SolveOpts(d["tol"], d["eps_krylov"], d["tol_cycle"], int(d["restart"]), int(d["max_cycles"]),
                     d["inner_tol"], d["inner_eps"], int(d["inner_maxit"]), int(d["verbose"]),
                     int(d["outer_explicit"]), int(d["inner_explicit"]), int(d["relax"]), int(d["precision"]),
                     float(d["inner_rhs_eps"]), float(d["cycle_rhs_factor"]), int(d["inner_mode"]),
                     int(d["schur"]), int(d["graph"]))


# ------------------------------------------------------------------ host-only
class HostProblem:
    """Host-side setup of the library (no device calls)."""

    def __init__(self, cfg: dict):
        self._h = _P()
        d = make_desc(cfg)
        rc = _lib.sgtt_host_problem_create(C.byref(d), C.byref(self._h))
        if rc != 0:
            raise SgttError(rc, "host problem setup failed")
        s = (C.c_int * 6)()
        _lib.sgtt_host_sizes(self._h, s)
        self.n_s, self.n_u, self.n_p, self.n_xi, self.nt, self.n_all = list(s)
        self.m = int(cfg["m"])

    def csr(self, which: int):
        import scipy.sparse as sp
        nr, nc, nnz = C.c_int(), C.c_int(), C.c_int()
        _lib.sgtt_host_csr(self._h, which, C.byref(nr), C.byref(nc), C.byref(nnz), None, None, None)
        rp = np.zeros(nr.value + 1, np.int32)
        col = np.zeros(nnz.value, np.int32)
        val = np.zeros(nnz.value, np.float64)
        _lib.sgtt_host_csr(self._h, which, None, None, None, rp.ctypes.data_as(C.POINTER(C.c_int)),
                           col.ctypes.data_as(C.POINTER(C.c_int)), val.ctypes.data_as(C.POINTER(C.c_double)))
        return sp.csr_matrix((val, col, rp), shape=(nr.value, nc.value))

    def bcr_solve(self, which: int, b, tau: float = 0.0, nu: float = 0.0):
        """Host application of the block cyclic reduction factor (which 0:
        M/tau + nu A on the velocity slabs, 1: B M*^-1 B^T on the pressure
        slabs) to the columns of b (n x ncols); returns (x, number of passes)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        if b.ndim == 1:
            b = b[:, None]
        if which in (0, 1) and (b.ndim != 2 or b.shape[0] != (self.n_s if which == 0 else self.n_p)):
            raise ValueError(f"b has shape {b.shape}; expected {self.n_s if which == 0 else self.n_p} rows")
        x = np.zeros_like(b)
        npass = C.c_int()
        rc = _lib.sgtt_host_bcr_solve(self._h, which, tau, nu, b.shape[1], b.ctypes.data_as(C.POINTER(C.c_double)),
                                      x.ctypes.data_as(C.POINTER(C.c_double)), C.byref(npass))
        if rc != 0:
            raise SgttError(rc, "host block cyclic reduction failed")
        return x, npass.value

    def gpc(self, which: int):
        n = self.n_xi
        nv = self.kl()[2] if which == 3 else 0
        size = {0: (self.m + 1) * n * n, 1: n ** 3, 2: n * n, 3: nv * n * n}[which]
        out = np.zeros(size)
        _lib.sgtt_host_gpc(self._h, which, out.ctypes.data_as(C.POINTER(C.c_double)))
        shape = {0: (self.m + 1, n, n), 1: (n, n, n), 2: (n, n), 3: (nv, n, n)}[which]
        return out.reshape(shape)

    def kl(self):
        """(beta, modes (m x n_p), number of viscous terms) of the KL law;
        empty arrays for the other law."""
        nm, nv = C.c_int(), C.c_int()
        _lib.sgtt_host_kl(self._h, C.byref(nm), C.byref(nv), None, None)
        beta = np.zeros(nm.value)
        modes = np.zeros((nm.value, self.n_p))
        _lib.sgtt_host_kl(self._h, None, None, beta.ctypes.data_as(C.POINTER(C.c_double)),
                          modes.ctypes.data_as(C.POINTER(C.c_double)))
        return beta, modes, nv.value

    def mesh(self):
        coords = np.zeros(2 * self.n_all)
        free = np.zeros(self.n_s, np.int32)
        g = np.zeros(2 * self.n_all)
        _lib.sgtt_host_mesh(self._h, coords.ctypes.data_as(C.POINTER(C.c_double)),
                            free.ctypes.data_as(C.POINTER(C.c_int)), g.ctypes.data_as(C.POINTER(C.c_double)))
        return coords.reshape(-1, 2), free, g

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sgtt_host_problem_destroy(self._h)
            self._h = None


# ------------------------------------------------------------------ device
def _torch():
    import torch
    return torch


class TTBuf:
    """Device buffers (torch, float64) for one TT with fixed capacities."""

    def __init__(self, n1, n2, n3, cap1, cap2, device="cuda:0"):
        torch = _torch()
        self.n1, self.n2, self.n3, self.cap1, self.cap2 = n1, n2, n3, cap1, cap2
        self.c1 = torch.zeros(n1 * cap1, dtype=torch.float64, device=device)
        self.c2 = torch.zeros(cap1 * n2 * cap2, dtype=torch.float64, device=device)
        self.c3 = torch.zeros(n3 * cap2, dtype=torch.float64, device=device)
        # live ranks mirrored in device memory by every call that writes this TT
        self.d_ranks = torch.zeros(2, dtype=torch.int32, device=device)
        self.r1 = self.r2 = 1

    def struct(self) -> SgttTT:
        return SgttTT(self.n1, self.n2, self.n3, self.r1, self.r2, self.cap1, self.cap2, self.c1.data_ptr(),
                      self.c2.data_ptr(), self.c3.data_ptr(), SGTT_DTYPE_F64, self.d_ranks.data_ptr())

    def update(self, s: SgttTT):
        self.r1, self.r2 = s.r1, s.r2

    def set_cores(self, G1, G2, G3):
        """Paper-convention cores G1 (n1 x r1), G2 (r1 x n2 x r2), G3 (r2 x n3)."""
        torch = _torch()
        r1, r2 = G1.shape[1], G3.shape[0]
        if r1 > self.cap1 or r2 > self.cap2:
            raise ValueError("ranks exceed capacity")
        self.c1[: self.n1 * r1].copy_(torch.from_numpy(np.ascontiguousarray(G1).ravel()))
        self.c2[: r1 * self.n2 * r2].copy_(torch.from_numpy(np.ascontiguousarray(G2).ravel()))
        self.c3[: self.n3 * r2].copy_(torch.from_numpy(np.ascontiguousarray(G3.T).ravel()))
        self.r1, self.r2 = r1, r2
        return self

    def cores(self):
        r1, r2 = self.r1, self.r2
        G1 = self.c1[: self.n1 * r1].cpu().numpy().reshape(self.n1, r1)
        G2 = self.c2[: r1 * self.n2 * r2].cpu().numpy().reshape(r1, self.n2, r2)
        G3 = self.c3[: self.n3 * r2].cpu().numpy().reshape(self.n3, r2).T.copy()
        return G1, G2, G3


class PairBuf:
    def __init__(self, nt, nxi, nu, npp, cap1=64, cap2=256, capp1=None, capp2=None, device="cuda:0"):
        self.u = TTBuf(nt, nxi, nu, cap1, cap2, device)
        self.p = TTBuf(nt, nxi, npp, capp1 or cap1, capp2 or cap2, device)

    def struct(self) -> SgttPair:
        return SgttPair(self.u.struct(), self.p.struct())

    def update(self, s: SgttPair):
        self.u.update(s.u)
        self.p.update(s.p)

    def set(self, pair):
        self.u.set_cores(*pair[0])
        self.p.set_cores(*pair[1])
        return self

    def cores(self):
        return self.u.cores(), self.p.cores()

    @property
    def ranks(self):
        return (self.u.r1, self.u.r2), (self.p.r1, self.p.r2)


class Context:
    def __init__(self, device: int = 0, use_torch_stream: bool = True):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("sgtt needs a GPU (no HIP device visible)")
        self.device = device
        stream = torch.cuda.current_stream(device).cuda_stream if use_torch_stream else None
        self._c = _P()
        rc = _lib.sgtt_context_create(device, stream, C.byref(self._c))
        if rc != 0:
            raise SgttError(rc, "context create failed: " + _lib.sgtt_last_error(None).decode())

    def check(self, rc):
        if rc < 0:
            raise SgttError(rc, _lib.sgtt_last_error(self._c).decode())
        return rc

    def reserve(self, nbytes: int):
        """Allocate the context's device arena up front (sgtt_context_reserve)."""
        self.check(_lib.sgtt_context_reserve(self._c, int(nbytes)))

    def memory(self) -> dict:
        m = MemoryInfo()
        self.check(_lib.sgtt_context_memory(self._c, C.byref(m)))
        return {k: getattr(m, k) for k, _ in m._fields_}

    def round(self, buf: TTBuf, eps: float, max_rank: int = 0):
        s = buf.struct()
        self.check(_lib.sgtt_round(self._c, C.byref(s), eps, max_rank))
        buf.update(s)
        return buf

    def dot(self, x: PairBuf, y: PairBuf) -> float:
        out = C.c_double()
        sx, sy = x.struct(), y.struct()
        self.check(_lib.sgtt_dot(self._c, C.byref(sx), C.byref(sy), C.byref(out)))
        return out.value

    def axpby(self, alpha, x: PairBuf, beta, y: PairBuf):
        sx, sy = x.struct(), y.struct()
        self.check(_lib.sgtt_axpby(self._c, alpha, C.byref(sx), beta, C.byref(sy)))
        y.update(sy)
        return y

    def expand(self, buf: TTBuf):
        torch = _torch()
        out = torch.empty(buf.n1 * buf.n2 * buf.n3, dtype=torch.float64, device=buf.c1.device)
        s = buf.struct()
        self.check(_lib.sgtt_expand(self._c, C.byref(s), out.data_ptr()))
        return out.reshape(buf.n1, buf.n2, buf.n3)

    def profile(self, enable: bool, classes=None):
        """Switch the event profiler; classes (iterable of class names) limits
        it to those kernel classes."""
        if classes is None:
            self.check(_lib.sgtt_profile_enable(self._c, int(enable)))
            return
        names = [_lib.sgtt_profile_class_name(i).decode() for i in range(16)]
        mask = 0
        for cname in classes:
            mask |= 1 << names.index(cname)
        self.check(_lib.sgtt_profile_enable_classes(self._c, mask if enable else 0))

    def gemm(self, A, B, C=None, alpha=1.0, beta=0.0):
        """C = alpha A B + beta C with the library's FP64 product kernels;
        A, B, C row-major float64 device tensors (C created when None)."""
        torch = _torch()
        m, k = A.shape
        n = B.shape[1]
        if C is None:
            C = torch.zeros((m, n), dtype=torch.float64, device=A.device)
        self.check(_lib.sgtt_gemm(self._c, m, n, k, float(alpha), A.data_ptr(), A.stride(0), B.data_ptr(),
                                  B.stride(0), float(beta), C.data_ptr(), C.stride(0)))
        return C

    def save_pair(self, buf: "PairBuf", path: str):
        """Write the TT pair in buf to a checkpoint file."""
        s = buf.struct()
        self.check(_lib.sgtt_pair_save(self._c, C.byref(s), os.fsencode(path)))

    def load_pair(self, path: str, buf: "PairBuf"):
        """Read a checkpoint file into buf (its capacities bound the ranks)."""
        s = buf.struct()
        self.check(_lib.sgtt_pair_load(self._c, os.fsencode(path), C.byref(s)))
        buf.update(s)
        return buf

    def profile_sample(self, period: int):
        """Record one event scope in every `period` of each kernel class."""
        self.check(_lib.sgtt_profile_sample(self._c, int(period)))

    def profile_read(self):
        n = 16
        sec = (C.c_double * n)()
        by = (C.c_double * n)()
        fl = (C.c_double * n)()
        la = (C.c_long * n)()
        nc = C.c_int()
        self.check(_lib.sgtt_profile_read(self._c, n, sec, by, fl, la, C.byref(nc)))
        out = {}
        for i in range(nc.value):
            out[_lib.sgtt_profile_class_name(i).decode()] = dict(seconds=sec[i], bytes=by[i], flops=fl[i],
                                                                 launches=la[i])
        return out

    def profile_regions(self):
        """{phase: {kernel class: event seconds}} since profiling was enabled."""
        nr, ncls = 32, 16
        sec = (C.c_double * (nr * ncls))()
        got = C.c_int()
        self.check(_lib.sgtt_profile_read_regions(self._c, nr, ncls, sec, C.byref(got)))
        out = {}
        for r in range(min(got.value, nr)):
            row = {_lib.sgtt_profile_class_name(c).decode(): sec[r * ncls + c] for c in range(ncls)
                   if sec[r * ncls + c] > 0}
            if row:
                out[_lib.sgtt_profile_region_name(r).decode()] = row
        return out

    def hessenberg_lsq(self, H: np.ndarray, beta: float):
        k = H.shape[1]
        Hc = np.asfortranarray(H, dtype=np.float64)
        y = np.zeros(k)
        res = C.c_double()
        self.check(_lib.sgtt_hessenberg_lsq(self._c, Hc.ctypes.data_as(C.POINTER(C.c_double)), k, beta,
                                            y.ctypes.data_as(C.POINTER(C.c_double)), C.byref(res)))
        return y, res.value

    def __del__(self):
        if getattr(self, "_c", None) and _lib is not None:
            _lib.sgtt_context_destroy(self._c)
            self._c = None


def bcr_variant_count() -> int:
    return _lib.sgtt_bcr_variant_count()


class System:
    def __init__(self, ctx: Context, cfg: dict, prior: PairBuf | None = None, eps_conv=1e-3, eps_rhs=1e-6):
        self.ctx = ctx
        self.cfg = dict(cfg)
        d = make_desc(cfg, eps_conv, eps_rhs)
        self._s = _P()
        pr = prior.struct() if prior is not None else None
        ctx.check(_lib.sgtt_assemble(ctx._c, C.byref(d), C.byref(pr) if pr is not None else None,
                                     C.byref(self._s)))
        info = SystemInfo()
        _lib.sgtt_system_info_get(self._s, C.byref(info))
        self.info = info
        self.nt, self.nxi, self.nu, self.np = info.nt, info.n_xi, info.n_u, info.n_p

    def history(self):
        """Outer iterations and refinement-cycle ends of the last solve (list of dicts)."""
        n = C.c_int()
        self.ctx.check(_lib.sgtt_solve_history(self._s, 0, None, C.byref(n)))
        buf = (IterRecord * max(n.value, 1))()
        self.ctx.check(_lib.sgtt_solve_history(self._s, n.value, buf, C.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    def pair(self, cap1=64, cap2=256, capp1=None, capp2=None):
        return PairBuf(self.nt, self.nxi, self.nu, self.np, cap1, cap2, capp1, capp2,
                       device=f"cuda:{self.ctx.device}")

    def rhs(self, out: PairBuf | None = None):
        out = out or self.pair(16, 128)
        s = out.struct()
        self.ctx.check(_lib.sgtt_rhs(self._s, C.byref(s)))
        out.update(s)
        return out

    def apply(self, x: PairBuf, out: PairBuf | None = None, eps: float = 0.0):
        out = out or self.pair(4 * x.u.cap1 + 8, 4 * x.u.cap2 + 8)
        sx, so = x.struct(), out.struct()
        self.ctx.check(_lib.sgtt_apply(self._s, C.byref(sx), C.byref(so), eps))
        out.update(so)
        return out

    def bcr_apply(self, which: int, b, variant: int = -1):
        """Device block cyclic reduction solve (which 0: F_avg on both
        velocity components, 2 n_s rows; 1: B M*^-1 B^T, n_p rows) of the
        columns of b (a 2-D float64 tensor on the context's device); returns x
        (new tensor).  variant -1: tuned choice; else that kernel variant for
        every pass."""
        import torch
        rows = 2 * (self.nu // 2) if which == 0 else self.np
        if b.dim() != 2 or b.shape[0] != rows or b.dtype != torch.float64 or b.device.type != "cuda":
            raise ValueError(f"b must be a float64 device tensor with {rows} rows")
        b = b.contiguous()
        x = torch.empty_like(b)
        torch.cuda.synchronize(b.device)   # b is ready before the library's stream reads it
        self.ctx.check(_lib.sgtt_bcr_apply(self._s, which, variant, b.shape[1], C.c_void_p(b.data_ptr()),
                                           C.c_void_p(x.data_ptr())))
        return x

    def bcr_apply_noalloc(self, which: int, b, x, variant: int = -1):
        """The same solve through the allocation-free entry point, into the
        caller's x (a float64 device tensor shaped like b); waits for the
        context's stream before returning."""
        import torch
        rows = 2 * (self.nu // 2) if which == 0 else self.np
        for t in (b, x):
            if t.dim() != 2 or t.shape[0] != rows or t.dtype != torch.float64 or t.device.type != "cuda" \
                    or not t.is_contiguous():
                raise ValueError(f"b and x must be contiguous float64 device tensors with {rows} rows")
        if x.shape != b.shape:
            raise ValueError("x must have the shape of b")
        torch.cuda.synchronize(b.device)
        self.ctx.check(_lib.sgtt_bcr_apply_noalloc(self._s, which, variant, b.shape[1], C.c_void_p(b.data_ptr()),
                                                   C.c_void_p(x.data_ptr())))
        torch.cuda.synchronize(b.device)   # the call does not wait for its stream
        return x

    def precondition(self, r: PairBuf, out: PairBuf | None = None, with_stats: bool = False, **opts):
        """z = P^-1 r; with_stats=True returns (z, inner iteration count)."""
        out = out or self.pair()
        o = make_opts(**opts)
        st = SolveStats()
        sr, so = r.struct(), out.struct()
        self.ctx.check(_lib.sgtt_precondition(self._s, C.byref(sr), C.byref(so), C.byref(o), C.byref(st)))
        out.update(so)
        return (out, st.inner_iters) if with_stats else out

    def solve(self, b: PairBuf, out: PairBuf | None = None, **opts):
        out = out or self.pair(96, 512)
        o = make_opts(**opts)
        st = SolveStats()
        sb, so = b.struct(), out.struct()
        rc = self.ctx.check(_lib.sgtt_solve(self._s, C.byref(sb), C.byref(so), C.byref(o), C.byref(st)))
        out.update(so)
        return out, st.as_dict(), rc

    def residual(self, b: PairBuf, x: PairBuf) -> float:
        r = C.c_double()
        sb, sx = b.struct(), x.struct()
        self.ctx.check(_lib.sgtt_residual(self._s, C.byref(sb), C.byref(sx), C.byref(r)))
        return r.value

    def residual_tensor(self, b: PairBuf, x: PairBuf):
        """(ru, rp, rel): the exact residual b - L x as full device tensors."""
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        ru = torch.empty((self.nt, self.nxi, self.nu), dtype=torch.float64, device=dev)
        rp = torch.empty((self.nt, self.nxi, self.np), dtype=torch.float64, device=dev)
        r = C.c_double()
        sb, sx = b.struct(), x.struct()
        self.ctx.check(_lib.sgtt_residual_tensor(self._s, C.byref(sb), C.byref(sx), ru.data_ptr(), rp.data_ptr(),
                                                 C.byref(r)))
        return ru, rp, r.value

    def __del__(self):
        if getattr(self, "_s", None) and _lib is not None:
            _lib.sgtt_system_destroy(self._s)
            self._s = None


class Mlp:
    """Learned correction of the mean spatial solve (see include/sgtt.h)."""

    def __init__(self, ctx: Context, n: int, width: int = 256, capacity: int = 0, seed: int = 0):
        self.ctx = ctx
        self.n, self.width = n, width
        self._m = _P()
        ctx.check(_lib.sgtt_mlp_create(ctx._c, n, width, capacity, seed, C.byref(self._m)))

    def size(self):
        npar, npairs = C.c_long(), C.c_long()
        _lib.sgtt_mlp_size(self._m, C.byref(npar), C.byref(npairs))
        return npar.value, npairs.value

    def split(self, flat):
        """flat parameter vector -> dict W1, b1, W2, b2, W3, b3 (views)."""
        n, w = self.n, self.width
        out, o = {}, 0
        for k, shp in (("W1", (w, n)), ("b1", (w,)), ("W2", (w, w)), ("b2", (w,)), ("W3", (n, w)), ("b3", (n,))):
            sz = int(np.prod(shp))
            out[k] = flat[o:o + sz].reshape(shp)
            o += sz
        return out

    def flatten(self, p):
        return np.concatenate([np.asarray(p[k], dtype=np.float32).ravel()
                               for k in ("W1", "b1", "W2", "b2", "W3", "b3")])

    def set_params(self, p):
        flat = np.ascontiguousarray(self.flatten(p) if isinstance(p, dict) else p, dtype=np.float32)
        self.ctx.check(_lib.sgtt_mlp_set_params(self._m, flat.ctypes.data_as(C.POINTER(C.c_float))))

    def get_params(self):
        flat = np.zeros(self.size()[0], dtype=np.float32)
        self.ctx.check(_lib.sgtt_mlp_get_params(self._m, flat.ctypes.data_as(C.POINTER(C.c_float))))
        return self.split(flat)

    def save(self, path: str):
        """Write the parameters to a network file (sgtt_mlp_save)."""
        self.ctx.check(_lib.sgtt_mlp_save(self._m, os.fsencode(path)))

    def load(self, path: str):
        """Set the parameters from a network file of the same shape."""
        self.ctx.check(_lib.sgtt_mlp_load(self._m, os.fsencode(path)))

    def forward(self, X, f16: bool = False):
        """X: (n, B) -> (n, B) float32; f16 runs the products on FP16
        operands (the preconditioner's form)."""
        Xc = np.ascontiguousarray(np.asarray(X, dtype=np.float32).T)
        B = Xc.shape[0]
        Y = np.zeros_like(Xc)
        fn = _lib.sgtt_mlp_forward_f16 if f16 else _lib.sgtt_mlp_forward
        self.ctx.check(fn(self._m, Xc.ctypes.data_as(C.POINTER(C.c_float)), B,
                          Y.ctypes.data_as(C.POINTER(C.c_float))))
        return Y.T

    def loss_grad(self, X, T):
        Xc = np.ascontiguousarray(np.asarray(X, dtype=np.float32).T)
        Tc = np.ascontiguousarray(np.asarray(T, dtype=np.float32).T)
        g = np.zeros(self.size()[0], dtype=np.float32)
        L = C.c_double()
        self.ctx.check(_lib.sgtt_mlp_loss_grad(self._m, Xc.ctypes.data_as(C.POINTER(C.c_float)),
                                               Tc.ctypes.data_as(C.POINTER(C.c_float)), Xc.shape[0], C.byref(L),
                                               g.ctypes.data_as(C.POINTER(C.c_float))))
        return L.value, self.split(g)

    def train(self, steps, batch=64, lr=1e-3, seed=0):
        losses = np.zeros(max(steps, 1))
        self.ctx.check(_lib.sgtt_mlp_train(self._m, steps, batch, lr, seed,
                                           losses.ctypes.data_as(C.POINTER(C.c_double))))
        return losses[:steps]

    def add_pairs(self, X, T):
        """Append columns of X, T ((n, k) each) as training pairs; returns how many fit."""
        Xc = np.ascontiguousarray(np.asarray(X, dtype=np.float32).T)
        Tc = np.ascontiguousarray(np.asarray(T, dtype=np.float32).T)
        k = C.c_long()
        self.ctx.check(_lib.sgtt_mlp_add_pairs(self._m, Xc.ctypes.data_as(C.POINTER(C.c_float)),
                                               Tc.ctypes.data_as(C.POINTER(C.c_float)), Xc.shape[0], C.byref(k)))
        return k.value

    def collect(self, system, on=True):
        self.ctx.check(_lib.sgtt_mlp_collect(system._s, self._m if on else None))
        # the system keeps the network alive while it refers to it
        system._mlp_collect = self if on else None

    def attach(self, system, on=True):
        self.ctx.check(_lib.sgtt_mlp_attach(system._s, self._m if on else None))
        system._mlp_apply = self if on else None

    def __del__(self):
        if getattr(self, "_m", None) and _lib is not None:
            _lib.sgtt_mlp_destroy(self._m)
            self._m = None


def solve_batched(systems, bs, xs, **opts):
    """Solve independent systems; those on different contexts run concurrently.
    Returns ([stats dict], [status])."""
    n = len(systems)
    o = make_opts(**opts)
    sysarr = (_P * n)(*[S._s for S in systems])
    bstructs = [b.struct() for b in bs]
    xstructs = [x.struct() for x in xs]
    barr = (C.POINTER(SgttPair) * n)(*[C.pointer(t) for t in bstructs])
    xarr = (C.POINTER(SgttPair) * n)(*[C.pointer(t) for t in xstructs])
    st = (SolveStats * n)()
    status = (C.c_int * n)()
    rc = _lib.sgtt_solve_batched(sysarr, n, barr, xarr, C.byref(o), st, status)
    for x, t in zip(xs, xstructs):
        x.update(t)
    if rc < 0:
        bad = [i for i in range(n) if status[i] < 0]
        raise SgttError(rc, f"batched solve failed for problems {bad}: "
                            + _lib.sgtt_last_error(systems[bad[0]].ctx._c).decode())
    return [st[i].as_dict() for i in range(n)], list(status)


def picard(ctx: Context, cfg: dict, steps: int = 5, tol_picard: float = 1e-5, eps_soln: float = 1e-10,
           eps_conv: float = 1e-3, eps_rhs: float = 1e-6, out: PairBuf | None = None, caps=(128, 2048),
           update_mode: int = 0, **solve_opts):
    """Picard's method (Alg. 3.1, eq. 4.8) on the device: returns (iterate, stats dict, status).
    update_mode 0 truncates the updated iterate, 1 the update alone (the sum kept exact)."""
    d = make_desc(cfg, eps_conv, eps_rhs)
    o = PicardOpts(int(steps), float(tol_picard), float(eps_soln), make_opts(**solve_opts), int(update_mode))
    if out is None:
        hp = HostProblem(cfg)
        out = PairBuf(hp.nt, hp.n_xi, hp.n_u, hp.n_p, caps[0], caps[1], device=f"cuda:{ctx.device}")
    st = PicardStats()
    so = out.struct()
    rc = ctx.check(_lib.sgtt_picard(ctx._c, C.byref(d), C.byref(o), C.byref(so), C.byref(st)))
    out.update(so)
    return out, st.as_dict(), rc


def mlp_file_info(path: str):
    """(n, width, nparam) of a network file; raises SgttError for a missing
    or foreign file."""
    n, w, npar = C.c_int(), C.c_int(), C.c_long()
    rc = _lib.sgtt_mlp_file_info(os.fsencode(path), C.byref(n), C.byref(w), C.byref(npar))
    if rc != 0:
        raise SgttError(rc, f"network file {path}")
    return n.value, w.value, npar.value


def write_mlp_host(path: str, n: int, width: int, params):
    """Write a network file from a host FP32 parameter vector."""
    flat = np.ascontiguousarray(params, dtype=np.float32).ravel()
    if flat.size != width * n + width + width * width + width + n * width + n:
        raise ValueError("parameter count does not match the shape")
    rc = _lib.sgtt_mlp_file_write_host(os.fsencode(path), n, width, flat.ctypes.data)
    if rc != 0:
        raise SgttError(rc, f"network file {path}")


def read_mlp_host(path: str, n: int, width: int):
    """FP32 parameters of a network file of the given shape (host)."""
    flat = np.zeros(width * n + width + width * width + width + n * width + n, dtype=np.float32)
    rc = _lib.sgtt_mlp_file_read_host(os.fsencode(path), n, width, flat.ctypes.data)
    if rc != 0:
        raise SgttError(rc, f"network file {path}")
    return flat


def pair_file_info(path: str):
    """(n1, n2, n3, r1, r2) of the velocity and pressure TTs of a checkpoint
    file; raises SgttError for a missing or foreign file."""
    d = (C.c_int * 10)()
    rc = _lib.sgtt_pair_file_info(os.fsencode(path), d)
    if rc != 0:
        raise SgttError(rc, f"checkpoint file {path}")
    return tuple(d[0:5]), tuple(d[5:10])


def write_pair_host(path: str, cores):
    """Write a checkpoint from host arrays: cores = ((G1, G2, G3), (P1, P2, P3))
    in the library's layout (core 1 n1 x r1, core 2 r1 x n2 x r2, core 3
    n3 x r2)."""
    arrs, dims = [], []
    for g1, g2, g3 in cores:
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (g1, g2, g3)]
        arrs += a
        dims += [a[0].shape[0], a[1].shape[1], a[2].shape[0], a[0].shape[1], a[2].shape[1]]
    d = (C.c_int * 10)(*dims)
    ptrs = (C.c_void_p * 6)(*[x.ctypes.data for x in arrs])
    rc = _lib.sgtt_pair_file_write_host(os.fsencode(path), d, ptrs)
    if rc != 0:
        raise SgttError(rc, f"checkpoint file {path}")


def read_pair_host(path: str, caps=None):
    """Read a checkpoint into host arrays; caps = ((n1, n2, n3, cap1, cap2),
    (...)) sizes the buffers (default: the file's own sizes)."""
    if caps is None:
        caps = pair_file_info(path)
    bufs = []
    for n1, n2, n3, c1, c2 in caps:
        bufs += [np.zeros(n1 * c1), np.zeros(c1 * n2 * c2), np.zeros(n3 * c2)]
    cp = (C.c_int * 10)(*[v for c in caps for v in c])
    ptrs = (C.c_void_p * 6)(*[x.ctypes.data for x in bufs])
    d = (C.c_int * 10)()
    rc = _lib.sgtt_pair_file_read_host(os.fsencode(path), cp, ptrs, d)
    if rc != 0:
        raise SgttError(rc, f"checkpoint file {path}")
    out = []
    for q in range(2):
        n1, n2, n3, r1, r2 = d[5 * q:5 * q + 5]
        b = bufs[3 * q:3 * q + 3]
        out.append((b[0][:n1 * r1].reshape(n1, r1), b[1][:r1 * n2 * r2].reshape(r1, n2, r2),
                    b[2][:n3 * r2].reshape(n3, r2)))
    return tuple(out)


ABI_STRUCTS = ("SgttTT", "SgttPair", "ProblemDesc", "SystemInfo", "SolveOpts", "SolveStats", "MemoryInfo",
               "PicardOpts", "PicardStats", "IterRecord")


def abi_sizes() -> dict:
    """sizeof of each public struct as the library was compiled, keyed by
    the name of its ctypes mirror here."""
    n = len(ABI_STRUCTS)
    buf = (C.c_long * n)()
    _lib.sgtt_abi_sizes(buf, n)
    return dict(zip(ABI_STRUCTS, list(buf)))


def version() -> str:
    return _lib.sgtt_version().decode()
