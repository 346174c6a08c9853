"""MI355X-native low-rank solver for one Picard step of the stochastic
Galerkin, all-at-once unsteady Navier-Stokes system (Elman & Su).

The compute path is the HIP library ``libsgtt.so`` (C ABI in
include/sgtt.h); ``paper_1906_06785_amd.sgtt`` is its ctypes binding.
"""
from .sgtt import (Context, HostProblem, PairBuf, SgttError, System, TTBuf, make_desc,  # noqa: F401
                   make_opts, version)
