"""MI355X solver for stochastic-Galerkin KKT systems of PDE-constrained
optimal control (Li, Onwunta, Sousedik, arXiv 2512.23804).

The computation lives in the HIP library ``libsgkkt.so`` (C ABI in
``include/sg.h``); this package only marshals arguments to it.
"""
from ._lib import (SG_ARNOLDI_CGS2, SG_ARNOLDI_DCGS2, SG_FIELD_AFFINE, SG_FIELD_LOGNORMAL, SG_MEAN_EXACT,
                   SG_PRECOND_BLOCK_DIAGONAL, SG_PRECOND_HGSOC,
                   SG_MEAN_MULTIGRID, SG_ERR_CANCELLED, SG_ERR_HIP, SG_ERR_INVALID, SG_ERR_NOMEM,
                   SG_ERR_NONCOERCIVE, SG_ERR_NONFINITE, SG_ERR_UNKNOWN, SG_FP32, SG_FP64, SG_NOT_CONVERGED, SG_OK,
                   SG_PENDING, SG_PREC_FP32_PRECOND, SG_PREC_FP32_REFINE, SG_PREC_FP64, SIGNATURES, Handle,
                   ProblemData, Server, SGError, check, default_options, lib, tune_clear, tune_count, tune_load,
                   tune_save, validate)

__all__ = [
    "Handle", "ProblemData", "Server", "SGError", "default_options", "validate", "lib", "check", "SIGNATURES",
    "tune_save", "tune_load", "tune_count", "tune_clear",
    "SG_OK", "SG_PENDING", "SG_NOT_CONVERGED", "SG_ERR_INVALID", "SG_ERR_NONCOERCIVE", "SG_ERR_NONFINITE",
    "SG_ERR_NOMEM", "SG_ERR_HIP", "SG_ERR_CANCELLED", "SG_ERR_UNKNOWN", "SG_FP64", "SG_FP32",
    "SG_PREC_FP64", "SG_PREC_FP32_REFINE", "SG_PREC_FP32_PRECOND", "SG_ARNOLDI_DCGS2", "SG_ARNOLDI_CGS2",
    "SG_MEAN_MULTIGRID", "SG_MEAN_EXACT", "SG_FIELD_AFFINE", "SG_FIELD_LOGNORMAL", "SG_PRECOND_BLOCK_DIAGONAL",
    "SG_PRECOND_HGSOC",
]
