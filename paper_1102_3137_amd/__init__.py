"""MI355X library for diag(H(i w_k)^{-1}) of the lattice Dyson matrix by the
Lanczos-based low-rank correction method (arXiv:1102.3137).

The compute path is the HIP library libdyson_mi355x.so (C ABI in
include/dyson.h); `binding` marshals arguments to it.  There is no CPU
fallback: loading fails loudly when the library is missing.
"""
from .binding import (DysonError, Lattice, Opts, Report, PlanInfo, Plan, Context, Request,
                      Allocator, load_library, PART_NESTED, PART_SINGLE, PREC_FP64, PREC_MIXED,
                      PREC_MIXED16, MEM_DEVICE, MEM_HOST)

__all__ = ["DysonError", "Lattice", "Opts", "Report", "PlanInfo", "Plan", "Context", "Request",
           "Allocator", "load_library", "PART_NESTED", "PART_SINGLE", "PREC_FP64", "PREC_MIXED",
           "PREC_MIXED16", "MEM_DEVICE", "MEM_HOST"]
