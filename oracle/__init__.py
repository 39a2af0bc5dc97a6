"""CPU FP64 oracle for diag(H(i w_k)^{-1}) of the lattice Dyson matrix.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the GPU library.

Modules
-------
dyson    -- the definition (eq. (1)) and three independent ways to take the
            diagonal of the inverse: dense inversion (O1), the exact
            block-tridiagonal recursive Green's function (O2) and a sparse LU
            with per-site unit solves (O3); plus the closed forms used as pins.
lowrank  -- a plain mirror of the paper's Lanczos-based low-rank correction
            method (Sec. II.B-C, eqs. (4)-(13)) with exact sparse solves; it is
            used to pin the oracle's agreement with the method at full
            interface rank, not as an oracle of G itself; and the Lanczos run
            on the Schur complement (interface space) as a studied variant.

Every function cites the passage of the paper it follows.  "parity unpinned"
marks a function with no independent pin (none at present).
"""
from .dyson import (assemble_diag, assemble_diag_z, hamiltonian, dense_hamiltonian, diag_inv_dense,
                    diag_inv_rgf, diag_inv_sampled, closed_form_periodic,
                    closed_form_open_uniform, closed_form_uniform, oracle_diag, rel_err)
from .lowrank import lowrank_diag, interface_lanczos_diag, separator_positions, plan_boxes

__all__ = ["assemble_diag", "assemble_diag_z", "hamiltonian", "dense_hamiltonian", "diag_inv_dense",
           "diag_inv_rgf", "diag_inv_sampled", "closed_form_periodic",
           "closed_form_open_uniform", "closed_form_uniform", "oracle_diag", "rel_err",
           "lowrank_diag", "interface_lanczos_diag",
           "separator_positions", "plan_boxes"]
