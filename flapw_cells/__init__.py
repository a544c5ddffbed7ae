"""Seeded synthetic unit cells shaped like the paper's FLAPW workloads.

This package only draws inputs: lattice, atom positions, radial boundary
values, the per-type T blocks, the k-point and its plane-wave basis (the set
of reciprocal vectors G with |k+G| below a cut-off, ordered by |k+G|).  It
contains none of the arithmetic that turns those inputs into the matching
coefficients, H or S; both the oracle and the GPU library consume the arrays
it returns and recompute everything else on their own.
"""
from .cells import CONFIGS, CellConfig, make_case, make_batch_case, basis_for_k, sub_case, perturb_positions, \
    shell_sizes, at_k

__all__ = ["CONFIGS", "CellConfig", "make_case", "make_batch_case", "basis_for_k", "sub_case",
           "perturb_positions", "shell_sizes", "at_k"]
