"""CPU FP64 oracle for RSAI(tol) -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this package. The GPU product path never touches it.
"""
from .oracle import (DROP_ADAPTIVE, DROP_FIXED, DROP_NONE, backward, bicgstab, build_lib,
                     fixed_pattern, model_solve_flops, permute_rows, rsai, transversal)

__all__ = ["rsai", "fixed_pattern", "backward", "bicgstab", "build_lib", "model_solve_flops", "transversal", "permute_rows",
           "DROP_NONE",
           "DROP_FIXED", "DROP_ADAPTIVE"]
