"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is built from ``oracle/sf_oracle.c`` by
``oracle.build.build()`` and shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    lib_path, load, gate_matrix, full_state, path_sum, num_cut, cut_gates,
    sample_paths, num_paths, pext, num_threads,
    rejection_m, sample_bitstrings, splitmix64_at, rejection_accept,
    fidelity_estimate, xeb_fidelity, gate_matrix2, branch_ops,
)
