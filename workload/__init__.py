"""Seeded synthetic inputs shared by the GPU path, the oracle and the tests.

This package only generates inputs: gate lists of random grid circuits,
requested bitstrings and blocks of path ids.  It holds none of the
simulation arithmetic, so neither side of a parity test can borrow the
other's computation through it.
"""
from .generator import (  # noqa: F401
    GATE_DTYPE, H, XH, YH, T, CZ, ISWAP, GATE_NAMES,
    SplitMix64, splitmix64_array,
    cz_pattern_edges, grid_circuit, random_bitstrings, path_block, equal_bit_pairs, is_live, live_path_block,
    column_cut_mask, row_cut_mask, CONFIGS, WorkloadConfig, make_workload, serving_mix, workload_block,
)
