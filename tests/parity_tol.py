"""Tolerance of the GPU parity tests against the FP64 oracle.

For amplitudes a (GPU) and o (oracle) over a set of m of the 2^k paths of an
n-qubit circuit,
    e_x = | |a_x|^2 - |o_x|^2 | / max(|o_x|^2, floor),
the floor being the mean |amp|^2 of such a partial sum: (m / 2^k) 2^-n for the
full sum or a random subset of paths, or the oracle's own mean over the
requested bitstrings where that is larger (path sets chosen among the paths
whose term is not zero carry more than their share of the norm);
max_x e_x <= 1e-5 for complex64 sweeps and <= 1e-10 for complex128 sweeps.
"""
import numpy as np

TOL_C64 = 1e-5
TOL_C128 = 1e-10


def c11_error(a, o, m, k, n):
    floor = max((m / 2.0 ** k) * 2.0 ** (-n), float(np.mean(np.abs(o) ** 2)))
    return float(np.max(np.abs(np.abs(a) ** 2 - np.abs(o) ** 2) / np.maximum(np.abs(o) ** 2, floor)))
