"""ctypes access to the FP64 oracle library (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    """This host's build of the oracle (the file name carries a hash of the CPU it is built for)."""
    from .build import out_path
    return out_path()


def load():
    """Load this host's oracle library, building it first if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        from .build import build
        build()
    lib = ctypes.CDLL(path)
    c_u64p = ctypes.POINTER(ctypes.c_uint64)
    c_dp = ctypes.POINTER(ctypes.c_double)
    c_i64p = ctypes.POINTER(ctypes.c_int64)
    lib.or_gate_matrix.argtypes = [ctypes.c_int, c_dp]
    lib.or_full_state.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, c_dp]
    lib.or_pext.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.or_pext.restype = ctypes.c_uint64
    lib.or_cut_gates.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64,
                                 c_i64p, ctypes.c_int]
    lib.or_num_cut.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64]
    lib.or_path_sum.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64,
                                c_u64p, ctypes.c_int64, c_u64p, ctypes.c_int64, c_dp, c_dp, c_dp]
    lib.or_num_paths.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.or_num_paths.restype = ctypes.c_int64
    lib.or_sample_paths.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, c_u64p,
                                    ctypes.c_int64, c_i64p]
    lib.or_gate_matrix2.argtypes = [ctypes.c_int, c_dp]
    lib.or_branch_ops.argtypes = [ctypes.c_int, ctypes.c_int, c_dp, c_dp]
    lib.or_sample_bitstrings.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, c_u64p]
    lib.or_splitmix64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.or_splitmix64_at.restype = ctypes.c_uint64
    lib.or_rejection_accept.argtypes = [c_dp, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_uint8), c_dp]
    _LIB = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def num_threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS, else all cores)."""
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else (os.cpu_count() or 1)


def gate_matrix(kind: int) -> np.ndarray:
    out = np.zeros(8, dtype=np.float64)
    if load().or_gate_matrix(kind, _ptr(out, ctypes.c_double)):
        raise ValueError("not a one-qubit gate kind")
    return (out[0::2] + 1j * out[1::2]).reshape(2, 2)


def full_state(n: int, gates: np.ndarray) -> np.ndarray:
    """O1: the 2^n complex128 state after all gates (list order)."""
    g = np.ascontiguousarray(gates)
    psi = np.empty(2 << n, dtype=np.float64)
    if load().or_full_state(n, g.ctypes.data, g.size, _ptr(psi, ctypes.c_double)):
        raise ValueError("invalid circuit")
    return psi.view(np.complex128)


def pext(x: int, mask: int) -> int:
    return int(load().or_pext(x, mask))


def num_cut(n: int, gates: np.ndarray, mask_a: int) -> int:
    g = np.ascontiguousarray(gates)
    return int(load().or_num_cut(n, g.ctypes.data, g.size, mask_a))


def cut_gates(n: int, gates: np.ndarray, mask_a: int) -> np.ndarray:
    """Indices (into ``gates``) of the crossing two-qubit gates in path-bit order."""
    g = np.ascontiguousarray(gates)
    lib = load()
    nc = int(lib.or_cut_gates(n, g.ctypes.data, g.size, mask_a, None, 0))
    if nc < 0:
        raise ValueError("bad gates")
    idx = np.zeros(max(nc, 1), dtype=np.int64)
    lib.or_cut_gates(n, g.ctypes.data, g.size, mask_a, _ptr(idx, ctypes.c_int64), nc)
    return idx[:nc]


def path_sum(n: int, gates: np.ndarray, mask_a: int, paths, bits, norms: bool = False):
    """O2: sum over ``paths`` of psiA_p(x_A) psiB_p(x_B) for each bitstring.

    Returns complex128 amplitudes, plus (||psiA_p||^2, ||psiB_p||^2) arrays
    when ``norms`` is true.
    """
    g = np.ascontiguousarray(gates)
    p = np.ascontiguousarray(np.asarray(paths, dtype=np.uint64))
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint64))
    amps = np.zeros(2 * max(b.size, 1), dtype=np.float64)
    na = np.zeros(max(p.size, 1)) if norms else None
    nb = np.zeros(max(p.size, 1)) if norms else None
    rc = load().or_path_sum(n, g.ctypes.data, g.size, mask_a,
                            _ptr(p, ctypes.c_uint64), p.size, _ptr(b, ctypes.c_uint64), b.size,
                            _ptr(amps, ctypes.c_double),
                            _ptr(na, ctypes.c_double) if norms else None,
                            _ptr(nb, ctypes.c_double) if norms else None)
    if rc:
        raise ValueError("invalid path-sum request")
    out = amps.view(np.complex128)[: b.size]
    if norms:
        return out, na[: p.size], nb[: p.size]
    return out


def num_paths(k: int, f: float) -> int:
    return int(load().or_num_paths(k, f))


def sample_paths(k: int, f: float, seed: int) -> np.ndarray:
    m = num_paths(k, f)
    if m < 0:
        raise ValueError("bad k or f")
    out = np.zeros(m, dtype=np.uint64)
    n_out = ctypes.c_int64(0)
    if load().or_sample_paths(k, f, seed, _ptr(out, ctypes.c_uint64), m, ctypes.byref(n_out)):
        raise ValueError("sampling failed")
    return out[: n_out.value]


# ---------------------------------------------------------------- rejection sampling
# Section "Frugal rejection sampling" and its figure (Algorithm 1 basic, Algorithm 2 frugal).

def rejection_m(n_qubits: int, eps: float, basic: bool = False) -> float:
    """Step 1.  Algorithm 1: M = ceil(ln(N / eps)), N = 2^n.  Algorithm 2 under Porter-Thomas
    statistics: the smallest integer M' >= 1 with sum_{p > M'/N} p = e^{-M'} (1 + M') <= eps."""
    import math
    if not (eps > 0.0) or n_qubits < 1:
        raise ValueError("bad eps or n")
    if basic:
        return float(math.ceil(n_qubits * math.log(2.0) - math.log(eps)))
    m = 1
    while math.exp(-m) * (1.0 + m) > eps:
        m += 1
    return float(m)


def sample_bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    """Step 2: count distinct uniform n-qubit bitstrings in SplitMix64 draw order."""
    out = np.zeros(count, dtype=np.uint64)
    if load().or_sample_bitstrings(n_qubits, count, seed, _ptr(out, ctypes.c_uint64)):
        raise ValueError("bad n or count")
    return out


def splitmix64_at(seed: int, j: int) -> int:
    return int(load().or_splitmix64_at(seed, j))


def rejection_accept(amps, n_qubits: int, m: float, seed: int, basic: bool = False):
    """Step 4 (Algorithm 2; Algorithm 1 steps 4-5 with basic=True) on a batch of amplitudes.
    Returns (accept flags as bool array, batch estimate of the mass above M/N)."""
    a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128))
    flat = a.view(np.float64)
    acc = np.zeros(a.size, dtype=np.uint8)
    err = ctypes.c_double(0.0)
    if load().or_rejection_accept(_ptr(flat, ctypes.c_double), a.size, n_qubits, m, seed, int(basic),
                                  _ptr(acc, ctypes.c_uint8), ctypes.byref(err)):
        raise ValueError("bad arguments")
    return acc.astype(bool), err.value


# ---------------------------------------------------------------- validation of results
# Appendix on validating simulation results: the state overlap estimated from k amplitudes at the
# same indices, and the two-party protocol built on it; cross-entropy fidelity as a comparison.

def fidelity_estimate(a, b):
    """|sum conj(a) b|^2 / (sum |a|^2 sum |b|^2) over the given amplitudes (FP64 sums in order);
    returns (f_e, sum |a|^2, sum |b|^2)."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    ov = complex(0.0)
    na = nb = 0.0
    for x, y in zip(a.tolist(), b.tolist()):
        ov += x.conjugate() * y
        na += x.real * x.real + x.imag * x.imag
        nb += y.real * y.real + y.imag * y.imag
    f = (ov.real * ov.real + ov.imag * ov.imag) / (na * nb) if na > 0 and nb > 0 else 0.0
    return f, na, nb


def xeb_fidelity(amps, n_qubits: int) -> float:
    """Linear cross-entropy fidelity N <p(x)> - 1 over the ideal amplitudes of sampled x."""
    a = np.asarray(amps, dtype=np.complex128)
    s = 0.0
    for x in a.tolist():
        s += x.real * x.real + x.imag * x.imag
    return 2.0 ** n_qubits * s / len(a) - 1.0 if len(a) else 0.0


# ---------------------------------------------------------------- two-qubit gates
# Section on harder benchmarks through two-qubit gates: iSWAP and Eq. (4way).

def gate_matrix2(kind: int) -> np.ndarray:
    out = np.zeros(32, dtype=np.float64)
    if load().or_gate_matrix2(kind, _ptr(out, ctypes.c_double)):
        raise ValueError("not a two-qubit gate kind")
    return (out[0::2] + 1j * out[1::2]).reshape(4, 4)


def branch_ops(kind: int, r: int):
    """Term r = 2i + j of Eq. (4way) for a crossing gate: (|i><j| on the block-A endpoint,
    the 2x2 block G_ij on the block-B endpoint)."""
    ea = np.zeros(8, dtype=np.float64)
    gb = np.zeros(8, dtype=np.float64)
    if load().or_branch_ops(kind, r, _ptr(ea, ctypes.c_double), _ptr(gb, ctypes.c_double)):
        raise ValueError("bad kind or term")
    return (ea[0::2] + 1j * ea[1::2]).reshape(2, 2), (gb[0::2] + 1j * gb[1::2]).reshape(2, 2)
