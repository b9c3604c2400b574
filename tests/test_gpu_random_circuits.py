"""Randomised GPU parity: small random grid circuits (CZ, iSWAP or mixed), random straight cuts,
random tunings within their documented ranges, random path subsets, complex64 and complex128
sweeps, each against the FP64 oracle.  Seeded, so every run checks the same cases."""
import numpy as np
import pytest

import oracle
from parity_tol import TOL_C128, TOL_C64, c11_error
from workload import CZ, ISWAP, column_cut_mask, grid_circuit, random_bitstrings, row_cut_mask

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


def _case(i):
    rng = np.random.default_rng(9000 + i)
    rows, cols = int(rng.integers(2, 5)), int(rng.integers(2, 6))
    if rows * cols < 4:
        cols = 2
        rows = 2
    depth = int(rng.integers(3, 15))
    kind = ("cz", "iswap", "mixed")[int(rng.integers(0, 3))]
    g = grid_circuit(rows, cols, depth, 500 + i, two_qubit=ISWAP if kind == "iswap" else CZ)
    horizontal = rows > 1 and (cols == 1 or rng.integers(0, 2) == 1)
    if horizontal:
        mask = row_cut_mask(rows, cols, int(rng.integers(1, rows)))
    else:
        mask = column_cut_mask(rows, cols, int(rng.integers(1, cols)))
    if kind == "mixed":     # every other crossing or in-block two-qubit gate an iSWAP
        two = np.flatnonzero(g["kind"] == CZ)
        g["kind"][two[::2]] = ISWAP
    tuning = dict(reg_qubits=int(rng.integers(1, 6)), dense_qubits=int(rng.choice([0, 4])),
                  no_leaf_fold=int(rng.integers(0, 2)), fold_levels=int(rng.integers(0, 3)),
                  waves_per_cu=int(rng.choice([0, 16, 64])))
    fp64 = bool(rng.integers(0, 2))
    if fp64:
        tuning["reg_qubits"] = min(tuning["reg_qubits"], 4)
    return rows, cols, g, mask, kind, tuning, fp64, rng


@pytest.mark.parametrize("i", range(600))
def test_random_circuit(sf, i):
    rows, cols, g, mask, kind, tuning, fp64, rng = _case(i)
    n = rows * cols
    c = sf.Circuit(rows, cols, g, mask)
    c.tune(**tuning)
    k = c.k
    mode = int(rng.integers(0, 3))
    if (mode == 0 and k <= 12) or k <= 2:
        ids = np.arange(1 << k, dtype=np.uint64)
        kw = {}
    elif mode == 1:
        m = int(rng.integers(1, min(1 << k, 300) + 1))
        ids = np.unique(rng.integers(0, 1 << k, m).astype(np.uint64))
        kw = {"path_ids": ids}
    else:
        cnt = int(rng.integers(1, min(1 << k, 512) + 1))
        begin = int(rng.integers(0, (1 << k) - cnt + 1))
        ids = np.arange(begin, begin + cnt, dtype=np.uint64)
        kw = {"path_begin": begin, "n_paths": cnt}
    bits = random_bitstrings(n, min(1 << n, 700), 7000 + i)
    say(f"random case {i}: {rows}x{cols} {kind} cut {mask:#x} k={k} paths={ids.size} fp64={fp64} {tuning}")
    a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS if fp64 else 0, **kw)
    o = oracle.path_sum(n, g, mask, ids, bits)
    err = c11_error(a, o, ids.size, k, n)
    assert err <= (TOL_C128 if fp64 else TOL_C64), (i, err)
    c.close()


def _large_case(i):
    """Larger blocks (up to 15 qubits) and sparse path subsets, so levels hold 64 or more slots:
    passes with a qubit in lane bit 5, zero-subspace loads and tiles of padding slots occur."""
    rng = np.random.default_rng(19000 + i)
    rows, cols = int(rng.integers(4, 6)), int(rng.integers(4, 7))
    depth = int(rng.integers(16, 33))
    kind = ("cz", "cz", "iswap")[int(rng.integers(0, 3))]
    g = grid_circuit(rows, cols, depth, 1500 + i, two_qubit=ISWAP if kind == "iswap" else CZ)
    mask = column_cut_mask(rows, cols, cols // 2)
    tuning = dict(reg_qubits=int(rng.integers(4, 6)), dense_qubits=int(rng.choice([0, 4])),
                  no_leaf_fold=int(rng.integers(0, 2)))
    return rows, cols, g, mask, kind, tuning, rng


@pytest.mark.parametrize("i", range(24))
def test_random_large_blocks(sf, i):
    rows, cols, g, mask, kind, tuning, rng = _large_case(i)
    n = rows * cols
    c = sf.Circuit(rows, cols, g, mask)
    c.tune(**tuning)
    k = c.k
    m = int(rng.integers(150, 401))
    ids = np.unique(rng.integers(0, 1 << k, m).astype(np.uint64)) if k > 8 else np.arange(1 << k, dtype=np.uint64)
    bits = random_bitstrings(n, 96, 17000 + i)
    say(f"large case {i}: {rows}x{cols} {kind} k={k} paths={ids.size} {tuning}")
    a = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(n, g, mask, ids, bits)
    err = c11_error(a, o, ids.size, k, n)
    assert err <= TOL_C64, (i, err)
    c.close()
