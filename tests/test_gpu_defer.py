"""Deferred block-A level (tuning no_defer = 0, the default).

When block A's operations at the level the general fold reads are the crossing CZs' projectors
P_s (Section 2, Eq. (CZ)) and one-qubit gates on the projected qubits, the level's block-A
states are not written: the fold reads the parent batch at the rows whose projected bits equal
the slot's path bits and multiplies by the gates' 2x2 entries.  The 7x8 benchmark's last written
level has that form; so do the 5x4 and 5x5 circuits below with the last level folded in the
general form.  Each case checks the oracle (Section 3's path sum) with and without deferral,
over all paths, path subsets (descendants missing, one-child chains) and several leaf batches.
"""
import numpy as np
import pytest

import oracle
from parity_tol import TOL_C128, TOL_C64, c11_error
from workload import grid_circuit, random_bitstrings

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


CASES = [(5, 4, 16, 1), (5, 4, 16, 3), (5, 5, 16, 2)]


@pytest.mark.parametrize("rows,cols,depth,seed", CASES)
@pytest.mark.parametrize("paths", ["all", "subset", "sparse"])
def test_deferred_level_matches_oracle(sf, rows, cols, depth, seed, paths):
    n = rows * cols
    g = grid_circuit(rows, cols, depth, seed)
    c = sf.Circuit(rows, cols, g)
    c.tune(fold_levels=1)
    assert "A deferred" in sf.describe_plan(c.handle)
    rng = np.random.default_rng(seed)
    if paths == "all":
        ids = np.arange(1 << c.k, dtype=np.uint64)
    elif paths == "subset":
        ids = np.sort(rng.choice(1 << c.k, size=(1 << c.k) // 3, replace=False)).astype(np.uint64)
    else:
        ids = np.sort(rng.choice(1 << c.k, size=12, replace=False)).astype(np.uint64)
    bits = random_bitstrings(n, 700, seed + 10)
    say(f"deferred level {rows}x{cols} d{depth} seed {seed} {paths} ({ids.size} paths)")
    o = oracle.path_sum(n, g, c.mask_a, ids, bits)
    for no_defer in (0, 1):
        for tune in ({}, {"max_slots": 4}):
            c.tune(fold_levels=1, no_defer=no_defer, **tune)
            a = c.amplitudes(bits, path_ids=ids)
            assert c11_error(a, o, ids.size, c.k, n) <= TOL_C64, (no_defer, tune)
    c.close()


def test_deferred_level_fp64_sweeps(sf):
    rows, cols, depth, seed = 5, 4, 16, 2
    n = rows * cols
    g = grid_circuit(rows, cols, depth, seed)
    c = sf.Circuit(rows, cols, g)
    bits = random_bitstrings(n, 500, 77)
    ids = np.arange(1 << c.k, dtype=np.uint64)
    o = oracle.path_sum(n, g, c.mask_a, ids, bits)
    say("deferred level 5x4 d16 FP64 sweeps")
    for no_defer in (0, 1):
        c.tune(fold_levels=1, no_defer=no_defer)
        a = c.amplitudes(bits, path_ids=ids, flags=sf.SF_FP64_SWEEPS)
        assert c11_error(a, o, ids.size, c.k, n) <= TOL_C128, no_defer
    c.close()


def test_deferred_level_writes_fewer_bytes(sf):
    """Deferral drops block A's passes of the read level: fewer planned passes and sweep bytes."""
    rows, cols, depth, seed = 5, 5, 16, 2
    g = grid_circuit(rows, cols, depth, seed)
    c = sf.Circuit(rows, cols, g)
    bits = random_bitstrings(rows * cols, 300, 5)
    out = []
    for no_defer in (0, 1):
        c.tune(fold_levels=1, no_defer=no_defer)
        c.amplitudes(bits)
        out.append(c.stats())
    assert out[0]["sweep_bytes"] < out[1]["sweep_bytes"]
    assert out[0]["n_passes_a"] < out[1]["n_passes_a"]
    c.close()
