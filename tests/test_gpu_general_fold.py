"""GPU parity of the general fold and of skipped zero-term paths, against the FP64 oracle.

General fold: the last tree level(s) applied inside the gather although their non-diagonal
gates also act on qubits other than the branch qubits (S' = those qubits plus the branch
qubits; 2^|S'| rows of the level above per bitstring and parent).  fold_levels set explicitly
forces it.  Zero-term paths: two projectors of Eq. (CZ) on one block-A qubit with only diagonal
gates in between and different path bits (Section 2 zero blocks); the library skips them and
the oracle, which evolves every listed path, gives them zero amplitude.

Tolerance: parity_tol.c11_error, 1e-5 (complex64 sweeps), 1e-10 (complex128 sweeps).
"""
import numpy as np
import pytest

import oracle
from parity_tol import TOL_C128, TOL_C64, c11_error
from workload import CONFIGS, column_cut_mask, equal_bit_pairs, grid_circuit, is_live, random_bitstrings

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


CIRCUITS = [(4, 4, 16, 1001, 2), (4, 5, 24, 2, 2), (5, 4, 24, 3, 2), (4, 4, 24, 3, 2)]


@pytest.mark.parametrize("rows,cols,depth,seed,ncols_a", CIRCUITS)
def test_general_fold_matches_oracle(sf, rows, cols, depth, seed, ncols_a):
    """All paths (the full output state), a sampled subset (parents with some descendants) and
    the plain form, at every fold depth whose plan is the general form, complex64 and
    complex128, against the oracle."""
    n = rows * cols
    g = grid_circuit(rows, cols, depth, seed)
    mask = column_cut_mask(rows, cols, ncols_a)
    c = sf.Circuit(rows, cols, g, mask)
    bits = np.arange(1 << n, dtype=np.uint64)[:: max(1, (1 << n) // 3000)]
    full = oracle.full_state(n, g)[bits.astype(np.int64)]
    ran = 0
    for F in (1, 2):
        c.tune(fold_levels=F)
        if "general form" not in sf.describe_plan(c.handle):
            continue
        ran += 1
        for fp64 in (False, True):
            say(f"{rows}x{cols} d{depth} seed {seed}: general fold F={F} all paths fp64={fp64}")
            a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS if fp64 else 0)
            assert c11_error(a, full, 1, 0, n) <= (TOL_C128 if fp64 else TOL_C64), (F, fp64)
        sub = sf.sample_paths(c.k, 0.4, 91 + F)
        say(f"{rows}x{cols} d{depth}: general fold F={F}, {sub.size} sampled paths")
        a = c.amplitudes(bits, path_ids=sub)
        o = oracle.path_sum(n, g, mask, sub, bits)
        assert c11_error(a, o, sub.size, c.k, n) <= TOL_C64, F
        # three paths of the subset whose terms are nonzero (by the oracle's block-A norms)
        _, na, _ = oracle.path_sum(n, g, mask, sub[:64], bits[:2], norms=True)
        live = [int(p) for p, v in zip(sub[:64], na) if v > 0][:3]
        assert len(live) == 3
        say(f"{rows}x{cols} d{depth}: general fold F={F}, plain form and single paths {live}")
        a = c.amplitudes(bits, path_ids=live, flags=sf.SF_PLAIN)
        o = oracle.path_sum(n, g, mask, live, bits)
        assert c11_error(a, o, len(live), c.k, n) <= TOL_C64, F
        for p in live:
            a = c.amplitudes(bits, path_ids=[p], flags=sf.SF_FP64_SWEEPS)
            o = oracle.path_sum(n, g, mask, [p], bits)
            assert np.abs(o).max() > 0
            assert c11_error(a, o, 1, c.k, n) <= TOL_C128, (F, p)
    assert ran, "no general-form fold depth in this circuit"
    c.close()


def test_zero_term_paths_are_skipped(sf):
    """A request mixing live and zero-term paths equals the oracle over the same list (the
    zero-term ones contribute nothing); a request of zero-term paths only writes zeros, or
    leaves the accumulated amplitudes unchanged."""
    cfg = CONFIGS["grid4x4_d16"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    mask = cfg.cut_mask()
    c = sf.Circuit(cfg.rows, cfg.cols, g, mask)
    pairs = equal_bit_pairs(g, mask)
    assert pairs
    ids = np.arange(1 << c.k, dtype=np.uint64)
    live = np.array([is_live(int(p), pairs) for p in ids])
    bits = random_bitstrings(16, 700, 4)
    for fp64 in (False, True):
        say(f"4x4: {live.sum()} live of {ids.size} paths, fp64={fp64}")
        a = c.amplitudes(bits, path_ids=ids[100:180], flags=sf.SF_FP64_SWEEPS if fp64 else 0)
        assert c.stats()["n_paths_live"] == int(live[100:180].sum())
        o = oracle.path_sum(16, g, mask, ids[100:180], bits)
        assert c11_error(a, o, 80, c.k, 16) <= (TOL_C128 if fp64 else TOL_C64)
    dead = ids[~live][:20]
    say("4x4: zero-term paths only")
    a = c.amplitudes(bits, path_ids=dead)
    assert np.all(a == 0) and c.stats()["n_paths_live"] == 0
    acc = np.full(2 * bits.size, 3.0)
    sf.run_paths(c.handle, dead, 0, dead.size, bits, bits.size, acc, sf.SF_ACCUMULATE)
    assert np.all(acc == 3.0)
    c.close()
