"""Paths whose term is exactly zero (host only).

Two projectors of Section 2, Eq. (CZ) on one block-A qubit with only diagonal gates on it in
between multiply to zero unless their path bits agree, so such paths carry no amplitude (the
paper's zero blocks, Section 2).  The seeded input generator (workload.equal_bit_pairs, which
picks live benchmark blocks) and the library (equal_bit_pairs in the planner, which skips dead
paths; printed by describe_plan) each derive the pairs of path bits that must agree from the
gate list.  Both are pinned here against the FP64 oracle's arithmetic: every path that
disagrees on a pair has block-A norm zero (the rule is sound: it never drops a nonzero term),
and on these circuits, the benchmark's 5x6 and 6x7 among them, the converse holds too.  Terms
can also vanish through longer chains of gates on several qubits (the last case below), which
the rule does not see; such paths are computed and contribute zero.
"""
import re

import numpy as np
import pytest

import oracle
from workload import (CONFIGS, GATE_DTYPE, CZ, H, T, XH, equal_bit_pairs, grid_circuit, is_live,
                      random_bitstrings, workload_block)


@pytest.fixture(scope="module")
def sf():
    from paper_1807_10749_amd import binding
    return binding


def library_pairs(sf, rows, cols, gates, mask):
    c = sf.create_circuit(rows, cols, gates)
    sf.set_cut(c, mask)
    line = [l for l in sf.describe_plan(c).splitlines() if l.startswith("equal path bits:")][0]
    sf.destroy_circuit(c)
    return sorted(tuple(int(v) for v in m.split("=")) for m in re.findall(r"\d+=\d+", line))


@pytest.mark.parametrize("rows,cols,depth,seed,ncols_a", [(4, 4, 16, 1001, 2), (3, 4, 18, 7, 2), (4, 4, 24, 3, 2),
                                                         (3, 5, 20, 11, 3)])
def test_zero_terms_are_exactly_the_unequal_pairs(sf, rows, cols, depth, seed, ncols_a):
    from workload import column_cut_mask
    n = rows * cols
    g = grid_circuit(rows, cols, depth, seed)
    mask = column_cut_mask(rows, cols, ncols_a)
    k = oracle.num_cut(n, g, mask)
    pairs = equal_bit_pairs(g, mask)
    assert sorted(pairs) == library_pairs(sf, rows, cols, g, mask)
    ids = np.arange(1 << k, dtype=np.uint64) if k <= 10 else np.sort(
        np.random.default_rng(seed).choice(1 << k, 512, replace=False)).astype(np.uint64)
    _, na, nb = oracle.path_sum(n, g, mask, ids, random_bitstrings(n, 4, 1), norms=True)
    live = np.array([is_live(int(p), pairs) for p in ids])
    assert np.all(nb > 0.5)                       # block B sees only unitaries (I and Z)
    assert np.all(na[~live] == 0.0)
    assert np.all(na[live] > 1e-12)
    assert 0 < live.sum() < ids.size or not pairs


def test_rule_is_sound_where_other_zeros_exist(sf):
    """A 5x4 circuit with zero terms beyond the pairs: no path the rule rejects has a nonzero
    term, and the library finds the same pairs."""
    from workload import column_cut_mask
    g = grid_circuit(5, 4, 24, 3)
    mask = column_cut_mask(5, 4, 2)
    pairs = equal_bit_pairs(g, mask)
    assert sorted(pairs) == library_pairs(sf, 5, 4, g, mask)
    k = oracle.num_cut(20, g, mask)
    ids = np.sort(np.random.default_rng(2).choice(1 << k, 600, replace=False)).astype(np.uint64)
    _, na, _ = oracle.path_sum(20, g, mask, ids, random_bitstrings(20, 2, 1), norms=True)
    live = np.array([is_live(int(p), pairs) for p in ids])
    assert np.all(na[~live] == 0.0)
    assert np.any(na[live] == 0.0)


def test_hand_built_pairs():
    """Qubit 0 (block A) meets crossing CZs at cycles 1, 3 and 5 with a T (diagonal) between the
    first two and an X^1/2 between the last two: the bits of the first two must agree, the third
    is free.  Qubit 2's two crossing CZs are separated by an H."""
    # 2x2 grid with block A = column 0 (qubits 0, 2): crossing edges are 0-1 and 2-3
    g = [(H, 0, 0, q, 0) for q in range(4)]
    g += [(CZ, 0, 1, 0, 1), (CZ, 0, 1, 2, 3)]
    g += [(T, 0, 2, 0, 0), (H, 0, 2, 2, 0)]
    g += [(CZ, 0, 3, 0, 1), (CZ, 0, 3, 2, 3)]
    g += [(XH, 0, 4, 0, 0)]
    g += [(CZ, 0, 5, 0, 1)]
    g += [(H, 0, 6, q, 0) for q in range(4)]
    g = np.array(g, dtype=GATE_DTYPE)
    mask = 0b0101
    # path bits, earliest first: cycle 1 (0-1) bit 4, (2-3) bit 3; cycle 3 (0-1) bit 2, (2-3) bit 1;
    # cycle 5 (0-1) bit 0.  Qubit 0: cycle 1 and 3 separated by T only -> bits 4 and 2 agree.
    assert equal_bit_pairs(g, mask) == [(4, 2)]
    _, na, _ = oracle.path_sum(4, g, mask, np.arange(32, dtype=np.uint64), np.arange(16, dtype=np.uint64),
                               norms=True)
    for p in range(32):
        assert (na[p] == 0.0) == (((p >> 4) ^ (p >> 2)) & 1 == 1), p


def test_benchmark_block_is_live():
    """The 7x8 benchmark block is live (its shared prefix agrees on every pair) and every path of
    it too: the pairs only involve the bits of the first crossing cycles."""
    cfg = CONFIGS["grid7x8_d40"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    pairs = equal_bit_pairs(g, cfg.cut_mask())
    assert len(pairs) == 3
    begin, count = workload_block("grid7x8_d40")
    assert count == 1024 and begin % 1024 == 0
    assert all(is_live(p, pairs) for p in range(begin, begin + count))
