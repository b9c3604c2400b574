"""GPU parity of crossing and in-block iSWAP gates (Eq. (4way), Eq. (iSWAP1)).

Each crossing iSWAP takes two path bits; term r = 2i + j applies |i><j| on the
block-A endpoint and the 2x2 block G_ij on the block-B endpoint.  Single-path
runs compare individual terms, so a swapped term order or a wrong phase is an
O(1) error; full sums are also checked against the oracle's state vector.
"""
import numpy as np
import pytest

import oracle
from parity_tol import TOL_C128, TOL_C64, c11_error
from fold_circuits import iswap_tail_circuit
from workload import CONFIGS, CZ, ISWAP, column_cut_mask, grid_circuit, path_block, random_bitstrings, workload_block

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


def mixed_circuit(rows, cols, depth, seed, mask, iswap_before):
    """The CZ circuit with every crossing two-qubit gate of a cycle below iswap_before made an
    iSWAP (later crossing gates stay CZ, so the trailing tree levels can be folded)."""
    g = grid_circuit(rows, cols, depth, seed)
    for t in range(g.size):
        if g["kind"][t] == CZ and g["cycle"][t] < iswap_before:
            a, b = int(g["q0"][t]), int(g["q1"][t])
            if ((mask >> a) & 1) != ((mask >> b) & 1):
                g["kind"][t] = ISWAP
    return g


G44 = dict(rows=4, cols=4, depth=12, seed=5)


def _g44(sf):
    g = grid_circuit(G44["rows"], G44["cols"], G44["depth"], G44["seed"], two_qubit=ISWAP)
    m = CONFIGS["grid4x4_d16"].cut_mask()
    return g, m, sf.Circuit(4, 4, g, m)


@pytest.mark.parametrize("fp64", [True, False])
def test_iswap_grid4x4_all_paths(sf, fp64):
    g, m, c = _g44(sf)
    assert c.k == 12
    bits = random_bitstrings(16, 1024, 3)
    say(f"iswap 4x4 d12 all paths fp64={fp64}")
    a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS if fp64 else 0)
    o = oracle.path_sum(16, g, m, np.arange(1 << c.k, dtype=np.uint64), bits)
    assert np.abs(o - oracle.full_state(16, g)[bits.astype(np.int64)]).max() < 1e-14
    err = c11_error(a, o, 1 << c.k, c.k, 16)
    assert err <= (TOL_C128 if fp64 else TOL_C64), err


@pytest.mark.parametrize("path", [0, 1, 2, 3, 6, 9, 0x5A5, 2047, 4095])
def test_iswap_single_path_terms(sf, path):
    g, m, c = _g44(sf)
    bits = np.arange(1 << 16, dtype=np.uint64)[::37]
    say(f"iswap 4x4 d12 single path {path}")
    a = c.amplitudes(bits, path_begin=path, n_paths=1, flags=sf.SF_FP64_SWEEPS)
    o = oracle.path_sum(16, g, m, [path], bits)
    assert c11_error(a, o, 1, c.k, 16) <= TOL_C128   # terms 9 and 0x5A5 vanish on every bitstring


def test_iswap_plain_equals_batched(sf):
    g, m, c = _g44(sf)
    bits = random_bitstrings(16, 512, 6)
    ids = np.array([3, 4, 5, 17, 100, 101, 250, 1024, 1027, 4000], dtype=np.uint64)
    say("iswap 4x4 d12 plain vs batched")
    a = c.amplitudes(bits, path_ids=ids, flags=sf.SF_PLAIN)
    b = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(16, g, m, ids, bits)
    assert c11_error(a, o, ids.size, c.k, 16) <= TOL_C64
    assert c11_error(b, o, ids.size, c.k, 16) <= TOL_C64


@pytest.mark.parametrize("fp64", [True, False])
def test_iswap_small_blocks_lane_flips(sf, fp64):
    """4 + 4 qubit blocks: every qubit sits in a lane bit, so the per-path flips are shuffles."""
    g = grid_circuit(2, 4, 10, 44, two_qubit=ISWAP)
    mask = column_cut_mask(2, 4, 2)
    c = sf.Circuit(2, 4, g, mask)
    bits = np.arange(256, dtype=np.uint64)
    say(f"iswap 2x4 d10 fp64={fp64} k={c.k}")
    a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS if fp64 else 0)
    o = oracle.full_state(8, g)
    assert c11_error(a, o, 1, 0, 8) <= (TOL_C128 if fp64 else TOL_C64)


def test_iswap_grid5x6_aligned_block_and_ids(sf):
    cfg = CONFIGS["grid5x6_d24"]
    g = grid_circuit(5, 6, 24, cfg.circuit_seed, two_qubit=ISWAP)
    c = sf.Circuit(5, 6, g, cfg.cut_mask())
    assert c.k == 30
    bits = random_bitstrings(30, 2048, 4)
    begin, count = path_block(c.k, 10, 12)
    say(f"iswap 5x6 d24 aligned block begin={begin} count={count}")
    a = c.amplitudes(bits, path_begin=begin, n_paths=count)
    o = oracle.path_sum(30, g, cfg.cut_mask(), np.arange(begin, begin + count, dtype=np.uint64), bits)
    assert c11_error(a, o, count, c.k, 30) <= TOL_C64
    ids = np.unique(np.random.default_rng(1).integers(0, 1 << 30, 64).astype(np.uint64))
    say("iswap 5x6 d24 scattered ids fp64")
    a = c.amplitudes(bits, path_ids=ids, flags=sf.SF_FP64_SWEEPS)
    o = oracle.path_sum(30, g, cfg.cut_mask(), ids, bits)
    assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C128


@pytest.mark.parametrize("no_fold", [0, 1])
def test_mixed_cz_iswap_with_folded_tail(sf, no_fold):
    """iSWAPs in the early levels, CZs in the trailing ones: the CZ levels are folded into the
    gather (unless switched off) while the iSWAP levels run as passes."""
    cfg = CONFIGS["grid5x6_d24"]
    m = cfg.cut_mask()
    g = mixed_circuit(5, 6, 24, cfg.circuit_seed, m, 12)
    c = sf.Circuit(5, 6, g, m)
    c.tune(no_leaf_fold=no_fold)
    plan = sf.describe_plan(c.handle)
    assert ("folded" in plan) == (not no_fold), plan
    bits = random_bitstrings(30, 1024, 8)
    begin, count = path_block(c.k, 11, 3)
    say(f"mixed 5x6 d24 k={c.k} no_fold={no_fold} block {begin}+{count}")
    a = c.amplitudes(bits, path_begin=begin, n_paths=count)
    o = oracle.path_sum(30, g, m, np.arange(begin, begin + count, dtype=np.uint64), bits)
    assert c11_error(a, o, count, c.k, 30) <= TOL_C64


def test_iswap_grid6x7_sampled_paths(sf):
    cfg = CONFIGS["grid6x7_d32"]
    g = grid_circuit(6, 7, 32, cfg.circuit_seed, two_qubit=ISWAP)
    c = sf.Circuit(6, 7, g, cfg.cut_mask())
    assert c.k == 56
    bits = random_bitstrings(42, 256, 9)
    ids = np.array([0, (1 << 56) - 1, 0x00F0F0F0F0F0F0F], dtype=np.uint64)
    say("iswap 6x7 d32 three paths")
    a = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(42, g, cfg.cut_mask(), ids, bits)
    assert c11_error(a, o, ids.size, c.k, 42) <= TOL_C64


@pytest.mark.slow
def test_iswap_full_workload_block(sf):
    """The iSWAP variant at its measured size (aligned block of 2^18 paths, 1e5 bitstrings,
    default launch configuration): the block equals the sum of its quarters, and an aligned
    1024-path sub-block matches the oracle on every bitstring."""
    from workload import make_workload
    w = make_workload("grid5x6_d24_iswap")
    cfg, g, bits = w["cfg"], w["gates"], w["bitstrings"]
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    begin, count = workload_block(cfg.name)
    assert (c.k, count) == (30, 1 << 18)
    say(f"iswap 5x6 d24 full block {begin}+{count}, 1e5 bitstrings")
    a = c.amplitudes(bits, path_begin=begin, n_paths=count)
    q = np.zeros_like(a)
    for i in range(4):
        say(f"iswap 5x6 d24 quarter {i}")
        q += c.amplitudes(bits, path_begin=begin + i * (count // 4), n_paths=count // 4)
    assert np.abs(a - q).max() <= 1e-5 * np.abs(a).max()
    sub = begin + 173 * 1024
    say(f"iswap 5x6 d24 sub-block {sub}+1024 against the oracle")
    a = c.amplitudes(bits, path_begin=sub, n_paths=1024)
    o = oracle.path_sum(30, g, cfg.cut_mask(), np.arange(sub, sub + 1024, dtype=np.uint64), bits)
    assert c11_error(a, o, 1024, c.k, 30) <= TOL_C64


# ---------------------------------------------------------------- trailing iSWAP levels folded into the gather

@pytest.mark.parametrize("shape", [(3, 4, 6, 1), (3, 5, 10, 2), (2, 6, 16, 1), (3, 6, 16, 2)])
@pytest.mark.parametrize("fp64", [True, False])
def test_iswap_fold_small_grids(sf, shape, fp64):
    r, cc, d, seed = shape
    g = grid_circuit(r, cc, d, seed, two_qubit=ISWAP)
    m = column_cut_mask(r, cc, cc // 2)
    c = sf.Circuit(r, cc, g, m)
    assert "iSWAP gates" in sf.describe_plan(c.handle)
    n = r * cc
    bits = np.arange(1 << n, dtype=np.uint64)[:: max(1, (1 << n) // 4096)]
    flags = sf.SF_FP64_SWEEPS if fp64 else 0
    say(f"iswap fold {shape} fp64={fp64} k={c.k}")
    a = c.amplitudes(bits, flags=flags)
    o = oracle.path_sum(n, g, m, np.arange(1 << c.k, dtype=np.uint64), bits)
    assert c11_error(a, o, 1 << c.k, c.k, n) <= (TOL_C128 if fp64 else TOL_C64)
    c.tune(no_leaf_fold=1)
    b = c.amplitudes(bits, flags=flags)
    assert c11_error(b, o, 1 << c.k, c.k, n) <= (TOL_C128 if fp64 else TOL_C64)


@pytest.mark.parametrize("drop", [(), (5, 2), (1, 6)])
def test_iswap_fold_two_levels(sf, drop):
    """Two folded levels, gate qubits inside and outside S; all paths, every single path (the
    masked form), scattered subsets and the one-path-at-a-time form."""
    r, cc, g, m = iswap_tail_circuit(drop)
    c = sf.Circuit(r, cc, g, m)
    assert "2 levels" in sf.describe_plan(c.handle)
    bits = np.arange(256, dtype=np.uint64)
    say(f"iswap two-level fold drop={drop} all paths")
    a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS)
    assert c11_error(a, oracle.full_state(8, g), 1, 0, 8) <= TOL_C128
    for p in range(1 << c.k):
        a = c.amplitudes(bits, path_begin=p, n_paths=1, flags=sf.SF_FP64_SWEEPS)
        o = oracle.path_sum(8, g, m, [p], bits)
        assert c11_error(a, o, 1, c.k, 8) <= TOL_C128, p
    ids = np.array([1, 2, 7, 8, 13, 14], dtype=np.uint64)
    say(f"iswap two-level fold drop={drop} subsets, plain")
    o = oracle.path_sum(8, g, m, ids, bits)
    for flags in (0, sf.SF_FP64_SWEEPS, sf.SF_PLAIN):
        a = c.amplitudes(bits, path_ids=ids, flags=flags)
        assert c11_error(a, o, ids.size, c.k, 8) <= (TOL_C128 if flags == sf.SF_FP64_SWEEPS else TOL_C64), flags
