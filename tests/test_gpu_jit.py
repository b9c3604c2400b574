"""Compiled passes (tuning jit = 1): every pass outside a chained launch that is not a dense block
runs a kernel compiled at run time for its program.

The compiled kernel runs the same device code as the interpreted one with the program's
operations as constants, so its amplitudes agree with the interpreted passes' to rounding (the
compiler contracts the constant-folded arithmetic into fused multiply-adds differently).  Each
case checks both against the oracle (Section 3's path sum), that the compiled passes did run,
and that a repeated request compiles nothing and gives the same amplitudes bit for bit.
"""
import numpy as np
import pytest

import oracle
from parity_tol import TOL_C128, TOL_C64, c11_error
from workload import ISWAP, grid_circuit, make_workload, random_bitstrings

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


def _both(c, bits, tune, **kw):
    """(amplitudes, stats) with compiled passes, again with compiled passes (cached kernels),
    and with interpreted passes."""
    out = []
    for jit in (1, 1, 0):
        c.tune(jit=jit, **tune)
        a = c.amplitudes(bits, **kw)
        out.append((a, c.stats()))
    return out


def _check_runs(out, expect_jit=True):
    (a0, s0), (a1, s1), (a2, s2) = out
    if expect_jit:
        assert s0["n_jit_passes"] > 0, s0
    assert s1["n_jit_passes"] == s0["n_jit_passes"]
    assert s1["jit_compile_ms"] == 0.0
    assert s2["n_jit_passes"] == 0
    assert np.array_equal(a0, a1)
    assert s0["sweep_bytes"] == s2["sweep_bytes"]
    return a0, a2


@pytest.mark.parametrize("tune", [{"reg_qubits": 5}, {"reg_qubits": 4}, {"reg_qubits": 3},
                                  {"reg_qubits": 5, "dense_qubits": 2}, {"reg_qubits": 5, "no_leaf_fold": 1},
                                  {"reg_qubits": 5, "fold_levels": 1}])
def test_jit_grid5x6_all_paths(sf, tune):
    w = make_workload("grid5x6_d24", n_bits=1500)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    say(f"compiled passes grid5x6_d24 all paths {tune}")
    a_jit, a_int = _check_runs(_both(c, w["bitstrings"], tune))
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), np.arange(1 << c.k, dtype=np.uint64), w["bitstrings"])
    for a in (a_jit, a_int):
        assert c11_error(a, o, 1 << c.k, c.k, 30) <= TOL_C64
    assert c11_error(a_jit, a_int, 1 << c.k, c.k, 30) <= TOL_C64
    c.close()


@pytest.mark.parametrize("paths", ["sparse", "subset"])
def test_jit_grid5x6_path_subsets(sf, paths):
    """Fan-outs, chain levels and padded batches with compiled passes."""
    w = make_workload("grid5x6_d24", n_bits=1200)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    rng = np.random.default_rng(21)
    size = 11 if paths == "sparse" else 900
    ids = np.sort(rng.choice(1 << c.k, size=size, replace=False)).astype(np.uint64)
    say(f"compiled passes grid5x6_d24 {paths} ({ids.size} paths)")
    a_jit, a_int = _check_runs(_both(c, w["bitstrings"], {"reg_qubits": 5, "max_slots": 64}, path_ids=ids))
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    for a in (a_jit, a_int):
        assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64
    c.close()


def test_jit_fp64_sweeps(sf):
    w = make_workload("grid4x4_d16", n_bits=1024)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    say("compiled passes grid4x4_d16 all paths, FP64 sweeps")
    a_jit, a_int = _check_runs(_both(c, w["bitstrings"], {"reg_qubits": 3}, flags=sf.SF_FP64_SWEEPS))
    o = oracle.path_sum(16, w["gates"], cfg.cut_mask(), np.arange(1 << c.k, dtype=np.uint64), w["bitstrings"])
    for a in (a_jit, a_int):
        assert c11_error(a, o, 1 << c.k, c.k, 16) <= TOL_C128
    c.close()


@pytest.mark.parametrize("seed", [1, 3])
def test_jit_deferred_level(sf, seed):
    g = grid_circuit(5, 4, 16, seed)
    c = sf.Circuit(5, 4, g)
    bits = random_bitstrings(20, 700, seed + 10)
    ids = np.arange(1 << c.k, dtype=np.uint64)
    say(f"compiled passes 5x4 d16 seed {seed}, deferred level")
    a_jit, a_int = _check_runs(_both(c, bits, {"fold_levels": 1}, path_ids=ids))
    o = oracle.path_sum(20, g, c.mask_a, ids, bits)
    for a in (a_jit, a_int):
        assert c11_error(a, o, ids.size, c.k, 20) <= TOL_C64
    c.close()


def test_jit_plain_form(sf):
    w = make_workload("grid5x6_d24", n_bits=600)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    ids = np.array([7, 1000, 20001], dtype=np.uint64)
    say("compiled passes grid5x6_d24 plain form, 3 paths")
    a_jit, a_int = _check_runs(_both(c, w["bitstrings"], {"reg_qubits": 5}, path_ids=ids, flags=sf.SF_PLAIN))
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    for a in (a_jit, a_int):
        assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64
    c.close()


@pytest.mark.parametrize("tune", [{"reg_qubits": 4}, {"reg_qubits": 2}, {"reg_qubits": 4, "no_leaf_fold": 1}])
def test_jit_iswap_circuit(sf, tune):
    """Crossing iSWAPs: per-path flips (with the factor i) and in-block iSWAPs on registers and
    lanes, compiled with constant positions."""
    g = grid_circuit(4, 4, 12, 5, two_qubit=ISWAP)
    c = sf.Circuit(4, 4, g)
    bits = random_bitstrings(16, 1024, 3)
    say(f"compiled passes iswap 4x4 d12 all paths {tune}")
    out = _both(c, bits, tune)
    a_jit, a_int = _check_runs(out)
    o = oracle.path_sum(16, g, c.mask_a, np.arange(1 << c.k, dtype=np.uint64), bits)
    for a in (a_jit, a_int):
        assert c11_error(a, o, 1 << c.k, c.k, 16) <= TOL_C64
    c.close()


def test_jit_iswap_grid5x6_subset(sf):
    """The iSWAP variant of the 5x6 benchmark circuit on a path subset (fan-outs with flips)."""
    from workload import CONFIGS
    cfg = CONFIGS["grid5x6_d24"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed, two_qubit=ISWAP)
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    bits = random_bitstrings(30, 800, 12)
    rng = np.random.default_rng(4)
    ids = np.sort(rng.choice(1 << c.k, size=600, replace=False)).astype(np.uint64)
    say("compiled passes iswap 5x6 d24, 600 paths")
    a_jit, a_int = _check_runs(_both(c, bits, {"reg_qubits": 5}, path_ids=ids))
    o = oracle.path_sum(30, g, cfg.cut_mask(), ids, bits)
    for a in (a_jit, a_int):
        assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64
    c.close()


def test_jit_with_chained_passes(sf):
    """Passes inside a chained launch stay interpreted; the rest are compiled."""
    w = make_workload("grid5x6_d24", n_bits=900)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    say("compiled passes with chained passes, grid5x6_d24")
    c.tune(reg_qubits=5, chain_passes=1, jit=1)
    a = c.amplitudes(w["bitstrings"])
    s = c.stats()
    assert s["n_chained_passes"] > 0
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), np.arange(1 << c.k, dtype=np.uint64), w["bitstrings"])
    assert c11_error(a, o, 1 << c.k, c.k, 30) <= TOL_C64
    c.close()
