"""Chained launches: runs of small dependent passes in one cooperative launch, with a grid
barrier between the passes (tuning chain_passes = 1).

A chain runs the same pass code on the same arguments as one launch per pass; only which
workgroup takes which tile differs, and no tile's arithmetic depends on that, so the results
with and without chaining are equal bit for bit.  Each case also checks the oracle (Section 3's
path sum) and that chaining did happen: fewer sweep launches, passes reported as chained.
"""
import numpy as np
import pytest

import oracle
from parity_tol import TOL_C128, TOL_C64, c11_error
from workload import CONFIGS, ISWAP, grid_circuit, make_workload, random_bitstrings

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


def _both(sf, c, bits, tune, **kw):
    """Amplitudes and run statistics with chaining on, then off."""
    out = []
    for chain in (1, 0):
        c.tune(chain_passes=chain, **tune)
        a = c.amplitudes(bits, **kw)
        out.append((a, c.stats()))
    (a0, s0), (a1, s1) = out
    return a0, s0, a1, s1


@pytest.mark.parametrize("tune", [{"reg_qubits": 5}, {"reg_qubits": 4}, {"reg_qubits": 5, "dense_qubits": 2},
                                  {"reg_qubits": 5, "no_leaf_fold": 1}])
def test_chain_grid5x6_all_paths(sf, tune):
    w = make_workload("grid5x6_d24", n_bits=2000)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    say(f"chain grid5x6_d24 all paths {tune}")
    a0, s0, a1, s1 = _both(sf, c, w["bitstrings"], tune)
    assert s1["n_chained_passes"] == 0
    assert s0["n_chained_passes"] > 0, s0
    assert s0["n_sweep_launches"] < s1["n_sweep_launches"], (s0, s1)
    assert s0["sweep_bytes"] == s1["sweep_bytes"]
    assert np.array_equal(a0, a1)
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), np.arange(1 << c.k, dtype=np.uint64), w["bitstrings"])
    assert c11_error(a0, o, 1 << c.k, c.k, 30) <= TOL_C64
    c.close()


def test_chain_fp64_sweeps(sf):
    w = make_workload("grid4x4_d16", n_bits=1024)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    say("chain grid4x4_d16 all paths, FP64 sweeps")
    a0, s0, a1, s1 = _both(sf, c, w["bitstrings"], {"reg_qubits": 3}, flags=sf.SF_FP64_SWEEPS)
    assert s0["n_chained_passes"] > 0 and s0["n_sweep_launches"] < s1["n_sweep_launches"]
    assert np.array_equal(a0, a1)
    o = oracle.path_sum(16, w["gates"], cfg.cut_mask(), np.arange(1 << c.k, dtype=np.uint64), w["bitstrings"])
    assert c11_error(a0, o, 1 << c.k, c.k, 16) <= TOL_C128
    c.close()


def test_chain_iswap_flips(sf):
    """Crossing iSWAPs: passes that carry per-path flips run the flip variant of the chain."""
    g = grid_circuit(4, 4, 12, 5, two_qubit=ISWAP)
    m = CONFIGS["grid4x4_d16"].cut_mask()
    c = sf.Circuit(4, 4, g, m)
    bits = random_bitstrings(16, 1024, 3)
    say("chain iswap 4x4 d12 all paths")
    a0, s0, a1, s1 = _both(sf, c, bits, {"reg_qubits": 4})
    assert s0["n_chained_passes"] > 0
    assert np.array_equal(a0, a1)
    o = oracle.path_sum(16, g, m, np.arange(1 << c.k, dtype=np.uint64), bits)
    assert c11_error(a0, o, 1 << c.k, c.k, 16) <= TOL_C64
    c.close()


def test_chain_plain_form_rounds(sf):
    """Plain form: the launch sequence repeats once per path; the barrier counter keeps growing
    across the rounds of one call."""
    w = make_workload("grid5x6_d24", n_bits=500)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    ids = np.array([3, 77, 1000, 4097, 20000, 32767], dtype=np.uint64)
    say("chain grid5x6_d24 plain form, 6 paths")
    a0, s0, a1, s1 = _both(sf, c, w["bitstrings"], {"reg_qubits": 5}, path_ids=ids, flags=sf.SF_PLAIN)
    assert s0["n_chained_passes"] > 0
    assert np.array_equal(a0, a1)
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    assert c11_error(a0, o, ids.size, c.k, 30) <= TOL_C64
    c.close()


def test_chain_repeated_calls_same_plan(sf):
    """A repeated request reuses its plan; the chains' arguments are uploaded again and the
    barrier counter is cleared per call, so every call gives the same amplitudes."""
    w = make_workload("grid5x6_d24", n_bits=1000)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    c.tune(reg_qubits=5, chain_passes=1)
    say("chain grid5x6_d24 three calls")
    first = c.amplitudes(w["bitstrings"], path_begin=4096, n_paths=8192)
    for _ in range(2):
        assert np.array_equal(c.amplitudes(w["bitstrings"], path_begin=4096, n_paths=8192), first)
    assert c.stats()["n_chained_passes"] > 0
    c.close()
