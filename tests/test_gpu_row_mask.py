"""Row masks: the last pass of each block at the level the path sum reads computes only the
tiles holding rows that the requested bitstrings read (tuning no_row_skip = 0, the default).

The tiles that are computed run the same code on the same inputs either way, and the path sum
reads nothing else, so the amplitudes with and without the masks are equal bit for bit.  The
cases cover the plain gather, the narrow and the general fold, the iSWAP fold, FP64 sweeps, the
plain form and several batches at the read level; each also checks the oracle (Section 3's path
sum) and that a mask was used (run statistic row_mask_frac).
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


def _both(c, bits, tune, **kw):
    """Amplitudes and statistics with the masks, then without."""
    out = []
    for off in (0, 1):
        c.tune(no_row_skip=off, **tune)
        out.append((c.amplitudes(bits, **kw), c.stats()))
    return out[0][0], out[0][1], out[1][0], out[1][1]


@pytest.fixture(scope="module")
def w5x6():
    w = make_workload("grid5x6_d24", n_bits=3)
    cfg = w["cfg"]
    say("oracle grid5x6_d24 all paths, 3 bitstrings")
    w["oracle"] = oracle.path_sum(30, w["gates"], cfg.cut_mask(), np.arange(1 << 15, dtype=np.uint64),
                                  w["bitstrings"])
    return w


@pytest.mark.parametrize("tune", [{"reg_qubits": 5, "fold_levels": 2}, {"reg_qubits": 5, "no_leaf_fold": 1},
                                  {"reg_qubits": 4, "fold_levels": 1}, {"reg_qubits": 5, "no_leaf_fold": 1,
                                                                        "leaf_batch": 256}])
def test_row_mask_grid5x6(sf, w5x6, tune):
    w = w5x6
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    assert c.k == 15
    bits = w["bitstrings"]
    say(f"row mask grid5x6_d24 all paths, 3 bitstrings {tune}")
    a0, s0, a1, s1 = _both(c, bits, tune)
    assert max(s0["row_mask_frac"]) > 0.0, s0["row_mask_frac"]
    assert s1["row_mask_frac"] == [0.0, 0.0]
    assert s0["sweep_bytes"] < s1["sweep_bytes"]
    assert np.array_equal(a0, a1)
    assert c11_error(a0, w["oracle"], 1 << c.k, c.k, 30) <= TOL_C64
    c.close()


def test_row_mask_plain_form(sf):
    w = make_workload("grid5x6_d24", n_bits=2)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    ids = np.array([5, 999, 4100, 30001], dtype=np.uint64)
    say("row mask grid5x6_d24 plain form")
    a0, s0, a1, _ = _both(c, w["bitstrings"], {"reg_qubits": 5}, path_ids=ids, flags=sf.SF_PLAIN)
    assert max(s0["row_mask_frac"]) > 0.0
    assert np.array_equal(a0, a1)
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    assert c11_error(a0, o, ids.size, c.k, 30) <= TOL_C64
    c.close()


def test_row_mask_fp64_and_iswap(sf):
    g = grid_circuit(5, 5, 14, 8, two_qubit=ISWAP)
    m = 0
    for q in range(25):
        if q % 5 < 2:
            m |= 1 << q
    c = sf.Circuit(5, 5, g, m)
    bits = random_bitstrings(25, 2, 4)
    ids = np.arange(1 << min(c.k, 10), dtype=np.uint64)
    for flags, tol in ((0, TOL_C64), (sf.SF_FP64_SWEEPS, TOL_C128)):
        say(f"row mask iswap 5x5 d14 flags={flags}")
        a0, s0, a1, _ = _both(c, bits, {"reg_qubits": 4}, path_ids=ids, flags=flags)
        assert np.array_equal(a0, a1)
        o = oracle.path_sum(25, g, m, ids, bits)
        assert c11_error(a0, o, ids.size, c.k, 25) <= tol
    c.close()


def test_row_mask_grid6x7_general_fold(sf):
    """The 6x7 circuit's last level folded in the general form, a few bitstrings: the tiles of a
    21-qubit block that the folds' rows touch."""
    cfg = CONFIGS["grid6x7_d32"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    bits = random_bitstrings(42, 16, cfg.bits_seed)
    ids = np.arange(64, dtype=np.uint64)          # live: every pair of equal path bits is 0
    say("row mask grid6x7_d32 64 paths, 16 bitstrings")
    a0, s0, a1, _ = _both(c, bits, {"fold_levels": 1}, path_ids=ids)
    assert max(s0["row_mask_frac"]) > 0.0, s0["row_mask_frac"]
    assert np.array_equal(a0, a1)
    live = s0["n_paths_live"]
    o = oracle.path_sum(42, g, cfg.cut_mask(), ids, bits)
    assert c11_error(a0, o, max(live, 1), c.k, 42) <= TOL_C64
    c.close()
