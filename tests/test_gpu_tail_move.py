"""A segment's last pass left to the children's fan-out (tuning no_tail_move = 0, the default).

When a block's children are written by a fan-out, the parent's last in-place pass can be applied
by the children's first pass instead (its operations in front of the children's own, Section 3's
prefix tree evolved one level further): the parent batch is then never written in its final
form, only read by the fan-out.  Each case checks the oracle (Section 3's path sum) with and
without the move, and that the move never adds passes.
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
    """Amplitudes and total planned passes with the move, then without."""
    out = []
    for nt in (0, 1):
        c.tune(no_tail_move=nt, **tune)
        a = c.amplitudes(bits, **kw)
        s = c.stats()
        out.append((a, s["n_passes_a"] + s["n_passes_b"], s["sweep_bytes"]))
    return out


@pytest.mark.parametrize("paths", ["all", "sparse", "subset", "block"])
@pytest.mark.parametrize("tune", [{"reg_qubits": 5}, {"reg_qubits": 4}, {"reg_qubits": 5, "dense_qubits": 2},
                                  {"reg_qubits": 5, "no_leaf_fold": 1}, {"reg_qubits": 5, "jit": 1},
                                  {"reg_qubits": 5, "max_slots": 64}])
def test_tail_move_grid5x6(sf, paths, tune):
    w = make_workload("grid5x6_d24", n_bits=1200)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    rng = np.random.default_rng(17)
    if paths == "all":
        ids = np.arange(1 << c.k, dtype=np.uint64)
    elif paths == "sparse":
        ids = np.sort(rng.choice(1 << c.k, size=13, replace=False)).astype(np.uint64)
    elif paths == "subset":
        ids = np.sort(rng.choice(1 << c.k, size=900, replace=False)).astype(np.uint64)
    else:
        ids = np.arange(8192, 8192 + 256, dtype=np.uint64)
    say(f"tail move grid5x6_d24 {paths} ({ids.size} paths) {tune}")
    (a0, n0, b0), (a1, n1, b1) = _both(c, w["bitstrings"], tune, path_ids=ids)
    assert n0 <= n1 and b0 <= b1, (n0, n1, b0, b1)
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    for a in (a0, a1):
        assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64
    c.close()


def test_tail_move_takes_place(sf):
    """On the 5x6 circuit's all-paths request some block leaves a pass to its children."""
    w = make_workload("grid5x6_d24", n_bits=300)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    moved = False
    for tune in ({"reg_qubits": 5}, {"reg_qubits": 4}, {"reg_qubits": 3}):
        say(f"tail move grid5x6_d24 pass counts {tune}")
        (_, n0, b0), (_, n1, b1) = _both(c, w["bitstrings"], tune)
        moved = moved or (n0 < n1 and b0 < b1)
    assert moved
    c.close()


def test_tail_move_fp64_sweeps(sf):
    w = make_workload("grid4x4_d16", n_bits=1024)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    ids = np.arange(1 << c.k, dtype=np.uint64)
    say("tail move grid4x4_d16 all paths, FP64 sweeps")
    for R in (2, 3):
        (a0, n0, _), (a1, n1, _) = _both(c, w["bitstrings"], {"reg_qubits": R, "no_leaf_fold": 1}, path_ids=ids,
                                         flags=sf.SF_FP64_SWEEPS)
        assert n0 <= n1
        o = oracle.path_sum(16, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
        for a in (a0, a1):
            assert c11_error(a, o, ids.size, c.k, 16) <= TOL_C128
    c.close()


@pytest.mark.parametrize("tune", [{"reg_qubits": 4}, {"reg_qubits": 3}, {"reg_qubits": 4, "jit": 1}])
def test_tail_move_iswap(sf, tune):
    """Crossing iSWAPs: the moved pass may hold per-path flips, which the children apply with
    their own path bits."""
    g = grid_circuit(4, 5, 14, 6, two_qubit=ISWAP)
    c = sf.Circuit(4, 5, g)
    bits = random_bitstrings(20, 900, 8)
    ids = np.arange(1 << c.k, dtype=np.uint64)
    say(f"tail move iswap 4x5 d14 all paths {tune}")
    (a0, n0, _), (a1, n1, _) = _both(c, bits, tune, path_ids=ids)
    assert n0 <= n1
    o = oracle.path_sum(20, g, c.mask_a, ids, bits)
    for a in (a0, a1):
        assert c11_error(a, o, ids.size, c.k, 20) <= TOL_C64
    c.close()


@pytest.mark.parametrize("seed", [1, 3])
def test_tail_move_with_deferred_level(sf, seed):
    """Block A's batch that the fold reads as the deferred level's parent keeps its last pass."""
    g = grid_circuit(5, 4, 16, seed)
    c = sf.Circuit(5, 4, g)
    bits = random_bitstrings(20, 700, seed + 10)
    for paths in ("all", "subset"):
        ids = np.arange(1 << c.k, dtype=np.uint64) if paths == "all" else \
            np.sort(np.random.default_rng(seed).choice(1 << c.k, size=(1 << c.k) // 3, replace=False)).astype(np.uint64)
        say(f"tail move 5x4 d16 seed {seed} deferred level, {paths}")
        (a0, n0, _), (a1, n1, _) = _both(c, bits, {"fold_levels": 1}, path_ids=ids)
        assert n0 <= n1
        o = oracle.path_sum(20, g, c.mask_a, ids, bits)
        for a in (a0, a1):
            assert c11_error(a, o, ids.size, c.k, 20) <= TOL_C64
    c.close()


def test_tail_move_plain_form(sf):
    w = make_workload("grid5x6_d24", n_bits=600)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    ids = np.array([9, 2222, 30001], dtype=np.uint64)
    say("tail move grid5x6_d24 plain form, 3 paths")
    (a0, _, _), (a1, _, _) = _both(c, w["bitstrings"], {"reg_qubits": 5}, path_ids=ids, flags=sf.SF_PLAIN)
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    for a in (a0, a1):
        assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64
    c.close()
