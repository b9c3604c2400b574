"""Chain levels planned as one segment (tuning no_chain_merge = 0, the default).

A chain level is a tree level where every node has exactly one child (Section 3's prefix tree
over a path subset: the descendants of a node decided by a single requested path), so its block
states are evolved in place.  A run of such levels, with the root in front of it, is planned as
one segment: the operations of all its levels (their branch operators included, Section 2,
Eq. (CZ)) share passes, which the planner takes only when that needs no more passes than one
segment per level.  Each case checks the oracle (Section 3's path sum) with and without merging,
and that merging never adds passes.
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
    """Amplitudes and pass counts with merging on, then off."""
    out = []
    for nm in (0, 1):
        c.tune(no_chain_merge=nm, **tune)
        a = c.amplitudes(bits, **kw)
        s = c.stats()
        out.append((a, s["n_passes_a"] + s["n_passes_b"]))
    return out


@pytest.mark.parametrize("paths", ["sparse", "subset", "block"])
@pytest.mark.parametrize("tune", [{"reg_qubits": 5}, {"reg_qubits": 4}, {"reg_qubits": 5, "dense_qubits": 2},
                                  {"reg_qubits": 5, "no_leaf_fold": 1}])
def test_chain_merge_grid5x6(sf, paths, tune):
    w = make_workload("grid5x6_d24", n_bits=1500)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    rng = np.random.default_rng(11)
    if paths == "sparse":
        ids = np.sort(rng.choice(1 << c.k, size=9, replace=False)).astype(np.uint64)
    elif paths == "subset":
        ids = np.sort(rng.choice(1 << c.k, size=700, replace=False)).astype(np.uint64)
    else:
        ids = np.arange(4096, 4096 + 64, dtype=np.uint64)
    say(f"chain merge grid5x6_d24 {paths} ({ids.size} paths) {tune}")
    (a0, n0), (a1, n1) = _both(c, w["bitstrings"], tune, path_ids=ids)
    assert n0 <= n1, (n0, n1)
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    for a in (a0, a1):
        assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64
    c.close()


def test_chain_merge_plain_form(sf):
    """Plain form: every path its own one-node-per-level tree, so the whole tree above the path
    sum is one chain; merging takes fewer passes."""
    w = make_workload("grid5x6_d24", n_bits=800)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    ids = np.array([5, 900, 4097, 31000], dtype=np.uint64)
    say("chain merge grid5x6_d24 plain form, 4 paths")
    (a0, n0), (a1, n1) = _both(c, w["bitstrings"], {"reg_qubits": 5}, path_ids=ids, flags=sf.SF_PLAIN)
    assert n0 < n1, (n0, n1)
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    for a in (a0, a1):
        assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64
    c.close()


def test_chain_merge_fp64_sweeps(sf):
    w = make_workload("grid4x4_d16", n_bits=1024)
    cfg = w["cfg"]
    c = sf.Circuit(cfg.rows, cfg.cols, w["gates"], cfg.cut_mask())
    ids = np.array([1, 40, 77, 200], dtype=np.uint64)
    say("chain merge grid4x4_d16 4 paths, FP64 sweeps")
    (a0, n0), (a1, n1) = _both(c, w["bitstrings"], {"reg_qubits": 3}, path_ids=ids, flags=sf.SF_FP64_SWEEPS)
    assert n0 <= n1
    o = oracle.path_sum(16, w["gates"], cfg.cut_mask(), ids, w["bitstrings"])
    for a in (a0, a1):
        assert c11_error(a, o, ids.size, c.k, 16) <= TOL_C128
    c.close()


def test_chain_merge_iswap(sf):
    """Crossing iSWAPs: the merged segment carries the branch operators of several levels, each
    with its per-path flips."""
    g = grid_circuit(4, 5, 14, 6, two_qubit=ISWAP)
    c = sf.Circuit(4, 5, g)
    bits = random_bitstrings(20, 900, 8)
    rng = np.random.default_rng(3)
    ids = np.sort(rng.choice(1 << c.k, size=min(6, 1 << c.k), replace=False)).astype(np.uint64)
    say(f"chain merge iswap 4x5 d14, {ids.size} paths")
    (a0, n0), (a1, n1) = _both(c, bits, {"reg_qubits": 4}, path_ids=ids)
    assert n0 <= n1
    o = oracle.path_sum(20, g, c.mask_a, ids, bits)
    for a in (a0, a1):
        assert c11_error(a, o, ids.size, c.k, 20) <= TOL_C64
    c.close()


@pytest.mark.parametrize("seed", [1, 3])
def test_chain_merge_stops_before_deferred_level(sf, seed):
    """With the deferred block-A level, a chain run ends above it: the fold reads the parent
    batch in place."""
    g = grid_circuit(5, 4, 16, seed)
    c = sf.Circuit(5, 4, g)
    c.tune(fold_levels=1)
    assert "A deferred" in sf.describe_plan(c.handle)
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(1 << c.k, size=5, replace=False)).astype(np.uint64)
    bits = random_bitstrings(20, 600, seed + 4)
    say(f"chain merge 5x4 d16 seed {seed} deferred level, 5 paths")
    (a0, n0), (a1, n1) = _both(c, bits, {"fold_levels": 1}, path_ids=ids)
    assert n0 <= n1
    o = oracle.path_sum(20, g, c.mask_a, ids, bits)
    for a in (a0, a1):
        assert c11_error(a, o, ids.size, c.k, 20) <= TOL_C64
    c.close()
