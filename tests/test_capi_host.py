"""Host-only checks of the C-ABI library: exports, validation, cut, path selection.

No GPU compute is called here: run_paths is only exercised on argument
errors that the library rejects before touching the device.
"""
import json
import math
import os
import re

import numpy as np
import pytest

import oracle
from workload import CONFIGS, CZ, GATE_DTYPE, H, ISWAP, grid_circuit, make_workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfpath.h")


@pytest.fixture(scope="module")
def sf():
    from paper_1807_10749_amd import binding
    return binding


def test_library_exports_every_declared_function(sf):
    text = open(HEADER).read()
    declared = set(re.findall(r"^(?:int|const char \*)\s*(\w+)\(", text, re.M))
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(sf.lib, name), name
    assert declared == set(sf.EXPORTS)


def test_create_circuit_validation(sf):
    ok = np.array([(H, 0, 0, 0, 0), (CZ, 0, 1, 0, 1)], dtype=GATE_DTYPE)
    c = sf.create_circuit(2, 2, ok)
    sf.destroy_circuit(c)
    bad = [
        np.array([(7, 0, 0, 0, 0)], dtype=GATE_DTYPE),                       # unknown kind
        np.array([(H, 0, 0, 4, 0)], dtype=GATE_DTYPE),                       # outside grid
        np.array([(CZ, 0, 0, 0, 3)], dtype=GATE_DTYPE),                      # not neighbours (diagonal)
        np.array([(H, 0, 2, 0, 0), (H, 0, 1, 1, 0)], dtype=GATE_DTYPE),      # cycle decreases
        np.array([(H, 0, 1, 0, 0), (CZ, 0, 1, 0, 1)], dtype=GATE_DTYPE),     # qubit twice in a cycle
    ]
    for g in bad:
        with pytest.raises(sf.SFError) as e:
            sf.create_circuit(2, 2, g)
        assert e.value.code == sf.SF_ERR_INVALID
    with pytest.raises(sf.SFError) as e:
        sf.create_circuit(9, 8, ok)
    assert e.value.code == sf.SF_ERR_UNSUPPORTED


def test_set_cut_counts_match_oracle(sf):
    for name, cfg in CONFIGS.items():
        g = make_workload(name, n_bits=1)["gates"]
        c = sf.create_circuit(cfg.rows, cfg.cols, g)
        k = sf.set_cut(c, cfg.cut_mask())
        assert k == oracle.num_cut(cfg.n_qubits, g, cfg.cut_mask()), name
        sf.destroy_circuit(c)


def test_iswap_path_bits(sf):
    """A crossing iSWAP takes two path bits (four terms, Eq. (4way)); 80 bits are refused."""
    for name, cfg in CONFIGS.items():
        g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed, two_qubit=ISWAP)
        kcz = oracle.num_cut(cfg.n_qubits, grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed),
                             cfg.cut_mask())
        assert oracle.num_cut(cfg.n_qubits, g, cfg.cut_mask()) == 2 * kcz
        c = sf.create_circuit(cfg.rows, cfg.cols, g)
        if 2 * kcz <= 62:
            assert sf.set_cut(c, cfg.cut_mask()) == 2 * kcz, name
            plan = sf.describe_plan(c)
            if cfg.rows * cfg.cols == 30:       # three crossing iSWAPs in the last cycle: folded
                assert "1 levels, branch bits 6, 3 iSWAP gates; A: S 3 qubits, T 3; B: S 3 qubits, T 3" in plan
            else:                               # four or more: not folded
                assert "folded" not in plan, name
        else:
            with pytest.raises(sf.SFError) as e:
                sf.set_cut(c, cfg.cut_mask())
            assert e.value.code == sf.SF_ERR_UNSUPPORTED
        sf.destroy_circuit(c)
    bad = np.array([(ISWAP, 0, 0, 0, 5)], dtype=GATE_DTYPE)          # not neighbours on 2 x 4
    with pytest.raises(sf.SFError) as e:
        sf.create_circuit(2, 4, bad)
    assert e.value.code == sf.SF_ERR_INVALID


def test_set_cut_validation(sf):
    g = grid_circuit(4, 4, 8, 1)
    c = sf.create_circuit(4, 4, g)
    for mask, code in [(0b10, sf.SF_ERR_INVALID), ((1 << 16) - 1, sf.SF_ERR_INVALID),
                       (1 << 20 | 1, sf.SF_ERR_INVALID)]:
        with pytest.raises(sf.SFError) as e:
            sf.set_cut(c, mask)
        assert e.value.code == code
    sf.destroy_circuit(c)
    g = grid_circuit(8, 8, 8, 1)
    c = sf.create_circuit(8, 8, g)
    with pytest.raises(sf.SFError) as e:
        sf.set_cut(c, (1 << 40) - 1)     # block A of 40 qubits
    assert e.value.code == sf.SF_ERR_UNSUPPORTED
    sf.destroy_circuit(c)


def test_choose_cut_straight_line(sf):
    """Section 9: a single straight cut minimising the larger block, then crossing CZs."""
    expect = {(4, 4): ("col", 2), (5, 6): ("col", 3), (6, 7): ("row", 3), (7, 8): ("col", 4)}
    for (r, cc), (kind, nn) in expect.items():
        g = grid_circuit(r, cc, 16, 3)
        c = sf.create_circuit(r, cc, g)
        m = sf.choose_cut(c)
        n = r * cc
        assert bin(m).count("1") * 2 == n and m & 1
        from workload import column_cut_mask, row_cut_mask
        want = column_cut_mask(r, cc, nn) if kind == "col" else row_cut_mask(r, cc, nn)
        assert m == want, (r, cc)
        sf.destroy_circuit(c)


def test_num_paths_matches_paper_logs(sf):
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_numbers.json")))
    for e in gold["path_counts"]:
        f = e.get("f", None)
        if f is None:
            f = e["f_num"] / e["f_den"] if "f_den" in e else 2.0 ** e["f_pow2"]
        assert sf.num_paths(e["prefix_bits"], f) == e["count"], e["cite"]
    with pytest.raises(sf.SFError):
        sf.num_paths(10, 0.0)
    with pytest.raises(sf.SFError):
        sf.num_paths(10, 1.5)


@pytest.mark.parametrize("k,f,seed", [(8, 1.0, 3), (15, 0.1, 7), (28, 0.001, 3003), (35, 1e-7, 11),
                                      (20, 0.5, 0)])
def test_sample_paths_bit_exact_with_oracle(sf, k, f, seed):
    a = sf.sample_paths(k, f, seed)
    b = oracle.sample_paths(k, f, seed)
    assert a.size == math.ceil(f * 2 ** k)
    np.testing.assert_array_equal(a, b)


def test_workspace_size_and_run_validation(sf):
    w = make_workload("grid4x4_d16", n_bits=16)
    c = sf.create_circuit(4, 4, w["gates"])
    with pytest.raises(sf.SFError) as e:
        sf.run_paths(c, None, 0, 1, w["bitstrings"], 16, np.zeros(32))
    assert e.value.code == sf.SF_ERR_NO_CUT
    k = sf.set_cut(c, w["mask_a"])
    assert sf.workspace_size(c, 1 << k, 16) > 0
    amps = np.zeros(32)
    bad_bits = w["bitstrings"].copy()
    bad_bits[3] = 1 << 16
    with pytest.raises(sf.SFError) as e:
        sf.run_paths(c, None, 0, 1 << k, bad_bits, 16, amps)
    assert e.value.code == sf.SF_ERR_INVALID
    with pytest.raises(sf.SFError) as e:
        sf.run_paths(c, None, 0, (1 << k) + 1, w["bitstrings"], 16, amps)
    assert e.value.code == sf.SF_ERR_INVALID
    with pytest.raises(sf.SFError) as e:
        sf.run_paths(c, None, 0, 1, w["bitstrings"], 16, amps, flags=1 << 10)
    assert e.value.code == sf.SF_ERR_INVALID
    with pytest.raises(sf.SFError) as e:
        sf.run_paths(c, None, 0, 1, w["bitstrings"], 16, amps, workspace=12345, workspace_bytes=1 << 20)
    assert e.value.code == sf.SF_ERR_OOM
    sf.destroy_circuit(c)


def test_autotune_and_run_paths_reject_bad_arguments_before_device_work(sf):
    """autotune takes run_paths' argument rules (it ends in the same executor): NULL bitstrings
    or amplitudes, a workspace under 256 MiB and more than 2^31 - 1 bitstrings are refused, and
    so is SF_ACCUMULATE (autotune overwrites amps once per timed candidate).  Every case returns
    before any device call."""
    w = make_workload("grid4x4_d16", n_bits=16)
    c = sf.create_circuit(4, 4, w["gates"])
    sf.set_cut(c, w["mask_a"])
    bits, amps = w["bitstrings"], np.zeros(32)
    cases = [
        (dict(bitstrings=None, amps=amps), sf.SF_ERR_INVALID),
        (dict(bitstrings=bits, amps=None), sf.SF_ERR_INVALID),
        (dict(bitstrings=bits, amps=amps, flags=sf.SF_ACCUMULATE), sf.SF_ERR_INVALID),
        (dict(bitstrings=bits, amps=amps, flags=1 << 10), sf.SF_ERR_INVALID),
        (dict(bitstrings=bits, amps=amps, workspace=12345, workspace_bytes=1 << 20), sf.SF_ERR_OOM),
        (dict(bitstrings=bits, amps=amps, n_bits=2 ** 31), sf.SF_ERR_UNSUPPORTED),
    ]
    for kw, code in cases:
        kw = dict(kw)
        nb = kw.pop("n_bits", 16)
        with pytest.raises(sf.SFError) as e:
            sf.autotune(c, None, 0, 4, kw.pop("bitstrings"), nb, kw.pop("amps"), **kw)
        assert e.value.code == code, kw
    with pytest.raises(sf.SFError) as e:
        sf.run_paths(c, None, 0, 4, bits, 2 ** 31, amps)
    assert e.value.code == sf.SF_ERR_UNSUPPORTED
    assert sf.lib.autotune(c, None, 0, 4, bits.ctypes.data, 16, amps.ctypes.data, 0, None, None, 0, 2,
                           None) == sf.SF_ERR_INVALID      # best is NULL
    sf.destroy_circuit(c)
    # rejection_accept: more candidates than the device sort and select count in an int
    acc = np.zeros(4, dtype=np.uint32)
    ws = np.zeros(16, dtype=np.uint8)
    with pytest.raises(sf.SFError) as e:
        sf.rejection_accept(np.zeros(8), 2 ** 31, 20, 10.0, 1, acc, workspace=ws, workspace_bytes=ws.size)
    assert e.value.code == sf.SF_ERR_UNSUPPORTED


def test_dense_plan_uses_matrix_core_blocks(sf):
    """With dense_qubits set, the planner packs four-qubit windows into dense blocks."""
    w = make_workload("grid5x6_d24", n_bits=4)
    c = sf.create_circuit(5, 6, w["gates"])
    sf.set_cut(c, w["mask_a"])
    plain = sf.describe_plan(c)
    sf.set_tuning(c, dense_qubits=4)
    dense = sf.describe_plan(c)
    assert "dense" not in plain and "dense" in dense
    sf.destroy_circuit(c)


def test_leaf_fold_eligibility(sf):
    """Trailing tree levels are folded into the gather when every non-diagonal gate among them
    acts on one of their branch qubits (at most 5 path bits); otherwise, with at most 4 path
    bits, in the general form whose S' adds the branch qubits (used when it reads fewer bytes
    than writing the levels); fold_levels caps how many."""
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from fold_circuits import crossing_tail_circuit, two_level_tail_circuit
    general = {"grid4x4_d16": "2 levels, branch bits 4, general form; A: S' 7 qubits, T' 7; B: S' 7 qubits, T' 7",
               "grid6x7_d32": "1 levels, branch bits 3, general form; A: S' 6 qubits, T' 6; B: S' 3 qubits, T' 3",
               "grid7x8_d40": "1 levels, branch bits 4, general form; A: S' 8 qubits, T' 8; B: S' 5 qubits, T' 5"}
    expect = {**general, "grid5x6_d24": "2 levels, branch bits 5; A: S 5 qubits, T 5; B: S 5 qubits, T 5"}
    for name, fold in expect.items():
        cfg = CONFIGS[name]
        c = sf.create_circuit(cfg.rows, cfg.cols, grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed))
        sf.set_cut(c, cfg.cut_mask())
        plan = sf.describe_plan(c)
        assert fold in plan, plan
        if name in general:
            sf.set_tuning(c, no_leaf_fold=1)
            assert "folded" not in sf.describe_plan(c)
        else:
            assert fold in plan, plan
            sf.set_tuning(c, fold_levels=1)
            assert "1 levels, branch bits 3; A: S 3 qubits, T 3; B: S 3 qubits, T 3" in sf.describe_plan(c)
            # without the fold the leaf states are written: the workspace bound grows by them
            small = sf.workspace_size(c, 1 << 15, 100000)
            sf.set_tuning(c, no_leaf_fold=1)
            assert "folded" not in sf.describe_plan(c)
            assert sf.workspace_size(c, 1 << 15, 100000) - small >= 2 * (1 << 30) * 8
        sf.destroy_circuit(c)
    cases = [(crossing_tail_circuit(rows=3), "1 levels, branch bits 3; A: S 3 qubits, T 4; B: S 2 qubits, T 3"),
             (crossing_tail_circuit(rows=4), "1 levels, branch bits 4; A: S 3 qubits, T 4; B: S 2 qubits, T 3"),
             (two_level_tail_circuit(), "2 levels, branch bits 4; A: S 3 qubits, T 4; B: S 2 qubits, T 3")]
    for (r, cc, g, m), want in cases:
        c = sf.create_circuit(r, cc, g)
        sf.set_cut(c, m)
        assert want in sf.describe_plan(c)
        sf.destroy_circuit(c)
    # crossing iSWAPs: projector + per-path flip; a qubit without a later gate stays outside S
    from fold_circuits import iswap_tail_circuit
    for drop, want in [((), "2 levels, branch bits 4, 2 iSWAP gates; A: S 2 qubits, T 2; B: S 2 qubits, T 2"),
                       ((5, 2), "2 levels, branch bits 4, 2 iSWAP gates; A: S 1 qubits, T 1; B: S 1 qubits, T 1")]:
        r, cc, g, m = iswap_tail_circuit(drop)
        c = sf.create_circuit(r, cc, g)
        sf.set_cut(c, m)
        assert want in sf.describe_plan(c)
        sf.destroy_circuit(c)
    # a non-diagonal gate on a non-branch qubit in the last level: only the general form
    r, cc, g, m = crossing_tail_circuit(rows=3)
    extra = np.array([(H, 0, int(g["cycle"].max()) + 1, 0, 0)], dtype=GATE_DTYPE)   # H on (0,0) after its CZ
    c = sf.create_circuit(r, cc, np.concatenate([g, extra]))
    sf.set_cut(c, m)
    plan = sf.describe_plan(c)
    assert "general form" in plan and "A: S' 4 qubits" in plan, plan
    sf.destroy_circuit(c)


def test_tuning_roundtrip(sf):
    w = make_workload("grid4x4_d16", n_bits=4)
    c = sf.create_circuit(4, 4, w["gates"])
    sf.set_tuning(c, reg_qubits=3, leaf_batch=64, max_slots=1024, waves_per_cu=16, dense_qubits=4, no_leaf_fold=1,
                  fold_levels=2, chain_passes=1, no_row_skip=1, no_defer=1, no_chain_merge=1, jit=1, no_tail_move=1)
    assert sf.get_tuning(c) == {"reg_qubits": 3, "leaf_batch": 64, "max_slots": 1024, "waves_per_cu": 16,
                                "dense_qubits": 4, "no_leaf_fold": 1, "fold_levels": 2, "chain_passes": 1,
                                "no_row_skip": 1, "no_defer": 1, "no_chain_merge": 1, "jit": 1, "no_tail_move": 1}
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, no_leaf_fold=2)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, chain_passes=2)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, no_row_skip=2)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, no_defer=2)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, no_chain_merge=2)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, jit=2)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, no_tail_move=2)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, dense_qubits=1)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, leaf_batch=48)
    with pytest.raises(sf.SFError):
        sf.set_tuning(c, reg_qubits=9)
    sf.destroy_circuit(c)


def test_rejection_host_entries_match_oracle(sf):
    """Step 1 and step 2 of the rejection-sampling algorithms run on the host: M and M' as the
    oracle (and the paper's printed 41 and 10), candidates bit for bit."""
    assert sf.rejection_m(49, 1e-3, sf.SF_SAMPLE_BASIC) == oracle.rejection_m(49, 1e-3, basic=True) == 41
    for eps in (1e-2, 5e-4, 1e-6):
        assert sf.rejection_m(30, eps) == oracle.rejection_m(30, eps)
    for n, count, seed in ((30, 100000, 2002), (16, 65536, 3), (64, 5000, 9), (1, 2, 4)):
        np.testing.assert_array_equal(sf.sample_bitstrings(n, count, seed), oracle.sample_bitstrings(n, count, seed))
    for args in ((0, 1e-3, 0), (65, 1e-3, 0), (20, 0.0, 0), (20, 1.0, 0), (20, 1e-3, 1)):
        with pytest.raises(sf.SFError) as e:
            sf.rejection_m(*args)
        assert e.value.code == sf.SF_ERR_INVALID
    with pytest.raises(sf.SFError):
        sf.sample_bitstrings(4, 17, 1)


def test_tuning_cache_file_roundtrip(sf, tmp_path):
    """Autotuner results kept across processes: a text file of keyed tunings, validated on load
    (entries without the last fields, chain_passes, no_row_skip, no_defer, no_chain_merge, jit and
    no_tail_move, read as 0)."""
    src = tmp_path / "in.txt"
    src.write_text("# comment\n"
                   "gfx950:256/15/15/15/7/32768/100000/0 5 0 0 32 4 0 2\n"
                   "gfx950:256/15/15/30/7/262144/100000/0 4 4096 0 16 0 1 0 1 1\n"
                   "gfx950:256/15/15/28/7/1024/1000000/0 5 0 0 128 0 0 0 0 0 0 1\n"
                   "gfx950:256/15/15/28/7/2048/1000000/0 5 0 0 128 0 0 0 0 0 0 0 1\n")
    assert sf.load_tuning_cache(str(src)) == 4
    out = tmp_path / "out.txt"
    sf.save_tuning_cache(str(out))
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert "gfx950:256/15/15/15/7/32768/100000/0 5 0 0 32 4 0 2 0 0 0 0 0 0" in lines
    assert "gfx950:256/15/15/30/7/262144/100000/0 4 4096 0 16 0 1 0 1 1 0 0 0 0" in lines
    assert "gfx950:256/15/15/28/7/1024/1000000/0 5 0 0 128 0 0 0 0 0 0 1 0 0" in lines
    assert "gfx950:256/15/15/28/7/2048/1000000/0 5 0 0 128 0 0 0 0 0 0 0 1 0" in lines
    for bad in ["k 1 2 3\n", "k 9 0 0 32 0 0 0\n", "k 5 0 0 32 1 0 0\n", "k 5 0 0 32 0 0 0 7\n",
                "k 5 0 0 32 0 0 0 0 0 0 0 0 0 0\n", "k 5 0 0 32 0 0 0 0 2\n", "k 5 0 0 32 0 0 0 0 0 3\n",
                "k 5 0 0 32 0 0 0 0 0 0 2\n", "k 5 0 0 32 0 0 0 0 0 0 0 2\n",
                "k 5 0 0 32 0 0 0 0 0 0 0 0 2\n"]:
        f = tmp_path / "bad.txt"
        f.write_text(bad)
        with pytest.raises(sf.SFError) as e:
            sf.load_tuning_cache(str(f))
        assert e.value.code == sf.SF_ERR_INVALID
    with pytest.raises(sf.SFError):
        sf.load_tuning_cache(str(tmp_path / "missing.txt"))
    with pytest.raises(sf.SFError):
        sf.save_tuning_cache(str(tmp_path / "no_such_dir" / "x.txt"))


def _plan_parts(plan):
    """(level, block A part, block B part) of each describe_plan level line."""
    out = []
    for line in plan.splitlines():
        m = re.match(r"level (\d+) .*?: A (.*?)  B (.*)$", line)
        if m:
            out.append((int(m.group(1)), m.group(2), m.group(3)))
    return out


def test_zero_subspace_marked_in_plan(sf):
    """Section 2 zero blocks: after a crossing CZ's projector on a block-A qubit, and until the
    next non-diagonal gate on that qubit, half of block A's amplitudes are zero; block B gets no
    projector (its branch operator is Z), so it never has such zeros (the paper's zero counts
    are on A only).  The planner marks passes whose source has them with /z<qubits>."""
    from workload.generator import T
    # 2x2 grid, qubits 0 1 / 2 3, A = column 0 = {0, 2}; the second crossing CZ is on qubit 0
    # again, so the final H on qubit 0 cannot move up to level 1
    def circ(mix_between):
        g = [(H, 0, 0, q, 0) for q in range(4)]
        g.append((CZ, 0, 1, 0, 1))                       # crossing: level 1, projector on qubit 0
        g.append((T, 0, 2, 0, 0))                        # diagonal: keeps the zeros
        g.append((H, 0, 2, 2, 0))                        # other qubit: keeps the zeros
        if mix_between:
            g.append((H, 0, 3, 0, 0))                    # non-diagonal on qubit 0: mixes them
        g.append((CZ, 0, 4, 0, 1))                       # crossing: level 2
        g.append((H, 0, 5, 0, 0))
        g.append((H, 0, 5, 2, 0))
        return np.array(g, dtype=GATE_DTYPE)
    for mix, want in ((False, True), (True, False)):
        c = sf.create_circuit(2, 2, circ(mix))
        sf.set_cut(c, 0b0101)
        sf.set_tuning(c, no_leaf_fold=1)
        parts = _plan_parts(sf.describe_plan(c))
        lvl2 = [p for p in parts if p[0] == 2]
        assert lvl2, parts
        assert ("/z1" in lvl2[0][1]) == want, (mix, parts)
        assert all("/z" not in b for _, _, b in parts), parts
        sf.destroy_circuit(c)
    # the benchmark circuit: block A's fan-outs into levels 3 and 4 read a half-zero state
    cfg = CONFIGS["grid5x6_d24"]
    c = sf.create_circuit(cfg.rows, cfg.cols, grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed))
    sf.set_cut(c, cfg.cut_mask())
    parts = _plan_parts(sf.describe_plan(c))
    assert all("/z" not in b for _, _, b in parts), parts
    assert any("/z" in a for _, a, _ in parts), parts
    sf.destroy_circuit(c)


def test_read_bandwidth_rejects_bad_arguments(sf):
    """Argument checks come before any device work (no GPU needed)."""
    fake = 1 << 40        # never dereferenced: every call below fails its checks first
    for args in ((None, 1 << 20, 1, 0), (fake, 1024, 1, 0), (fake, (1 << 20) + 16, 1, 0), (fake, 1 << 20, 0, 0),
                 (fake, 1 << 20, 100001, 0)):
        with pytest.raises(sf.SFError) as e:
            sf.read_bandwidth(*args)
        assert e.value.code == sf.SF_ERR_INVALID


@pytest.mark.parametrize("circuit,tune", [("cz", {}), ("iswap", {}), ("cz_fp64", {"fp64": True})])
def test_compiled_pass_kernels_build_on_host(sf, circuit, tune):
    """The kernels tuning jit compiles per pass program (one-qubit gates, diagonal groups with
    their constant register weights, per-path flips and in-block iSWAPs for crossing iSWAPs)
    compile for gfx950 on the host: every non-dense pass of every level of both blocks."""
    from workload import ISWAP, grid_circuit
    g = grid_circuit(4, 5, 12, 7, two_qubit=ISWAP) if circuit == "iswap" else grid_circuit(4, 5, 12, 7)
    c = sf.create_circuit(4, 5, g)
    sf.set_cut(c, sf.choose_cut(c))
    levels = [int(l.split()[1]) for l in sf.describe_plan(c).splitlines() if l.startswith("level ")]
    R = 4 if tune.get("fp64") else 5
    total = 0
    for half in (0, 1):
        # the root with the levels below it as one segment, then the last levels one by one
        n, nb = sf.compile_segment_kernels(c, half, 0, 1, 0, R, **tune)
        total += n
        assert n >= 1 and nb > 0
        for lv in levels[2:]:
            n, nb = sf.compile_segment_kernels(c, half, lv, lv, min(lv * 2, 8), R, **tune)
            total += n
    assert total >= 4
    with pytest.raises(sf.SFError):
        sf.compile_segment_kernels(c, 2, 0, 0, 0, R)
    with pytest.raises(sf.SFError):
        sf.compile_segment_kernels(c, 0, 1, 0, 0, R)
    with pytest.raises(sf.SFError):
        sf.compile_segment_kernels(c, 0, 0, 0, 0, 6)
    sf.destroy_circuit(c)
