"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerance (floating point): the relative error in |amp|^2 of parity_tol,
at most 1e-5 for complex64 sweeps and 1e-10 for complex128 sweeps.  Path and
bitstring indexing is exact: single-path runs expose any permutation as an
O(1) error.
"""
import numpy as np
import pytest

import oracle
from parity_tol import TOL_C128, TOL_C64, c11_error
from workload import CONFIGS, grid_circuit, make_workload, random_bitstrings, workload_block

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


def _circuit(sf, name):
    cfg = CONFIGS[name]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    return cfg, g, sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())


# ---------------------------------------------------------------- 4x4, 1+16+1, 8+8

@pytest.mark.parametrize("fp64", [True, False])
def test_grid4x4_all_paths(sf, fp64):
    cfg, g, c = _circuit(sf, "grid4x4_d16")
    bits = random_bitstrings(16, cfg.n_bits, cfg.bits_seed)
    say(f"grid4x4_d16 all paths fp64={fp64}")
    a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS if fp64 else 0)
    o = oracle.path_sum(16, g, cfg.cut_mask(), np.arange(1 << c.k, dtype=np.uint64), bits)
    full = oracle.full_state(16, g)[bits.astype(np.int64)]
    err = c11_error(a, o, 1 << c.k, c.k, 16)
    assert err <= (TOL_C128 if fp64 else TOL_C64), err
    assert np.abs(o - full).max() < 1e-14


@pytest.mark.parametrize("path", [0, 1, 37, 128, 200, 255])
def test_grid4x4_single_path_indexing(sf, path):
    cfg, g, c = _circuit(sf, "grid4x4_d16")
    bits = random_bitstrings(16, 1024, 5)
    say(f"grid4x4_d16 single path {path}")
    a = c.amplitudes(bits, path_begin=path, n_paths=1, flags=sf.SF_FP64_SWEEPS)
    o = oracle.path_sum(16, g, cfg.cut_mask(), [path], bits)
    assert c11_error(a, o, 1, c.k, 16) <= TOL_C128


def test_grid4x4_plain_equals_batched(sf):
    cfg, g, c = _circuit(sf, "grid4x4_d16")
    bits = random_bitstrings(16, 512, 6)
    ids = np.array([3, 4, 5, 17, 100, 101, 250], dtype=np.uint64)
    say("grid4x4_d16 plain vs batched")
    a = c.amplitudes(bits, path_ids=ids, flags=sf.SF_PLAIN)
    b = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(16, g, cfg.cut_mask(), ids, bits)
    assert c11_error(a, o, ids.size, c.k, 16) <= TOL_C64
    assert c11_error(b, o, ids.size, c.k, 16) <= TOL_C64


def test_empty_and_accumulate(sf):
    import torch
    cfg, g, c = _circuit(sf, "grid4x4_d16")
    bits = random_bitstrings(16, 100, 7)
    say("grid4x4_d16 zero paths / accumulate / device buffers")
    z = c.amplitudes(bits, path_ids=np.zeros(0, dtype=np.uint64))
    assert np.all(z == 0)
    # two halves of the path space accumulated into one device buffer equal the whole
    dbits = torch.from_numpy(bits.view(np.int64)).cuda()
    acc = torch.zeros(2 * bits.size, dtype=torch.float64, device="cuda")
    ws = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    flags = sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE
    sf.run_paths(c.handle, None, 0, 128, dbits, bits.size, acc, flags, torch.cuda.current_stream(), ws, ws.numel())
    sf.run_paths(c.handle, None, 128, 128, dbits, bits.size, acc, flags | sf.SF_ACCUMULATE,
                 torch.cuda.current_stream(), ws, ws.numel())
    a = acc.cpu().numpy().view(np.complex128)
    o = oracle.path_sum(16, g, cfg.cut_mask(), np.arange(256, dtype=np.uint64), bits)
    assert c11_error(a, o, 256, c.k, 16) <= TOL_C64
    # a device bitstring outside the grid is reported after the run
    bad = dbits.clone()
    bad[5] = 1 << 20
    with pytest.raises(sf.SFError):
        sf.run_paths(c.handle, None, 0, 4, bad, bits.size, acc, flags, None, ws, ws.numel())


def test_small_blocks_and_no_crossing(sf):
    """Blocks below 6 qubits (padded slots) and a circuit without crossing CZs (k = 0)."""
    g = grid_circuit(2, 4, 10, 44)
    mask = 0b00110011                    # columns 0-1: 4 + 4 qubits
    c = sf.Circuit(2, 4, g, mask)
    bits = np.arange(256, dtype=np.uint64)
    say("2x4 grid, 4+4 blocks")
    a = c.amplitudes(bits)
    o = oracle.full_state(8, g)
    assert c11_error(a, o, 1, 0, 8) <= TOL_C64
    g0 = grid_circuit(4, 4, 1, 3)
    c0 = sf.Circuit(4, 4, g0, (1 << 8) - 1)   # rows 0-1 | rows 2-3, cycle 1 is V(0,0): no crossing
    assert c0.k == 0
    bits = random_bitstrings(16, 300, 4)
    say("4x4 depth 1, k = 0")
    a = c0.amplitudes(bits)
    o = oracle.full_state(16, g0)[bits.astype(np.int64)]
    assert c11_error(a, o, 1, 0, 16) <= TOL_C64


def test_register_widths_agree(sf):
    cfg, g, c = _circuit(sf, "grid4x4_d16")
    bits = random_bitstrings(16, 256, 8)
    o = oracle.path_sum(16, g, cfg.cut_mask(), np.arange(256, dtype=np.uint64), bits)
    for r in (1, 2, 3, 4, 5):
        say(f"grid4x4_d16 reg_qubits={r}")
        c.tune(reg_qubits=r)
        a = c.amplitudes(bits)
        assert c11_error(a, o, 256, c.k, 16) <= TOL_C64, r


# ---------------------------------------------------------------- 5x6, 1+24+1, 15+15

@pytest.mark.parametrize("no_fold", [0, 1])
def test_grid5x6_path_subsets(sf, no_fold):
    cfg, g, c = _circuit(sf, "grid5x6_d24")
    c.tune(no_leaf_fold=no_fold)
    say(f"grid5x6_d24 no_leaf_fold={no_fold}")
    bits = random_bitstrings(30, 4000, cfg.bits_seed)
    rng = np.random.default_rng(1)
    ids = np.sort(rng.choice(1 << c.k, size=200, replace=False)).astype(np.uint64)
    say("grid5x6_d24 200 random paths")
    a = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(30, g, cfg.cut_mask(), ids, bits)
    assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64
    say("grid5x6_d24 aligned block of 512 paths, tight workspace")
    import torch
    ws = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    a = c.amplitudes(bits, path_begin=3 * 512, n_paths=512, workspace=ws)
    o = oracle.path_sum(30, g, cfg.cut_mask(), np.arange(3 * 512, 4 * 512, dtype=np.uint64), bits)
    assert c11_error(a, o, 512, c.k, 30) <= TOL_C64


@pytest.mark.parametrize("no_fold", [0, 1])
def test_grid5x6_partial_fanouts(sf, no_fold):
    """A dense random subset (about 60% of an aligned block of 2048 paths): the deepest fan-outs
    keep about 60% of their children, so they are neither full (branch-major slots) nor sparse,
    and take parent-major child slots; with no_leaf_fold the last level is such a fan-out too."""
    cfg, g, c = _circuit(sf, "grid5x6_d24")
    c.tune(no_leaf_fold=no_fold)
    rng = np.random.default_rng(23)
    block = np.arange(13 * 2048, 14 * 2048, dtype=np.uint64)
    ids = np.sort(block[rng.random(block.size) < 0.6])
    bits = random_bitstrings(30, 600, cfg.bits_seed + 9)
    say(f"grid5x6_d24 no_leaf_fold={no_fold}: {ids.size} paths of an aligned block of 2048")
    a = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(30, g, cfg.cut_mask(), ids, bits)
    assert c11_error(a, o, ids.size, c.k, 30) <= TOL_C64


@pytest.mark.slow
def test_grid5x6_full_benchmark_size(sf):
    """All 2^15 paths, 1e5 bitstrings, default launch configuration (the benchmark's)."""
    w = make_workload("grid5x6_d24")
    cfg, g, c = _circuit(sf, "grid5x6_d24")
    say("grid5x6_d24 all paths, 1e5 bitstrings")
    a = c.amplitudes(w["bitstrings"])
    o = oracle.path_sum(30, g, cfg.cut_mask(), np.arange(1 << c.k, dtype=np.uint64), w["bitstrings"])
    assert c11_error(a, o, 1 << c.k, c.k, 30) <= TOL_C64


# ---------------------------------------------------------------- 6x7 and 7x8

def test_grid6x7_sampled_paths(sf):
    cfg, g, c = _circuit(sf, "grid6x7_d32")
    ids_all = sf.sample_paths(c.k, cfg.f, cfg.path_seed)
    assert ids_all.size == 2684355
    # four ids spread over the sample, each the first live one at or after its position (the
    # others have zero terms, which the library skips)
    from workload import equal_bit_pairs, is_live
    pairs = equal_bit_pairs(g, cfg.cut_mask())
    ids = []
    for start in range(0, ids_all.size, ids_all.size // 4):
        i = start
        while not is_live(int(ids_all[i]), pairs):
            i += 1
        ids.append(ids_all[i])
    ids = np.array(ids[:4], dtype=np.uint64)
    bits = random_bitstrings(42, 20000, cfg.bits_seed)
    say(f"grid6x7_d32 sampled paths {ids.tolist()}")
    a = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(42, g, cfg.cut_mask(), ids, bits)
    assert c11_error(a, o, ids.size, c.k, 42) <= TOL_C64
    for p in ids[:2]:
        say(f"grid6x7_d32 single path {int(p)}")
        a1 = c.amplitudes(bits[:2000], path_ids=[p])
        o1 = oracle.path_sum(42, g, cfg.cut_mask(), [p], bits[:2000])
        assert c11_error(a1, o1, 1, c.k, 42) <= TOL_C64


def test_grid7x8_block_properties(sf):
    """Full 28+28 shape: a path block equals the sum of its parts, the plain form, and each
    single-path term is rank one in (x_A, x_B)."""
    cfg, g, c = _circuit(sf, "grid7x8_d40")
    begin, count = workload_block("grid7x8_d40")
    bits = random_bitstrings(56, 4096, cfg.bits_seed)
    say("grid7x8_d40 16-path sub-block, tree")
    a = c.amplitudes(bits, path_begin=begin, n_paths=16)
    say("grid7x8_d40 two 8-path halves")
    a1 = c.amplitudes(bits, path_begin=begin, n_paths=8)
    a2 = c.amplitudes(bits, path_begin=begin + 8, n_paths=8)
    assert np.abs(a - (a1 + a2)).max() <= 1e-5 * np.abs(a).max()
    say("grid7x8_d40 plain form, 2 paths")
    p = c.amplitudes(bits, path_begin=begin, n_paths=2, flags=sf.SF_PLAIN)
    t = c.amplitudes(bits, path_begin=begin, n_paths=2)
    assert np.abs(p - t).max() <= 1e-5 * np.abs(t).max()
    # rank one: amp(a1,b1) amp(a2,b2) = amp(a1,b2) amp(a2,b1) for one path
    ma, mb = c.mask_a, ((1 << 56) - 1) & ~c.mask_a
    rng = np.random.default_rng(3)
    xa = [int(v) & ma for v in rng.integers(0, 1 << 62, 2, dtype=np.int64)]
    xb = [int(v) & mb for v in rng.integers(0, 1 << 62, 2, dtype=np.int64)]
    quad = np.array([xa[0] | xb[0], xa[1] | xb[1], xa[0] | xb[1], xa[1] | xb[0]], dtype=np.uint64)
    say("grid7x8_d40 rank-one check of a single path")
    q = c.amplitudes(quad, path_begin=begin + 5, n_paths=1)
    assert abs(q[0] * q[1] - q[2] * q[3]) <= 1e-4 * abs(q[0] * q[1])


# ---------------------------------------------------------------- dense blocks on matrix cores

@pytest.mark.parametrize("name,npaths", [("grid5x6_d24", 300), ("grid6x7_d32", 3)])
def test_dense_blocks_parity(sf, name, npaths):
    """Four-qubit windows applied as dense 16 x 16 blocks with MFMA give the oracle's result."""
    cfg, g, c = _circuit(sf, name)
    c.tune(dense_qubits=4)
    assert "dense" in sf.describe_plan(c.handle)
    rng = np.random.default_rng(11)
    ids = np.sort(rng.choice(1 << min(c.k, 40), size=npaths, replace=False)).astype(np.uint64)
    bits = random_bitstrings(cfg.n_qubits, 3000, 12)
    say(f"{name} dense blocks, {npaths} paths")
    a = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(cfg.n_qubits, g, cfg.cut_mask(), ids, bits)
    assert c11_error(a, o, ids.size, c.k, cfg.n_qubits) <= TOL_C64


# ---------------------------------------------------------------- trailing levels folded into the gather

def _hand_built(sf, which):
    import sys, os
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from fold_circuits import crossing_tail_circuit, two_level_tail_circuit
    r, cc, g, m = two_level_tail_circuit() if which == "two" else crossing_tail_circuit(rows=which)
    return r * cc, g, m, sf.Circuit(r, cc, g, m)


@pytest.mark.parametrize("which", [3, 4, "two"])
def test_leaf_fold_tail_circuits(sf, which):
    """Folded levels with 3 and 4 branch bits (one level) and 4 bits over two levels, phases
    after the branch gates, and branch qubits that only diagonal gates touch: every fold depth
    and the materialised leaves give the oracle's result."""
    n, g, m, c = _hand_built(sf, which)
    assert "folded" in sf.describe_plan(c.handle)
    bits = random_bitstrings(n, 3000, 21 + (which if which != "two" else 9))
    ids = np.arange(1 << c.k, dtype=np.uint64)
    o = oracle.path_sum(n, g, m, ids, bits)
    assert np.abs(o - oracle.full_state(n, g)[bits.astype(np.int64)]).max() < 1e-13
    for tune in ({"no_leaf_fold": 0}, {"fold_levels": 1}, {"no_leaf_fold": 1}):
        c.tune(**tune)
        say(f"hand-built circuit {which} all paths {tune}")
        a = c.amplitudes(bits)
        assert c11_error(a, o, ids.size, c.k, n) <= TOL_C64, tune
        say(f"hand-built circuit {which} all paths complex128 {tune}")
        a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS)
        assert c11_error(a, o, ids.size, c.k, n) <= TOL_C128, tune
    c.tune(no_leaf_fold=0)
    # sampled paths: parents with some of their descendants only
    sub = sf.sample_paths(c.k, 0.3, 77)
    say(f"hand-built circuit {which} {sub.size} sampled paths")
    a = c.amplitudes(bits, path_ids=sub)
    o = oracle.path_sum(n, g, m, sub, bits)
    assert c11_error(a, o, sub.size, c.k, n) <= TOL_C64
    # one path at a time (plain form) and single-path indexing
    ids3 = np.array([1, (1 << c.k) - 2, (1 << c.k) // 3 + 1], dtype=np.uint64)
    say(f"hand-built circuit {which} plain form {ids3.tolist()}")
    a = c.amplitudes(bits, path_ids=ids3, flags=sf.SF_PLAIN)
    o = oracle.path_sum(n, g, m, ids3, bits)
    assert c11_error(a, o, ids3.size, c.k, n) <= TOL_C64
    for p in ids3:
        a = c.amplitudes(bits[:500], path_ids=[p], flags=sf.SF_FP64_SWEEPS)
        o = oracle.path_sum(n, g, m, [p], bits[:500])
        assert c11_error(a, o, 1, c.k, n) <= TOL_C128, int(p)


@pytest.mark.parametrize("shape", [(2, 3, 3, 0), (2, 3, 5, 0), (2, 3, 21, 0), (4, 5, 7, 0), (4, 5, 15, 0)])
def test_leaf_fold_grid_circuits(sf, shape):
    """Grid circuits whose trailing levels qualify (one or two levels, 2 to 5 path bits), from
    one slot per batch (fewer slots than lanes) to 2^5; every bitstring of the smaller ones."""
    rows, cols, depth, seed = shape
    n = rows * cols
    g = grid_circuit(rows, cols, depth, seed)
    h = sf.create_circuit(rows, cols, g)
    m = sf.choose_cut(h)
    sf.destroy_circuit(h)
    c = sf.Circuit(rows, cols, g, m)
    assert "folded" in sf.describe_plan(c.handle)
    bits = np.arange(1 << n, dtype=np.uint64) if n <= 12 else random_bitstrings(n, 5000, 31)
    o = oracle.full_state(n, g)[bits.astype(np.int64)]
    for tune in ({"fold_levels": 0}, {"fold_levels": 1}):
        c.tune(**tune)
        say(f"grid {rows}x{cols} depth {depth} seed {seed} {tune}, {bits.size} bitstrings")
        a = c.amplitudes(bits)
        assert c11_error(a, o, 1, 0, n) <= TOL_C64, tune
        a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS)
        assert c11_error(a, o, 1, 0, n) <= TOL_C128, tune


def test_grid5x6_fold_depths_tight_workspace(sf):
    """The benchmark circuit with two and one folded levels and with materialised leaves: an
    aligned block of 4096 paths against the oracle, and all 2^15 paths in a 256 MiB workspace
    (several batches of the level the gather reads) against each other."""
    import torch
    cfg, g, c = _circuit(sf, "grid5x6_d24")
    bits = random_bitstrings(30, 2000, cfg.bits_seed)
    o = oracle.path_sum(30, g, cfg.cut_mask(), np.arange(8192, 8192 + 4096, dtype=np.uint64), bits)
    ws = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    full = {}
    for tune in ({"fold_levels": 2}, {"fold_levels": 1}, {"no_leaf_fold": 1}):
        c.tune(**tune)
        say(f"grid5x6_d24 {tune} 4096 paths")
        a = c.amplitudes(bits, path_begin=8192, n_paths=4096)
        assert c11_error(a, o, 4096, c.k, 30) <= TOL_C64, tune
        say(f"grid5x6_d24 {tune} 4096 paths, 256 MiB workspace")
        a = c.amplitudes(bits, path_begin=8192, n_paths=4096, workspace=ws)
        assert c11_error(a, o, 4096, c.k, 30) <= TOL_C64, tune
        say(f"grid5x6_d24 {tune} all paths, 256 MiB workspace")
        full[str(tune)] = c.amplitudes(bits, workspace=ws)
    ref = full[str({"no_leaf_fold": 1})]
    for k, a in full.items():
        assert c11_error(a, ref, 1 << c.k, c.k, 30) <= 2 * TOL_C64, k


def test_fold_empty_accumulate_device_buffers(sf):
    """Folded gather with device buffers and a caller's workspace (bitstring preprocessing is
    enqueued before planning): zero paths, two path blocks accumulated, a bad device bitstring,
    and a duplicated bitstring."""
    import torch
    cfg, g, c = _circuit(sf, "grid5x6_d24")
    assert "folded" in sf.describe_plan(c.handle)
    bits = random_bitstrings(30, 300, 17)
    bits = np.concatenate([bits, bits[:3]])               # repeated bitstrings get the same amplitude
    dbits = torch.from_numpy(bits.view(np.int64)).cuda()
    acc = torch.full((2 * bits.size,), 7.0, dtype=torch.float64, device="cuda")
    ws = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    flags = sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE
    stream = torch.cuda.current_stream()
    say("grid5x6_d24 folded: zero paths")
    sf.run_paths(c.handle, np.zeros(0, dtype=np.uint64), 0, 0, dbits, bits.size, acc, flags, stream, ws, ws.numel())
    assert torch.all(acc == 0)
    say("grid5x6_d24 folded: two blocks of 256 paths accumulated")
    sf.run_paths(c.handle, None, 1024, 256, dbits, bits.size, acc, flags, stream, ws, ws.numel())
    sf.run_paths(c.handle, None, 1280, 256, dbits, bits.size, acc, flags | sf.SF_ACCUMULATE, stream, ws, ws.numel())
    a = acc.cpu().numpy().view(np.complex128)
    o = oracle.path_sum(30, g, cfg.cut_mask(), np.arange(1024, 1536, dtype=np.uint64), bits)
    assert c11_error(a, o, 512, c.k, 30) <= TOL_C64
    assert np.array_equal(a[-3:], a[:3])
    say("grid5x6_d24 folded: bad device bitstring")
    bad = dbits.clone()
    bad[5] = 1 << 40
    with pytest.raises(sf.SFError):
        sf.run_paths(c.handle, None, 0, 64, bad, bits.size, acc, flags, stream, ws, ws.numel())
    # the library still works afterwards on the same workspace
    sf.run_paths(c.handle, None, 1024, 512, dbits, bits.size, acc, flags, stream, ws, ws.numel())
    a = acc.cpu().numpy().view(np.complex128)
    assert c11_error(a, o, 512, c.k, 30) <= TOL_C64


def test_repeated_request_reuses_plan(sf):
    """A call identical to the previous one reuses its plan: results are unchanged, ACCUMULATE
    still adds, and a different path list, bitstring count or tuning is planned afresh."""
    import torch
    cfg, g, c = _circuit(sf, "grid5x6_d24")
    bits = random_bitstrings(30, 500, 23)
    dbits = torch.from_numpy(bits.view(np.int64)).cuda()
    acc = torch.zeros(2 * bits.size, dtype=torch.float64, device="cuda")
    ws = torch.empty(1 << 29, dtype=torch.uint8, device="cuda")
    flags = sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE
    stream = torch.cuda.current_stream()
    ids = np.sort(np.random.default_rng(4).choice(1 << c.k, 700, replace=False)).astype(np.uint64)
    o = oracle.path_sum(30, g, cfg.cut_mask(), ids, bits)
    runs = []
    for rep in range(3):
        say(f"grid5x6_d24 repeated request {rep}")
        sf.run_paths(c.handle, ids, 0, ids.size, dbits, bits.size, acc, flags, stream, ws, ws.numel())
        runs.append(acc.cpu().numpy().view(np.complex128).copy())
    assert c11_error(runs[0], o, ids.size, c.k, 30) <= TOL_C64
    assert np.array_equal(runs[0], runs[1]) and np.array_equal(runs[0], runs[2])
    sf.run_paths(c.handle, ids, 0, ids.size, dbits, bits.size, acc, flags | sf.SF_ACCUMULATE, stream, ws, ws.numel())
    assert np.allclose(acc.cpu().numpy().view(np.complex128), 2 * runs[0], rtol=1e-12, atol=0)
    ids2 = ids[::2].copy()
    say("grid5x6_d24 other path list after a repeated request")
    sf.run_paths(c.handle, ids2, 0, ids2.size, dbits, bits.size, acc, flags, stream, ws, ws.numel())
    o2 = oracle.path_sum(30, g, cfg.cut_mask(), ids2, bits)
    assert c11_error(acc.cpu().numpy().view(np.complex128), o2, ids2.size, c.k, 30) <= TOL_C64
    say("grid5x6_d24 fewer bitstrings, other tuning")
    c.tune(fold_levels=1)
    sf.run_paths(c.handle, ids2, 0, ids2.size, dbits, 200, acc, flags, stream, ws, ws.numel())
    assert c11_error(acc.cpu().numpy().view(np.complex128)[:200], o2[:200], ids2.size, c.k, 30) <= TOL_C64


@pytest.mark.parametrize("fp64", [True, False])
def test_diagonal_group_quarter_turn_phases(sf, fp64):
    """Two T gates on a qubit with only diagonal gates between them give the phase i (weight 2
    of 8), which a merged diagonal group must not take for a sign."""
    from workload import GATE_DTYPE, H, T, CZ
    g = [(H, 0, 0, q, 0) for q in range(16)]
    for cyc in (1, 2):
        g += [(T, 0, cyc, q, 0) for q in range(0, 16, 3)]        # S = T^2 on every third qubit
    g += [(CZ, 0, 3, 1, 2), (CZ, 0, 3, 5, 6), (CZ, 0, 3, 8, 12)]
    g += [(H, 0, 4, q, 0) for q in range(16)]
    g = np.array(g, dtype=GATE_DTYPE)
    mask = CONFIGS["grid4x4_d16"].cut_mask()
    c = sf.Circuit(4, 4, g, mask)
    bits = np.arange(1 << 16, dtype=np.uint64)[::13]
    say(f"T^2 / T^3 phases fp64={fp64} k={c.k}")
    a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS if fp64 else 0)
    o = oracle.full_state(16, g)[bits.astype(np.int64)]
    assert c11_error(a, o, 1, 0, 16) <= (TOL_C128 if fp64 else TOL_C64)


@pytest.mark.parametrize("two_qubit,fp64", [(4, True), (4, False), (5, True), (5, False)])
def test_full_output_norm(sf, two_qubit, fp64):
    """All 2^16 amplitudes over all paths form the unit-norm output state (a property that holds
    at any size; here with FP64 sums over 256 or 4096 paths)."""
    from workload import ISWAP
    depth = 16 if two_qubit == 4 else 12
    g = grid_circuit(4, 4, depth, 5, two_qubit=two_qubit)
    c = sf.Circuit(4, 4, g, CONFIGS["grid4x4_d16"].cut_mask())
    bits = np.arange(1 << 16, dtype=np.uint64)
    say(f"full output norm, {'iSWAP' if two_qubit == ISWAP else 'CZ'} 4x4, k={c.k}, fp64={fp64}")
    a = c.amplitudes(bits, flags=sf.SF_FP64_SWEEPS if fp64 else 0)
    norm = float(np.sum(np.abs(a) ** 2))
    assert abs(norm - 1.0) <= (1e-12 if fp64 else 1e-5), norm
