"""GPU parity at the benchmark's shapes and launch configurations.

* 7x8 grid, depth 1+40+1, 28+28 cut (2 GiB block states): FP64 oracle amplitudes of an
  aligned 8-path sub-block of the benchmark's 1024-path block and of the block's last path,
  on the first 4096 of its 1e6 bitstrings (tests/golden/grid7x8_d40_paths.npz, written by
  tests/golden/make_grid7x8_golden.py from the oracle alone), against the HIP path run with
  the tuning the benchmark's autotuner picks for the full request and all 1e6 bitstrings;
  and the full block at that tuning equal to the sum of its two halves (linearity in the path
  set, Section 3).
* 6x7 grid, depth 1+32+1, f = 0.01: 64 live ids spread over the seeded sample of 2,684,355
  (most sampled ids have zero terms, which the library skips), on 1e5 of the workload's
  bitstrings, against the oracle's path sum over the same ids.
* 5x6 grid, all 2^15 paths, 1e5 bitstrings, at the tuning the benchmark's autotuner picks.

Tolerance: max relative |amp|^2 error (parity_tol.c11_error) 1e-5 for complex64 sweeps.
"""
import os

import numpy as np
import pytest

import oracle
from parity_tol import TOL_C64, c11_error
from workload import CONFIGS, equal_bit_pairs, grid_circuit, is_live, make_workload, random_bitstrings

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN_7X8 = os.path.join(HERE, "golden", "grid7x8_d40_paths.npz")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def bench():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import bench as b
    return b


def _release(req):
    import torch
    req["c"].close()
    req.clear()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def req7x8(bench):
    """The benchmark's 7x8 request (1024-path block, 1e6 bitstrings, device buffers, workspace),
    autotuned once for both tests."""
    say("grid7x8_d40: set-up and autotune of the full benchmark request")
    req = bench.prepare("grid7x8_d40", n_measure=3)
    say(f"grid7x8_d40 tuning {req['tuning']}")
    yield req
    _release(req)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_grid7x8_golden_at_benchmark_tuning(req7x8):
    """The sub-block, its paths one at a time and the block's last path against the oracle's
    stored FP64 amplitudes, in the benchmark's launch configuration."""
    from paper_1807_10749_amd import binding as sf
    if not os.path.exists(GOLDEN_7X8):
        pytest.skip("golden file not generated (tests/golden/make_grid7x8_golden.py)")
    gold = np.load(GOLDEN_7X8, allow_pickle=False)
    req = req7x8
    c = req["c"]
    begin, count = req["begin"], req["npaths"]
    assert c.k == int(gold["k"]) and begin == int(gold["block_begin"]) and count == int(gold["block_count"])
    gb = gold["bitstrings"]
    nb = gb.size
    assert np.array_equal(req["bits"][:nb], gb)
    ids = gold["ids"]

    def run(path_ids):
        sf.run_paths(c.handle, np.ascontiguousarray(path_ids, dtype=np.uint64), 0, len(path_ids), req["d_bits"],
                     req["bits"].size, req["d_amps"], req["flags"], req["stream"], req["ws"], req["ws_bytes"])
        return req["d_amps"].cpu().numpy().view(np.complex128)[:nb].copy()

    say(f"grid7x8_d40 sub-block {int(ids[0])}..{int(ids[7])} over all {req['bits'].size} bitstrings")
    a = run(ids[:8])
    assert c11_error(a, gold["sub_block_sum"], 8, c.k, 56) <= TOL_C64
    for i in (0, 5, 8):
        say(f"grid7x8_d40 single path {int(ids[i])}")
        a = run(ids[i:i + 1])
        assert c11_error(a, gold["amps"][i], 1, c.k, 56) <= TOL_C64, int(ids[i])


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_grid7x8_full_block_is_sum_of_halves(req7x8):
    """All 1024 paths of the block over 1e6 bitstrings, benchmark tuning, equal the sum of the
    two aligned 512-path halves run as separate requests."""
    from paper_1807_10749_amd import binding as sf
    req = req7x8
    c, begin, count = req["c"], req["begin"], req["npaths"]

    def run(b, n):
        sf.run_paths(c.handle, None, b, n, req["d_bits"], req["bits"].size, req["d_amps"], req["flags"],
                     req["stream"], req["ws"], req["ws_bytes"])
        return req["d_amps"].cpu().numpy().view(np.complex128).copy()

    say("grid7x8_d40 full block")
    full = run(begin, count)
    say("grid7x8_d40 first half")
    h1 = run(begin, count // 2)
    say("grid7x8_d40 second half")
    h2 = run(begin + count // 2, count // 2)
    err = c11_error(h1 + h2, full, count, c.k, 56)
    assert err <= 2 * TOL_C64, err
    # the block carries amplitude (its paths' terms are nonzero; the oracle goldens check values)
    assert float(np.mean(np.abs(full) ** 2)) > 0.0


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_grid6x7_64_sampled_paths(bench):
    """64 of the seeded f = 0.01 ids on 1e5 bitstrings, library default tuning and dense
    four-qubit blocks, against the oracle."""
    from paper_1807_10749_amd import binding as sf
    cfg = CONFIGS["grid6x7_d32"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    ids_all = sf.sample_paths(c.k, cfg.f, cfg.path_seed)
    pairs = equal_bit_pairs(g, cfg.cut_mask())
    live = np.array([is_live(int(p), pairs) for p in ids_all[:200_000]])
    ids = ids_all[:200_000][live][:: int(live.sum()) // 64][:64]      # 64 live ids spread over the sample
    dead = ids_all[:200_000][~live][:4]
    bits = random_bitstrings(42, 100_000, cfg.bits_seed)
    say(f"grid6x7_d32 oracle over 64 sampled live paths x {bits.size} bitstrings")
    o, na, _ = oracle.path_sum(42, g, cfg.cut_mask(), ids, bits, norms=True)
    assert np.all(na > 1e-12)
    say("grid6x7_d32 oracle norms of 4 zero-term paths of the sample")
    _, nd, _ = oracle.path_sum(42, g, cfg.cut_mask(), dead, bits[:10], norms=True)
    assert np.all(nd == 0.0)
    for tune in ({}, {"dense_qubits": 4}):
        c.tune(**tune)
        say(f"grid6x7_d32 64 sampled paths {tune}")
        a = c.amplitudes(bits, path_ids=ids)
        assert c11_error(a, o, ids.size, c.k, 42) <= TOL_C64, tune
    c.close()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_grid5x6_full_size_at_benchmark_tuning(bench):
    """All 2^15 paths over the 1e5 bitstrings in the launch configuration the benchmark's
    autotuner picks for that request."""
    say("grid5x6_d24: set-up and autotune")
    req = bench.prepare("grid5x6_d24", n_measure=3)
    say(f"grid5x6_d24 tuning {req['tuning']}")
    bench.run_step(req)
    a = req["d_amps"].cpu().numpy().view(np.complex128).copy()
    c = req["c"]
    w = make_workload("grid5x6_d24")
    cfg = w["cfg"]
    o = oracle.path_sum(30, w["gates"], cfg.cut_mask(), np.arange(1 << c.k, dtype=np.uint64), w["bitstrings"])
    assert c11_error(a, o, 1 << c.k, c.k, 30) <= TOL_C64
    _release(req)
