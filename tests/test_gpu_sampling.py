"""GPU parity of rejection sampling (Section "Frugal rejection sampling", Algorithms 1 and 2)
through the C ABI against the oracle.

Acceptance decisions are integers decided by floating point: both sides compute them in FP64
with every product and sum rounded on its own, so on the same amplitudes the accepted index
lists must be identical.  End to end, the GPU amplitudes differ from the oracle's by the sweep
rounding; decisions whose draw lies within that rounding of the threshold are not compared.
"""
import numpy as np
import pytest

import oracle
from workload import CONFIGS, grid_circuit

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


def _accept_gpu(sf, amps, n_qubits, m, seed, flags=0):
    import torch
    d_amps = torch.from_numpy(np.ascontiguousarray(amps).view(np.float64).copy()).cuda()
    acc = torch.zeros(max(amps.size, 1), dtype=torch.int32, device="cuda")
    nb = sf.rejection_workspace_size(amps.size)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    n_acc, err = sf.rejection_accept(d_amps, amps.size, n_qubits, m, seed, acc, flags, torch.cuda.current_stream(),
                                     ws, ws.numel())
    return acc[:n_acc].cpu().numpy().astype(np.int64), err


@pytest.mark.parametrize("basic", [False, True])
@pytest.mark.parametrize("count", [1, 1000, 2_000_000])
def test_accept_matches_oracle(sf, basic, count):
    n, mp, seed = 30, (41.0 if basic else 10.0), 123 + count
    t = np.random.default_rng(count).exponential(1.0, count)
    ph = np.random.default_rng(count + 1).uniform(0, 2 * np.pi, count)
    amps = (np.sqrt(t / 2.0 ** n) * np.exp(1j * ph)).astype(np.complex128)
    say(f"rejection_accept count={count} basic={basic}")
    idx, err = _accept_gpu(sf, amps, n, mp, seed, sf.SF_SAMPLE_BASIC if basic else 0)
    acc, err_o = oracle.rejection_accept(amps, n, mp, seed, basic=basic)
    np.testing.assert_array_equal(idx, np.flatnonzero(acc))
    assert abs(err - err_o) <= 1e-12 * max(abs(err_o), 1e-300)


def test_accept_constructed_edges(sf):
    """Zero probability, probabilities far above, exactly at and just around the draws and the
    threshold: the same decisions as the oracle."""
    n, mp, seed = 20, 10.0, 1234567
    N = 2.0 ** n
    u = [(oracle.splitmix64_at(seed, j) >> 11) * 2.0 ** -53 for j in range(8)]
    t = np.array([0.0, 3.0, u[2] * (1 + 1e-12), u[3] * (1 - 1e-12), 1.0, 1.5, u[6], 0.999])
    amps = np.sqrt(t * mp / N).astype(np.complex128)
    amps[4] = (3 + 1j) * 2.0 ** -10
    for flags, basic in ((0, False), (sf.SF_SAMPLE_BASIC, True)):
        say(f"rejection_accept constructed inputs basic={basic}")
        idx, err = _accept_gpu(sf, amps, n, mp, seed, flags)
        acc, err_o = oracle.rejection_accept(amps, n, mp, seed, basic=basic)
        np.testing.assert_array_equal(idx, np.flatnonzero(acc))
        assert err == err_o
    say("rejection_accept zero candidates")
    idx, err = _accept_gpu(sf, np.zeros(0, dtype=np.complex128), n, mp, seed)
    assert idx.size == 0 and err == 0.0


def _oracle_pipeline(cfg, g, ids, n_cand, m, seed_c, seed_u, basic=False):
    cand = oracle.sample_bitstrings(cfg.n_qubits, n_cand, seed_c)
    amps = oracle.path_sum(cfg.n_qubits, g, cfg.cut_mask(), ids, cand)
    acc, err = oracle.rejection_accept(amps, cfg.n_qubits, m, seed_u, basic=basic)
    return cand, amps, acc, err


@pytest.mark.parametrize("basic", [False, True])
def test_frugal_sample_end_to_end_4x4(sf, basic):
    """All 2^16 bitstrings of the 4x4 circuit as candidates, all 256 paths, complex128 sweeps:
    the accepted set equals the oracle pipeline's; about l = n/M' samples come out."""
    cfg = CONFIGS["grid4x4_d16"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    n_cand = 1 << 16
    m = sf.rejection_m(16, 1e-3, sf.SF_SAMPLE_BASIC) if basic else 10.0
    flags = sf.SF_FP64_SWEEPS | (sf.SF_SAMPLE_BASIC if basic else 0)
    say(f"frugal_sample 4x4 basic={basic}")
    out, err = sf.frugal_sample(c.handle, None, 0, 1 << c.k, n_cand, m, 77, 78, flags)
    cand, amps, acc, err_o = _oracle_pipeline(cfg, g, np.arange(1 << c.k, dtype=np.uint64), n_cand, m, 77, 78, basic)
    p = np.abs(amps) ** 2
    t = p * 2.0 ** 16 / m
    u = np.array([(oracle.splitmix64_at(78, j) >> 11) * 2.0 ** -53 for j in range(n_cand)])
    clear = np.abs(u - t) > 1e-9 * np.maximum(t, 1e-300)
    if basic:
        clear &= np.abs(t - 1.0) > 1e-9
    got = np.isin(cand, out)
    assert np.array_equal(got[clear], acc[clear])
    assert (~clear).sum() <= 2
    assert np.all(np.diff(np.flatnonzero(np.isin(cand, out))) > 0) and np.array_equal(out, cand[got])
    assert abs(err - err_o) <= 1e-6 * max(err_o, 1e-12)
    lo = n_cand / m * (1 - np.exp(-m)) if not basic else n_cand / m * 0.9
    assert abs(out.size - lo) < 6 * np.sqrt(n_cand / m) + 0.15 * lo


def test_frugal_sample_5x6_subset_and_workspace(sf):
    """Benchmark circuit, 300 sampled paths (f < 1), 20000 candidates, complex64 sweeps, with a
    caller workspace: decisions away from the sweep rounding equal the oracle pipeline's."""
    import torch
    cfg = CONFIGS["grid5x6_d24"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    ids = np.sort(np.random.default_rng(3).choice(1 << c.k, 300, replace=False)).astype(np.uint64)
    ws = torch.empty(1 << 29, dtype=torch.uint8, device="cuda")
    say("frugal_sample 5x6, 300 paths, 20000 candidates")
    out, err = sf.frugal_sample(c.handle, ids, 0, ids.size, 20000, 10.0, 5, 6, 0, torch.cuda.current_stream(), ws,
                                ws.numel())
    cand, amps, acc, err_o = _oracle_pipeline(cfg, g, ids, 20000, 10.0, 5, 6)
    t = np.abs(amps) ** 2 * 2.0 ** 30 / 10.0
    u = np.array([(oracle.splitmix64_at(6, j) >> 11) * 2.0 ** -53 for j in range(20000)])
    clear = np.abs(u - t) > 1e-4 * np.maximum(t, 1e-300)
    got = np.isin(cand, out)
    assert np.array_equal(got[clear], acc[clear])
    assert (~clear).sum() <= 3
    assert abs(err - err_o) <= 1e-3 * max(err_o, 1e-12) + 1e-9
    with pytest.raises(sf.SFError):
        sf.frugal_sample(c.handle, ids, 0, ids.size, 20000, 10.0, 5, 6, 0, None, ws, 1 << 20)
