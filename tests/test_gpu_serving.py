"""GPU tests of the serving runtime and the autotuner.

Each job's result must be the same alone and in a mix of concurrently
served jobs (same path chunks, same kernels: equal up to FP64 rounding),
must match the FP64 oracle (tolerance as in test_gpu_parity), and the
server must never hold more than its arena.
"""
import numpy as np
import pytest

import oracle
from workload import grid_circuit, random_bitstrings

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding
    return binding


JOBS = [  # rows, cols, depth, circuit seed, n_bits, f, path seed
    (4, 4, 16, 11, 500, 1.0, 0),
    (4, 5, 16, 12, 2000, 0.1, 5),
    (3, 5, 20, 13, 700, 1.0, 0),
    (4, 4, 24, 14, 300, 0.5, 9),
    (5, 4, 12, 15, 1500, 1.0, 0),
    (2, 6, 16, 16, 64, 1.0, 0),
    (5, 5, 16, 17, 3000, 0.01, 3),
]


def _submit(sf, srv, spec):
    rows, cols, depth, cseed, nb, f, pseed = spec
    g = grid_circuit(rows, cols, depth, cseed)
    bits = random_bitstrings(rows * cols, nb, cseed + 1000)
    return sf.server_submit(srv, rows, cols, g, bits, f=f, path_seed=pseed), g, bits


def _wait(sf, srv, jid, nb):
    sf.server_drain(srv)
    done, amps, info = sf.server_poll(srv, jid, nb)
    assert done and info["status"] == 0
    return amps, info


def test_server_alone_equals_mix(sf):
    alone = []
    for spec in JOBS:
        say(f"server alone {spec}")
        srv = sf.server_create(4 << 30, None, 2, 256)
        jid, g, bits = _submit(sf, srv, spec)
        a, _ = _wait(sf, srv, jid, bits.size)
        alone.append(a.copy())
        sf.server_destroy(srv)
    say("server mix of all jobs, 4 workers")
    srv = sf.server_create(8 << 30, None, 4, 256)
    ids = [(_submit(sf, srv, spec), spec) for spec in JOBS]
    sf.server_drain(srv)
    st = sf.server_stats(srv)
    for ((jid, g, bits), spec), a in zip(ids, alone):
        done, m, info = sf.server_poll(srv, jid, bits.size)
        assert done and info["status"] == 0
        assert np.abs(m - a).max() <= 1e-12 * max(np.abs(a).max(), 1e-300), spec
    assert st["peak_bytes"] <= st["arena_bytes"]
    assert st["max_concurrent_chunks"] >= 2, "jobs should overlap on the device"
    sf.server_destroy(srv)


def test_server_results_match_oracle(sf):
    srv = sf.server_create(2 << 30, None, 2, 64)
    for spec in (JOBS[0], JOBS[1]):
        rows, cols, depth, cseed, nb, f, pseed = spec
        say(f"server vs oracle {spec}")
        jid, g, bits = _submit(sf, srv, spec)
        a, info = _wait(sf, srv, jid, bits.size)
        n = rows * cols
        c = sf.Circuit(rows, cols, g)
        k = c.k
        ids = np.arange(1 << k, dtype=np.uint64) if f >= 1 else oracle.sample_paths(k, f, pseed)
        o = oracle.path_sum(n, g, c.mask_a, ids, bits)
        c.close()
        assert info["n_paths"] == ids.size
        floor = (ids.size / 2.0 ** k) * 2.0 ** (-n)
        err = np.max(np.abs(np.abs(a) ** 2 - np.abs(o) ** 2) / np.maximum(np.abs(o) ** 2, floor))
        assert err <= 1e-5, err
    sf.server_destroy(srv)


def test_server_iswap_jobs_match_oracle(sf):
    """iSWAP circuits (four terms per crossing gate) served next to a CZ job."""
    from workload import ISWAP
    srv = sf.server_create(2 << 30, None, 3, 64)
    specs = [(3, 4, 10, 21, 400, 1.0, 0, ISWAP), (4, 4, 12, 22, 600, 0.05, 7, ISWAP), (4, 4, 16, 11, 500, 1.0, 0, 4)]
    subs = []
    for rows, cols, depth, cseed, nb, f, pseed, two in specs:
        g = grid_circuit(rows, cols, depth, cseed, two_qubit=two)
        bits = random_bitstrings(rows * cols, nb, cseed + 1000)
        subs.append((sf.server_submit(srv, rows, cols, g, bits, f=f, path_seed=pseed), g, bits, rows, cols, f, pseed))
    say("server iSWAP + CZ mix")
    sf.server_drain(srv)
    for jid, g, bits, rows, cols, f, pseed in subs:
        done, a, info = sf.server_poll(srv, jid, bits.size)
        assert done and info["status"] == 0
        n = rows * cols
        c = sf.Circuit(rows, cols, g)
        k = c.k
        ids = np.arange(1 << k, dtype=np.uint64) if f >= 1 else oracle.sample_paths(k, f, pseed)
        o = oracle.path_sum(n, g, c.mask_a, ids, bits)
        c.close()
        assert info["n_paths"] == ids.size
        floor = (ids.size / 2.0 ** k) * 2.0 ** (-n)
        err = np.max(np.abs(np.abs(a) ** 2 - np.abs(o) ** 2) / np.maximum(np.abs(o) ** 2, floor))
        assert err <= 1e-5, (rows, cols, f, err)
    sf.server_destroy(srv)


def test_server_admission_respects_arena(sf):
    """Each job needs at least a 256 MiB workspace: a 1 GiB arena holds three at a time."""
    say("server admission, 1 GiB arena, 8 jobs")
    srv = sf.server_create(1 << 30, None, 4, 128)
    subs = [_submit(sf, srv, JOBS[i % 3]) for i in range(8)]
    sf.server_drain(srv)
    st = sf.server_stats(srv)
    assert st["peak_bytes"] <= 1 << 30
    assert st["waiting"] == 0 and st["active"] == 0
    for jid, g, bits in subs:
        done, a, info = sf.server_poll(srv, jid, bits.size)
        assert done and info["status"] == 0 and info["t_admit"] >= info["t_submit"]
    with pytest.raises(sf.SFError):
        # one job larger than the whole arena is refused at submission
        rows, cols = 5, 6
        g = grid_circuit(rows, cols, 16, 3)
        sf.server_submit(srv, rows, cols, g, np.arange(40_000_000, dtype=np.uint64))
    sf.server_destroy(srv)


def test_autotune_keeps_parity(sf):
    from workload import CONFIGS
    cfg = CONFIGS["grid5x6_d24"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    bits = random_bitstrings(30, 2000, 77)
    ids = np.arange(4096, 4096 + 1024, dtype=np.uint64)
    amps = np.zeros(2 * bits.size)
    say("autotune grid5x6_d24, 1024 paths")
    t = sf.autotune(c.handle, ids, 0, ids.size, bits, bits.size, amps, n_measure=3)
    assert 0 <= t["reg_qubits"] <= 5   # 0 = library default
    a = c.amplitudes(bits, path_ids=ids)
    o = oracle.path_sum(30, g, cfg.cut_mask(), ids, bits)
    floor = (ids.size / 2.0 ** c.k) * 2.0 ** (-30)
    err = np.max(np.abs(np.abs(a) ** 2 - np.abs(o) ** 2) / np.maximum(np.abs(o) ** 2, floor))
    assert err <= 1e-5, err
    c.close()


def test_autotune_cache_file(sf, tmp_path):
    """A tuning saved to a file and loaded again is taken by autotune without measuring."""
    import time
    from workload import CONFIGS
    cfg = CONFIGS["grid4x4_d16"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    bits = random_bitstrings(16, 333, 5)
    amps = np.zeros(2 * bits.size)
    say("autotune grid4x4_d16, 200 paths, then save / load the cache")
    t = sf.autotune(c.handle, None, 0, 200, bits, bits.size, amps, n_measure=2)
    path = tmp_path / "tune.txt"
    sf.save_tuning_cache(str(path))
    want = " ".join(str(t[k]) for k in ("reg_qubits", "leaf_batch", "max_slots", "waves_per_cu", "dense_qubits",
                                         "no_leaf_fold", "fold_levels", "chain_passes", "no_row_skip", "no_defer",
                                         "no_chain_merge", "jit", "no_tail_move"))
    lines = [l for l in path.read_text().splitlines() if l.endswith("/200/333/0 " + want)]
    assert len(lines) == 1 and lines[0].startswith("gfx950:"), path.read_text()
    # a stored tuning for this key replaces the cached one and is returned as is
    key = lines[0].split()[0]
    forced = "4 0 0 16 0 1 0 1 1 0 1 0 1"
    (tmp_path / "forced.txt").write_text(f"{key} {forced}\n")
    assert sf.load_tuning_cache(str(tmp_path / "forced.txt")) == 1
    c.tune()
    t0 = time.perf_counter()
    t2 = sf.autotune(c.handle, None, 0, 200, bits, bits.size, amps, n_measure=2)
    assert time.perf_counter() - t0 < 0.5
    assert " ".join(str(t2[k]) for k in ("reg_qubits", "leaf_batch", "max_slots", "waves_per_cu", "dense_qubits",
                                         "no_leaf_fold", "fold_levels", "chain_passes", "no_row_skip", "no_defer",
                                         "no_chain_merge", "jit", "no_tail_move")) == forced
    assert sf.get_tuning(c.handle) == t2
    a = c.amplitudes(bits, n_paths=200)
    o = oracle.path_sum(16, g, cfg.cut_mask(), np.arange(200, dtype=np.uint64), bits)
    floor = (200 / 2.0 ** c.k) * 2.0 ** (-16)
    assert np.max(np.abs(np.abs(a) ** 2 - np.abs(o) ** 2) / np.maximum(np.abs(o) ** 2, floor)) <= 1e-5
    c.close()
