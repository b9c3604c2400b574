"""run_paths_noalloc (the entry point without device allocations) against run_paths.

Two calls in a row through the C ABI on one GPU, the second with fewer bitstrings and paths,
each compared with run_paths on the same request (parity_tol.c11_error, 1e-5 for complex64
sweeps, 1e-10 for complex128) and with the FP64 oracle; then a request too large for the
library's 64 MiB workspace is refused with SF_ERR_OOM, and the entry point still works after it.
"""
import numpy as np
import pytest

import oracle
from parity_tol import TOL_C128, TOL_C64, c11_error
from workload import CONFIGS, column_cut_mask, grid_circuit, random_bitstrings

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def test_noalloc_matches_run_paths():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding as sf
    stream = torch.cuda.current_stream()
    flags_dev = sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE
    cases = [(4, 5, 18, 7, 2, 20_000, None, 0), (4, 4, 16, 1001, 2, 3_000, 100, sf.SF_FP64_SWEEPS)]
    for rows, cols, depth, seed, ncols_a, nb, npaths, fl in cases:
        n = rows * cols
        g = grid_circuit(rows, cols, depth, seed)
        mask = column_cut_mask(rows, cols, ncols_a)
        c = sf.Circuit(rows, cols, g, mask)
        bits = random_bitstrings(n, nb, seed + 1)
        ids = np.arange(npaths if npaths else 1 << c.k, dtype=np.uint64)
        d_bits = torch.from_numpy(bits.view(np.int64)).cuda()
        d_a = torch.zeros(2 * nb, dtype=torch.float64, device="cuda")
        d_b = torch.full((2 * nb,), 5.0, dtype=torch.float64, device="cuda")
        say(f"noalloc {rows}x{cols} d{depth}: {ids.size} paths, {nb} bitstrings, flags {fl}")
        sf.run_paths(c.handle, ids, 0, ids.size, d_bits, nb, d_a, fl | flags_dev, stream)
        sf.run_paths_noalloc(c.handle, ids, 0, ids.size, d_bits, nb, d_b, fl | flags_dev, stream)
        a = d_a.cpu().numpy().view(np.complex128)
        b = d_b.cpu().numpy().view(np.complex128)
        tol = TOL_C128 if fl else TOL_C64
        assert c11_error(b, a, ids.size, c.k, n) <= tol
        o = oracle.path_sum(n, g, mask, ids, bits)
        assert c11_error(b, o, ids.size, c.k, n) <= tol
        c.close()
    # too large for the 64 MiB workspace: 4x6 with 12-qubit blocks and 2^20 slots of paths
    cfg = CONFIGS["grid5x6_d24"]
    g = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    c = sf.Circuit(cfg.rows, cfg.cols, g, cfg.cut_mask())
    bits = random_bitstrings(30, 4_000_000, 3)
    d_bits = torch.from_numpy(bits.view(np.int64)).cuda()
    d_a = torch.zeros(2 * bits.size, dtype=torch.float64, device="cuda")
    say("noalloc: request beyond the 64 MiB workspace")
    with pytest.raises(sf.SFError) as e:
        sf.run_paths_noalloc(c.handle, None, 0, 64, d_bits, bits.size, d_a, flags_dev, stream)
    assert e.value.code == sf.SF_ERR_OOM and "64 MiB" in str(e.value)
    with pytest.raises(sf.SFError) as e:
        sf.run_paths_noalloc(c.handle, None, 0, 64, d_bits, 10, d_a, sf.SF_OUT_ON_DEVICE, stream)
    assert e.value.code == sf.SF_ERR_INVALID
    say("noalloc: a small request after the refusal")
    sf.run_paths_noalloc(c.handle, None, 0, 64, d_bits, 1000, d_a, flags_dev, stream)
    ref = np.zeros(2000)
    sf.run_paths(c.handle, None, 0, 64, bits[:1000], 1000, ref)
    assert c11_error(d_a.cpu().numpy()[:2000].view(np.complex128), ref.view(np.complex128), 64, c.k, 30) <= TOL_C64
    c.close()


def test_noalloc_with_compiled_passes_compiles_nothing():
    """With tuning jit the entry point compiles and loads no kernel (that allocates device memory):
    before any compile of the circuit's programs it runs interpreted, after run_paths compiled
    them it runs the cached kernels; both equal run_paths."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1807_10749_amd import binding as sf
    stream = torch.cuda.current_stream()
    flags_dev = sf.SF_OUT_ON_DEVICE | sf.SF_BITS_ON_DEVICE
    rows, cols, depth, seed, nb = 4, 5, 14, 4242, 5_000
    n = rows * cols
    g = grid_circuit(rows, cols, depth, seed)
    c = sf.Circuit(rows, cols, g, column_cut_mask(rows, cols, 2))
    bits = random_bitstrings(n, nb, seed + 1)
    ids = np.arange(1 << c.k, dtype=np.uint64)
    d_bits = torch.from_numpy(bits.view(np.int64)).cuda()
    d_a = torch.zeros(2 * nb, dtype=torch.float64, device="cuda")
    d_b = torch.zeros(2 * nb, dtype=torch.float64, device="cuda")
    say("noalloc with tuning jit before any compile of the circuit's programs")
    c.tune(jit=1)
    sf.run_paths_noalloc(c.handle, ids, 0, ids.size, d_bits, nb, d_b, flags_dev, stream)
    torch.cuda.synchronize()
    s = c.stats()
    assert s["n_jit_passes"] == 0 and s["jit_compile_ms"] == 0.0, s
    c.tune(jit=0)
    sf.run_paths(c.handle, ids, 0, ids.size, d_bits, nb, d_a, flags_dev, stream)
    torch.cuda.synchronize()
    a, b = d_a.cpu().numpy().view(np.complex128), d_b.cpu().numpy().view(np.complex128)
    assert c11_error(b, a, ids.size, c.k, n) <= TOL_C64
    say("noalloc with tuning jit after run_paths compiled the programs")
    c.tune(jit=1)
    sf.run_paths(c.handle, ids, 0, ids.size, d_bits, nb, d_a, flags_dev, stream)
    torch.cuda.synchronize()
    assert c.stats()["n_jit_passes"] > 0
    sf.run_paths_noalloc(c.handle, ids, 0, ids.size, d_bits, nb, d_b, flags_dev, stream)
    torch.cuda.synchronize()
    s = c.stats()
    assert s["n_jit_passes"] > 0 and s["jit_compile_ms"] == 0.0, s
    a, b = d_a.cpu().numpy().view(np.complex128), d_b.cpu().numpy().view(np.complex128)
    assert c11_error(b, a, ids.size, c.k, n) <= TOL_C64
    o = oracle.path_sum(n, g, column_cut_mask(rows, cols, 2), ids, bits)
    assert c11_error(b, o, ids.size, c.k, n) <= TOL_C64
    c.close()
