"""Pins of the oracle's validation tools (appendix on validating simulation results): the state
overlap estimated from amplitudes at common indices, the protocol's expectations, and the linear
cross-entropy fidelity, against algebraic properties, Eq. (fid) and Porter-Thomas statistics."""
import math

import numpy as np

import oracle
from workload import grid_circuit


def test_overlap_estimate_algebra():
    rng = np.random.default_rng(1)
    a = rng.normal(size=500) + 1j * rng.normal(size=500)
    b = rng.normal(size=500) + 1j * rng.normal(size=500)
    assert abs(oracle.fidelity_estimate(a, (0.3 - 2j) * a)[0] - 1.0) < 1e-12      # phase and scale
    fab, na, nb = oracle.fidelity_estimate(a, b)
    assert abs(fab - oracle.fidelity_estimate(b, a)[0]) < 1e-12 and 0.0 <= fab <= 1.0
    assert abs(na - np.sum(np.abs(a) ** 2)) < 1e-9 and abs(nb - np.sum(np.abs(b) ** 2)) < 1e-9
    # orthogonal vectors; a vector against itself plus an orthogonal part of equal norm
    e = np.zeros(4, complex); e[0] = 1
    g = np.zeros(4, complex); g[1] = 1
    assert oracle.fidelity_estimate(e, g)[0] == 0.0
    assert abs(oracle.fidelity_estimate(e, e + g)[0] - 0.5) < 1e-15


def _subset_state(n, g, mask, f, seed):
    k = oracle.num_cut(n, g, mask)
    ids = oracle.sample_paths(k, f, seed)
    return oracle.path_sum(n, g, mask, ids, np.arange(1 << n, dtype=np.uint64))


def test_fidelity_of_path_subsets_and_the_protocol():
    """Section 3, Eq. (fid): keeping a fraction f of the paths gives fidelity ~ f, which the
    estimate on all 2^n amplitudes and on a seeded subset of k amplitudes both show; and the
    appendix's claim that two independent approximate states with fidelities f1 and f have
    fidelity ~ f1 f to each other."""
    n = 16
    g = grid_circuit(4, 4, 24, 1000)          # 12 crossing CZs: 4096 paths
    mask = sum(1 << (r * 4 + c) for r in range(4) for c in range(2))
    psi = oracle.full_state(n, g)
    fs = []
    for f, seed in ((0.5, 1), (0.25, 2), (0.125, 3)):
        a = _subset_state(n, g, mask, f, seed)
        fe_all = oracle.fidelity_estimate(psi, a)[0]
        idx = oracle.sample_bitstrings(n, 20000, 40 + seed).astype(np.int64)
        fe_k = oracle.fidelity_estimate(psi[idx], a[idx])[0]
        assert abs(fe_all - f) < 0.25 * f, (f, fe_all)
        assert abs(fe_k - fe_all) < 0.15 * fe_all, (fe_k, fe_all)
        fs.append((f, a))
    (f1, a1), (f2, a2) = fs[0], fs[2]
    cross = oracle.fidelity_estimate(a1, a2)[0]
    assert abs(cross - f1 * f2) < 0.5 * f1 * f2, (cross, f1 * f2)


def test_cross_entropy_fidelity():
    """Linear cross-entropy N <p(x)> - 1: ~1 for samples from a Porter-Thomas output distribution
    (N sum p^2 - 1), ~0 for uniform samples, ~f for a mixture that is ideal with weight f."""
    from test_oracle_pins import _t_rich_circuit
    n = 20
    psi = oracle.full_state(n, _t_rich_circuit(4, 5, 40, 4242))
    p = np.abs(psi) ** 2
    rng = np.random.default_rng(9)
    ideal = rng.choice(1 << n, size=200000, p=p / p.sum())
    uniform = rng.integers(0, 1 << n, 200000)
    x_ideal = oracle.xeb_fidelity(psi[ideal], n)
    assert abs(x_ideal - ((1 << n) * np.sum(p * p) - 1)) < 0.03 and abs(x_ideal - 1) < 0.1
    assert abs(oracle.xeb_fidelity(psi[uniform], n)) < 0.02
    f = 0.3
    mix = np.where(rng.random(200000) < f, ideal, uniform)
    assert abs(oracle.xeb_fidelity(psi[mix], n) - f) < 0.03
