"""Pins of the oracle's rejection sampling (Section "Frugal rejection sampling", Algorithms 1
and 2) against the paper's printed numbers, closed forms under Porter-Thomas statistics, exact
decisions on constructed inputs and the published SplitMix64 outputs."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from workload import random_bitstrings, splitmix64_array

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rejection_sampling.json")))


def test_m_values_match_the_paper():
    g = GOLD["basic_m"]
    assert oracle.rejection_m(g["n_qubits"], g["eps"], basic=True) == g["M"]
    g = GOLD["frugal_truncation"]
    assert oracle.rejection_m(49, g["eps"]) == g["M_prime"]
    # the truncation distance e^{-M'} (1 + M') is the printed 5e-4 at M' = 10 ...
    assert abs(math.exp(-10) * 11 - g["eps"]) < 0.01 * g["eps"]
    # ... and M' does not depend on the number of qubits
    assert oracle.rejection_m(20, g["eps"]) == oracle.rejection_m(53, g["eps"]) == 10


def _pt_integrals(mp, always_accept):
    """Distance between p and the accepted distribution under Porter-Thomas statistics, by
    numerical integration over t = N p with density e^{-t} (x uniform) and mass t e^{-t}."""
    t = np.linspace(0.0, 80.0, 800001)
    dt = t[1] - t[0]
    a = np.minimum(1.0, t / mp) if always_accept else np.where(t <= mp, t / mp, 0.0)
    acc = a * np.exp(-t)
    pt = acc / (acc.sum() * dt)
    p = t * np.exp(-t)
    return 0.5 * np.abs(p - pt).sum() * dt, np.abs(p - pt).sum() * dt


def test_distance_closed_forms():
    """Truncation (Algorithm 1 rule with M'): e^{-M'}(1 + M') = 5e-4 at M' = 10.  Always
    accepting high probabilities: the total variation distance is exp(-M'/(1 - e^{-M'})) =
    4.5e-5 at M' = 10; the printed 9e-5 = 2 exp(...) equals the L1 distance sum |p - p~|."""
    tvd, _ = _pt_integrals(10.0, False)
    assert abs(tvd - math.exp(-10) * 11) < 1e-3 * tvd
    tvd, l1 = _pt_integrals(10.0, True)
    c = 10.0 / (1.0 - math.exp(-10.0))
    assert abs(tvd - math.exp(-c)) < 1e-3 * tvd
    g = GOLD["frugal_always_accept"]
    assert abs(l1 - g["printed"]) < 0.02 * g["printed"]


def test_candidates_distinct_uniform():
    for n, count, seed in ((16, 5000, 7), (30, 100000, 2002), (12, 4096, 3), (64, 1000, 5)):
        c = oracle.sample_bitstrings(n, count, seed)
        assert c.size == count and np.unique(c).size == count
        if n < 64:
            assert int(c.max()) < (1 << n)
        # the input generator implements the same published definition independently
        np.testing.assert_array_equal(c, random_bitstrings(n, count, seed))
    c = oracle.sample_bitstrings(12, 4096, 3)
    assert np.array_equal(np.sort(c), np.arange(4096, dtype=np.uint64))   # all of them
    c = oracle.sample_bitstrings(20, 200000, 11)
    hist = np.bincount((c >> np.uint64(14)).astype(np.int64), minlength=64)
    chi2 = ((hist - c.size / 64) ** 2 / (c.size / 64)).sum()
    assert chi2 < 120                                                     # 63 dof


def test_acceptance_draws_are_splitmix64():
    assert oracle.splitmix64_at(0, 0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64_at(0, 2) == 0x06C45D188009454F
    assert oracle.splitmix64_at(1234567, 1) == 3203168211198807973
    ref = splitmix64_array(99, 50)
    assert all(oracle.splitmix64_at(99, j) == int(ref[j]) for j in range(50))


def test_acceptance_decisions_on_constructed_inputs():
    n, mp, seed = 20, 10.0, 1234567
    N = 2.0 ** n
    u = [(oracle.splitmix64_at(seed, j) >> 11) * 2.0 ** -53 for j in range(8)]
    # candidate j has probability t_j M'/N: zero, far above the threshold, just above and just
    # below its own draw u_j, exactly at the threshold
    t = np.array([0.0, 3.0, u[2] * (1 + 1e-9), u[3] * (1 - 1e-9), 1.0, 1.5, u[6] * (1 + 1e-9), 0.999])
    amps = np.sqrt(t * mp / N).astype(np.complex128)
    amps[4] = (3 + 1j) * 2.0 ** -10          # p = 10 / 2^20 exactly: t = 1 exactly
    acc, err = oracle.rejection_accept(amps, n, mp, seed)
    assert list(acc[:5]) == [False, True, True, False, True] and acc[5] and acc[6]
    assert acc[7] == (u[7] < 0.999)
    # the mass above the threshold, scaled from the 8 uniform candidates to all N bitstrings
    assert abs(err - (3.0 + 1.5) * mp / N * N / 8) < 1e-12
    acc_b, err_b = oracle.rejection_accept(amps, n, mp, seed, basic=True)
    # Algorithm 1 removes candidates above M/N and keeps the rest of the decisions
    assert not acc_b[1] and not acc_b[5] and acc_b[4]
    assert list(acc_b[[0, 2, 3, 6, 7]]) == list(acc[[0, 2, 3, 6, 7]])
    assert err_b == err
    # a phase does not change the decision
    acc_p, _ = oracle.rejection_accept(amps * np.exp(0.7j), n, mp, seed)
    assert np.array_equal(acc_p, acc) or np.sum(acc_p != acc) <= 1     # |a e^{i phi}|^2 rounds


@pytest.mark.parametrize("basic", [False, True])
def test_porter_thomas_acceptance_statistics(basic):
    """Uniform candidates with Porter-Thomas probabilities: accepted fraction
    (1 - e^{-M'})/M' (Algorithm 2) or (1 - e^{-M}(1+M))/M (Algorithm 1), about l bitstrings from
    l M' candidates; the accepted t = N p follow the target density t e^{-t} (mean 2, or the
    truncated mean)."""
    n, mp = 30, 10.0
    count = 2_000_000
    t = np.random.default_rng(5).exponential(1.0, count)
    amps = np.sqrt(t / 2.0 ** n).astype(np.complex128)
    acc, err = oracle.rejection_accept(amps, n, mp, 777, basic=basic)
    rate = acc.mean()
    want = (1 - math.exp(-mp) * (1 + mp)) / mp if basic else (1 - math.exp(-mp)) / mp
    assert abs(rate - want) < 5 * math.sqrt(want * (1 - want) / count)
    ta = t[acc]
    if basic:
        mean = (2 - math.exp(-mp) * (mp * mp + 2 * mp + 2)) / (1 - math.exp(-mp) * (1 + mp))
    else:
        mean = 2.0
    assert abs(ta.mean() - mean) < 5 * math.sqrt(2.0 / ta.size)
    # the batch estimate of the mass above M'/N is e^{-M'}(1 + M') within its statistics
    assert abs(err - math.exp(-mp) * (1 + mp)) < 0.35 * math.exp(-mp) * (1 + mp)


def test_batch_error_on_circuits_matches_the_paper():
    """All 2^20 outputs of T-rich 20-qubit circuits as candidates: the batch estimate is the
    exact mass above 10/N, which the paper measured as (4.4 +- 0.7) 1e-4 on its circuits
    (5.3 +- 0.7 on the approximate simulation); Porter-Thomas gives 5.0e-4."""
    from test_oracle_pins import _t_rich_circuit
    n = 20
    errs = []
    for seed in (4242, 1, 2, 3, 4):
        psi = oracle.full_state(n, _t_rich_circuit(4, 5, 40, seed))
        cand = oracle.sample_bitstrings(n, 1 << n, seed)
        _, e = oracle.rejection_accept(psi[cand.astype(np.int64)], n, 10.0, seed)
        errs.append(e)
    g = GOLD["batch_error_exact"]
    assert g["value"] - 3 * g["err"] < np.mean(errs) < GOLD["batch_error_approx"]["value"] + 5 * g["err"]
