"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test compares the oracle with something it does not compute: matrix
algebra, a brute-force full-space construction written separately here
(Kronecker products of matrices derived from the Pauli matrices with
scipy's principal square root), closed forms, exact identities of the
projector decomposition (Section 2, Eq. (CZ)), statistics fixed by the
paper (Section 3 Eq. (fid), Section 4 Porter-Thomas), and numbers the
paper's logs print (tests/golden/paper_numbers.json).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from workload import (CZ, H, T, XH, YH, GATE_DTYPE, column_cut_mask, grid_circuit,
                      random_bitstrings, row_cut_mask)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")

PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.diag([1.0, -1.0]).astype(complex)
I2 = np.eye(2, dtype=complex)


def _reference_matrix(kind):
    """Gate matrices derived independently of the oracle's source."""
    if kind == H:
        return (PX + PZ) / math.sqrt(2.0)
    if kind == XH:
        return sl.sqrtm(PX)
    if kind == YH:
        return sl.sqrtm(PY)
    if kind == T:
        return sl.sqrtm(sl.sqrtm(PZ))
    raise ValueError(kind)


def _op_on(n, q, m):
    """Full 2^n operator applying 2x2 m on qubit q (bit q of the index)."""
    out = np.eye(1, dtype=complex)
    for j in reversed(range(n)):      # kron puts the first factor on the top bit
        out = np.kron(out, m if j == q else I2)
    return out


def _cz_full(n, a, b):
    d = np.ones(1 << n, dtype=complex)
    for i in range(1 << n):
        if (i >> a) & 1 and (i >> b) & 1:
            d[i] = -1
    return np.diag(d)


def _brute_state(n, gates):
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1
    for g in gates:
        if g["kind"] == CZ:
            psi = _cz_full(n, int(g["q0"]), int(g["q1"])) @ psi
        else:
            psi = _op_on(n, int(g["q0"]), _reference_matrix(int(g["kind"]))) @ psi
    return psi


def _random_gate_list(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(0, 5 if n > 1 else 4))
        if kind == CZ:
            a, b = rng.choice(n, size=2, replace=False)
            out.append((CZ, 0, 0, int(a), int(b)))
        else:
            out.append((kind, 0, 0, int(rng.integers(0, n)), 0))
    return np.array(out, dtype=GATE_DTYPE)


# ---------------------------------------------------------------- matrices

@pytest.mark.parametrize("kind", [H, XH, YH, T])
def test_gate_matrix_matches_independent_derivation(oracle_lib, kind):
    np.testing.assert_allclose(oracle.gate_matrix(kind), _reference_matrix(kind), atol=1e-15)


def test_gate_algebra(oracle_lib):
    h, x, y, t = (oracle.gate_matrix(k) for k in (H, XH, YH, T))
    np.testing.assert_allclose(x @ x, PX, atol=1e-15)
    np.testing.assert_allclose(y @ y, PY, atol=1e-15)
    np.testing.assert_allclose(h @ h, I2, atol=1e-15)
    np.testing.assert_allclose(np.linalg.matrix_power(t, 8), I2, atol=1e-15)
    np.testing.assert_allclose(t @ t, np.diag([1, 1j]), atol=1e-15)
    for m in (h, x, y, t):
        np.testing.assert_allclose(m.conj().T @ m, I2, atol=1e-15)


# ---------------------------------------------------------------- O1

@pytest.mark.parametrize("n,count,seed", [(1, 12, 1), (3, 40, 2), (5, 80, 3), (8, 120, 4)])
def test_full_state_matches_brute_force_unitaries(oracle_lib, n, count, seed):
    gates = _random_gate_list(n, count, seed)
    np.testing.assert_allclose(oracle.full_state(n, gates), _brute_state(n, gates), atol=1e-13)


def test_full_state_grid_circuit_matches_brute_force(oracle_lib):
    gates = grid_circuit(2, 4, 12, seed=7)
    np.testing.assert_allclose(oracle.full_state(8, gates), _brute_state(8, gates), atol=1e-13)


def test_h_layer_gives_uniform_state(oracle_lib):
    n = 12
    gates = grid_circuit(3, 4, 8, seed=1)[:n]        # cycle 0 only
    assert all(int(g["kind"]) == H for g in gates)
    psi = oracle.full_state(n, gates)
    np.testing.assert_allclose(psi, np.full(1 << n, 2.0 ** (-n / 2)), atol=1e-15)


def test_full_state_norm(oracle_lib):
    gates = grid_circuit(4, 5, 24, seed=11)
    psi = oracle.full_state(20, gates)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12


# ---------------------------------------------------------------- O2

def _cut_circuit(rows, cols, depth, seed, cut):
    gates = grid_circuit(rows, cols, depth, seed)
    mask = column_cut_mask(rows, cols, cut[1]) if cut[0] == "col" else row_cut_mask(rows, cols, cut[1])
    return gates, mask


def test_cz_split_two_qubits(oracle_lib):
    """P0 (x) I + P1 (x) Z = diag(1,1,1,-1): both paths of one crossing CZ sum to CZ."""
    rng = np.random.default_rng(5)
    gates = np.array([(H, 0, 0, 0, 0), (H, 0, 0, 1, 0), (XH, 0, 1, 0, 0), (YH, 0, 1, 1, 0),
                      (CZ, 0, 2, 0, 1), (T, 0, 3, 0, 0), (XH, 0, 3, 1, 0), (H, 0, 4, 0, 0),
                      (H, 0, 4, 1, 0)], dtype=GATE_DTYPE)
    del rng
    bits = np.arange(4, dtype=np.uint64)
    amps = oracle.path_sum(2, gates, 0b01, [0, 1], bits)
    np.testing.assert_allclose(amps, _brute_state(2, gates), atol=1e-15)
    # and the split itself, written with the two projectors
    P0, P1 = np.diag([1, 0]).astype(complex), np.diag([0, 1]).astype(complex)
    split = np.kron(I2, P0) + np.kron(PZ, P1)      # qubit 0 (block A) is the low bit
    np.testing.assert_allclose(split, _cz_full(2, 0, 1), atol=0)


@pytest.mark.parametrize("rows,cols,depth,cut", [(4, 4, 16, ("col", 2)), (4, 5, 16, ("col", 2)),
                                                  (5, 4, 12, ("row", 2)), (3, 5, 20, ("col", 3))])
def test_all_paths_equal_full_state(oracle_lib, rows, cols, depth, cut):
    n = rows * cols
    gates, mask = _cut_circuit(rows, cols, depth, 100 + n, cut)
    k = oracle.num_cut(n, gates, mask)
    psi = oracle.full_state(n, gates)
    bits = random_bitstrings(n, 512, 9)
    amps = oracle.path_sum(n, gates, mask, np.arange(1 << k, dtype=np.uint64), bits)
    ref = psi[bits.astype(np.int64)]
    assert np.linalg.norm(amps - ref) <= 1e-12 * np.linalg.norm(ref)


def test_no_crossing_gate_is_a_product_state(oracle_lib):
    """k = 0 (depth 1, the cycle-1 layout has no edge across the cut)."""
    gates, mask = _cut_circuit(4, 4, 1, 3, ("row", 2))  # cycle 1 = vertical V(0,0): rows 0-1, 2-3
    assert oracle.num_cut(16, gates, mask) == 0
    bits = random_bitstrings(16, 300, 4)
    amps = oracle.path_sum(16, gates, mask, [0], bits)
    np.testing.assert_allclose(amps, oracle.full_state(16, gates)[bits.astype(np.int64)], atol=1e-15)


def test_single_path_term_matches_full_space_construction(oracle_lib):
    """One path = the circuit with each crossing CZ j replaced by P_s (x) Z^s, s = bit (k-1-j)."""
    rows, cols, depth = 2, 4, 16
    n = rows * cols
    gates, mask = _cut_circuit(rows, cols, depth, 21, ("col", 2))
    cut = list(oracle.cut_gates(n, gates, mask))
    k = len(cut)
    assert k == 4
    P = [np.diag([1, 0]).astype(complex), np.diag([0, 1]).astype(complex)]
    bits = np.arange(1 << n, dtype=np.uint64)
    for path in (0, 1, 5, 10, 15):
        psi = np.zeros(1 << n, dtype=complex)
        psi[0] = 1
        for gi, g in enumerate(gates):
            if gi in cut:
                j = cut.index(gi)
                s = (path >> (k - 1 - j)) & 1
                a, b = int(g["q0"]), int(g["q1"])
                if not (mask >> a) & 1:
                    a, b = b, a
                psi = _op_on(n, a, P[s]) @ psi
                if s:
                    psi = _op_on(n, b, PZ) @ psi
            elif g["kind"] == CZ:
                psi = _cz_full(n, int(g["q0"]), int(g["q1"])) @ psi
            else:
                psi = _op_on(n, int(g["q0"]), _reference_matrix(int(g["kind"]))) @ psi
        amps = oracle.path_sum(n, gates, mask, [path], bits)
        np.testing.assert_allclose(amps, psi, atol=1e-14)


def test_block_norms(oracle_lib):
    """||psiB_p|| = 1 for every path; sum over all paths of ||psiA_p||^2 = 1 (P0 + P1 = I)."""
    gates, mask = _cut_circuit(4, 4, 16, 1001, ("col", 2))
    k = oracle.num_cut(16, gates, mask)
    _, na, nb = oracle.path_sum(16, gates, mask, np.arange(1 << k, dtype=np.uint64),
                                np.zeros(1, dtype=np.uint64), norms=True)
    np.testing.assert_allclose(nb, 1.0, atol=1e-13)
    assert abs(na.sum() - 1.0) < 1e-12
    # sibling paths (last bit 0/1) split their parent's norm: ||u||^2 = ||P0 u||^2 + ||P1 u||^2
    assert np.all(na >= -1e-15)


def test_partition_additivity(oracle_lib):
    gates, mask = _cut_circuit(4, 5, 16, 77, ("col", 2))
    k = oracle.num_cut(20, gates, mask)
    bits = random_bitstrings(20, 256, 3)
    rng = np.random.default_rng(0)
    ids = rng.permutation(1 << k).astype(np.uint64)
    s1, s2 = np.sort(ids[:300]), np.sort(ids[300:700])
    a1 = oracle.path_sum(20, gates, mask, s1, bits)
    a2 = oracle.path_sum(20, gates, mask, s2, bits)
    a12 = oracle.path_sum(20, gates, mask, np.concatenate([s1, s2]), bits)
    np.testing.assert_allclose(a1 + a2, a12, atol=1e-16, rtol=1e-12)


# ---------------------------------------------------------------- paper numbers

def test_crossing_counts_printed_in_logs(oracle_lib):
    gold = json.load(open(GOLDEN))
    for e in gold["crossing_cz_counts"]:
        gates, mask = _cut_circuit(e["rows"], e["cols"], e["depth"], 5, tuple(e["cut"]))
        assert oracle.num_cut(e["rows"] * e["cols"], gates, mask) == e["k"], e["cite"]


def test_path_counts_printed_in_logs(oracle_lib):
    gold = json.load(open(GOLDEN))
    for e in gold["path_counts"]:
        if "f" in e:
            f = e["f"]
        elif "f_den" in e:
            f = e["f_num"] / e["f_den"]
        else:
            f = 2.0 ** e["f_pow2"]
        assert oracle.num_paths(e["prefix_bits"], f) == e["count"], e["cite"]


def test_projector_zeros_only_in_block_a(oracle_lib):
    """Zeros appear only in the block carrying the projectors (cf. the zero counts in Appendix G)."""
    gates, mask = _cut_circuit(4, 4, 6, 8, ("col", 2))
    # evolve to just after the first crossing layer: truncate the gate list there
    cut = list(oracle.cut_gates(16, gates, mask))
    last = max(cut[:2]) + 1
    sub = gates[:last]
    bitsA = np.array([oracle_x for oracle_x in range(1 << 16)], dtype=np.uint64)
    amps = oracle.path_sum(16, sub, mask, [0], bitsA)
    # with s = 0 on both crossing CZs, A's endpoint qubits are forced to 0 -> amplitudes with
    # either endpoint bit set vanish; B is untouched by projectors
    a_ends = [int(sub[i]["q0"]) if (mask >> int(sub[i]["q0"])) & 1 else int(sub[i]["q1"]) for i in cut[:2]]
    forced = sum(1 << q for q in a_ends)
    nz = np.abs(amps) > 0
    assert not np.any(nz[(np.arange(1 << 16) & forced) != 0])
    assert np.all(nz[(np.arange(1 << 16) & forced) == 0])


# ---------------------------------------------------------------- statistics

def _t_rich_circuit(rows, cols, depth, seed):
    """A grid circuit whose later one-qubit gates are T with probability 1/3.

    Section 1 describes X^1/2, Y^1/2 and T interspersed at random; the
    generator used for the benchmarks places T only as a qubit's first
    gate, which leaves too few non-Clifford gates for the far tail of the
    output distribution to follow Porter-Thomas.
    """
    gates = grid_circuit(rows, cols, depth, seed).copy()
    rng = np.random.default_rng(seed)
    for i in range(len(gates)):
        if gates[i]["kind"] in (XH, YH) and rng.random() < 1.0 / 3.0:
            gates[i]["kind"] = T
    return gates


def test_porter_thomas_statistics(oracle_lib):
    """Deep random circuits follow Porter-Thomas, N e^{-Np} (Section 4).

    Averaged over five 20-qubit circuits: N sum p^2 ~ 2N/(N+1) (the Haar
    second moment), P(Np > t) ~ e^-t, and the mass above 10/N ~ 11 e^-10
    (the paper's 5e-4 for M' = 10).  The far tail varies a lot between
    20-qubit circuits, hence the wide band on it.
    """
    gold = json.load(open(GOLDEN))["porter_thomas"]
    assert abs(gold["tail_mass_model"] - math.exp(-10) * 11) < 1e-6
    n = 20
    N = 1 << n
    m2, f1, f5, tail = [], [], [], []
    for seed in (4242, 1, 2, 3, 4):
        p = np.abs(oracle.full_state(n, _t_rich_circuit(4, 5, 40, seed))) ** 2
        m2.append(N * np.sum(p * p))
        f1.append((N * p > 1).mean() / math.exp(-1))
        f5.append((N * p > 5).mean() / math.exp(-5))
        tail.append(p[N * p > gold["tail_threshold"]].sum() / gold["tail_mass_model"])
    assert abs(np.mean(m2) - 2 * N / (N + 1)) < 0.04
    assert abs(np.mean(f1) - 1) < 0.02
    assert abs(np.mean(f5) - 1) < 0.1
    assert 0.7 < np.mean(tail) < 1.6


@pytest.mark.slow
def test_fidelity_tracks_fraction(oracle_lib):
    """Section 3, Eq. (fid): keeping a fraction f of the paths gives ||psi_a||^2 ~ f and fidelity ~ f."""
    rows, cols = 4, 5
    n = rows * cols
    gates, mask = _cut_circuit(rows, cols, 24, 555, ("col", 2))
    k = oracle.num_cut(n, gates, mask)
    full = oracle.full_state(n, gates)
    bits = np.arange(1 << n, dtype=np.uint64)
    f = 0.25
    norms, fids = [], []
    for seed in range(4):
        ids = oracle.sample_paths(k, f, 900 + seed)
        a = oracle.path_sum(n, gates, mask, ids, bits)
        na = np.vdot(a, a).real
        norms.append(na)
        fids.append(abs(np.vdot(full, a)) ** 2 / na)
    assert abs(np.mean(norms) / f - 1) < 0.15
    assert abs(np.mean(fids) / f - 1) < 0.15


# ---------------------------------------------------------------- path sampling

def test_sample_paths_distinct_sorted_in_range(oracle_lib):
    for k, f in [(10, 0.3), (20, 0.01), (28, 1e-4), (5, 1.0)]:
        ids = oracle.sample_paths(k, f, 17)
        assert ids.size == math.ceil(f * 2 ** k)
        assert np.all(np.diff(ids.astype(np.int64)) > 0)
        assert int(ids.max()) < 2 ** k
    np.testing.assert_array_equal(oracle.sample_paths(6, 1.0, 3), np.arange(64, dtype=np.uint64))


def test_sample_paths_uniform_inclusion(oracle_lib):
    """Floyd's algorithm includes each id with probability m/N (statistical check)."""
    k, f = 6, 0.25
    counts = np.zeros(64)
    trials = 3000
    for s in range(trials):
        counts[oracle.sample_paths(k, f, 10_000 + s).astype(np.int64)] += 1
    expect = trials * 16 / 64
    chi2 = np.sum((counts - expect) ** 2 / (expect * (1 - 16 / 64)))
    assert chi2 < 120     # 63 degrees of freedom; p ~ 1e-5 cut-off
