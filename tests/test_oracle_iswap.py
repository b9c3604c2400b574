"""Pins of the oracle's two-qubit gate support (section on harder benchmarks through two-qubit
gates): the iSWAP matrix from its operator Schmidt form, Eq. (iSWAP2); the four-term split of a
crossing gate, Eq. (4way) and Eq. (iSWAP1); full states against brute-force unitaries; the path
sum over all paths against the full state; single-path terms against a full-space construction."""
import numpy as np
import pytest

import oracle
from test_oracle_pins import I2, PX, PY, PZ, _op_on, _reference_matrix
from workload import CZ, GATE_DTYPE, ISWAP, column_cut_mask, grid_circuit, random_bitstrings, row_cut_mask

KET0BRA1 = np.array([[0, 1], [0, 0]], dtype=complex)     # |0><1|
KET1BRA0 = np.array([[0, 0], [1, 0]], dtype=complex)     # |1><0|
P0 = np.diag([1, 0]).astype(complex)
P1 = np.diag([0, 1]).astype(complex)


def _iswap_reference():
    """Eq. (iSWAP2): 2 iSWAP = I(x)I + i X(x)X + i Y(x)Y + Z(x)Z (first factor = first qubit)."""
    return (np.kron(I2, I2) + 1j * np.kron(PX, PX) + 1j * np.kron(PY, PY) + np.kron(PZ, PZ)) / 2


def test_iswap_matrix_matches_schmidt_form():
    g = oracle.gate_matrix2(ISWAP)
    np.testing.assert_allclose(g, _iswap_reference(), atol=1e-15)
    np.testing.assert_allclose(g @ g.conj().T, np.eye(4), atol=1e-15)


def test_four_term_split():
    """Eq. (4way): G = sum_{i,j} |i><j| (x) G_ij; for iSWAP the terms are Eq. (iSWAP1); for CZ
    only P0 (x) I and P1 (x) Z are non-zero (the Section 2 split)."""
    want = {0: (P0, P0), 1: (KET0BRA1, 1j * KET1BRA0), 2: (KET1BRA0, 1j * KET0BRA1), 3: (P1, P1)}
    total = np.zeros((4, 4), complex)
    for r in range(4):
        ea, gb = oracle.branch_ops(ISWAP, r)
        np.testing.assert_allclose(ea, want[r][0], atol=0)
        np.testing.assert_allclose(gb, want[r][1], atol=0)
        total += np.kron(ea, gb)
    np.testing.assert_allclose(total, _iswap_reference(), atol=1e-15)
    cz = np.diag([1, 1, 1, -1]).astype(complex)
    np.testing.assert_allclose(sum(np.kron(*oracle.branch_ops(CZ, r)) for r in range(4)), cz, atol=0)
    np.testing.assert_allclose(oracle.branch_ops(CZ, 0)[1], I2, atol=0)
    np.testing.assert_allclose(oracle.branch_ops(CZ, 3)[1], PZ, atol=0)
    assert not oracle.branch_ops(CZ, 1)[1].any() and not oracle.branch_ops(CZ, 2)[1].any()


def _two_qubit_full(n, a, b, m4):
    """Full 2^n operator applying 4x4 m4 to qubits (a, b), a as the first (high) factor."""
    dim = 1 << n
    out = np.zeros((dim, dim), complex)
    for col in range(dim):
        ca, cb = (col >> a) & 1, (col >> b) & 1
        for r in range(4):
            ra, rb = r >> 1, r & 1
            row = (col & ~((1 << a) | (1 << b))) | (ra << a) | (rb << b)
            out[row, col] += m4[2 * ra + rb, 2 * ca + cb]
    return out


def _brute(n, gates, crossing_terms=None):
    psi = np.zeros(1 << n, complex)
    psi[0] = 1
    for gi, g in enumerate(gates):
        a, b = int(g["q0"]), int(g["q1"])
        if crossing_terms and gi in crossing_terms:
            psi = _two_qubit_full(n, *crossing_terms[gi]) @ psi
        elif g["kind"] == ISWAP:
            psi = _two_qubit_full(n, a, b, _iswap_reference()) @ psi
        elif g["kind"] == CZ:
            psi = _two_qubit_full(n, a, b, np.diag([1, 1, 1, -1]).astype(complex)) @ psi
        else:
            psi = _op_on(n, a, _reference_matrix(int(g["kind"]))) @ psi
    return psi


@pytest.mark.parametrize("n,count,seed", [(2, 12, 1), (5, 40, 2), (8, 60, 3)])
def test_full_state_with_iswap_matches_brute_force(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.choice([0, 1, 2, 3, CZ, ISWAP]))
        if kind in (CZ, ISWAP):
            a, b = rng.choice(n, size=2, replace=False)
            out.append((kind, 0, 0, int(a), int(b)))
        else:
            out.append((kind, 0, 0, int(rng.integers(0, n)), 0))
    g = np.array(out, dtype=GATE_DTYPE)
    np.testing.assert_allclose(oracle.full_state(n, g), _brute(n, g), atol=1e-13)


@pytest.mark.parametrize("rows,cols,depth,cut", [(3, 3, 6, ("col", 1)), (3, 4, 6, ("col", 2)),
                                                 (4, 4, 5, ("row", 2)), (2, 5, 9, ("col", 2))])
def test_iswap_path_sum_equals_full_state(rows, cols, depth, cut):
    """Every CZ replaced by an iSWAP: each crossing gate takes two path bits (branching factor
    four), and the sum over all 4^(crossing gates) paths is the full state."""
    n = rows * cols
    g = grid_circuit(rows, cols, depth, 31, two_qubit=ISWAP)
    gc = grid_circuit(rows, cols, depth, 31)
    mask = column_cut_mask(rows, cols, cut[1]) if cut[0] == "col" else row_cut_mask(rows, cols, cut[1])
    k = oracle.num_cut(n, g, mask)
    assert k == 2 * oracle.num_cut(n, gc, mask) == 2 * len(oracle.cut_gates(n, g, mask))
    assert k <= 14
    bits = np.arange(1 << n, dtype=np.uint64)
    amps = oracle.path_sum(n, g, mask, np.arange(1 << k, dtype=np.uint64), bits)
    np.testing.assert_allclose(amps, oracle.full_state(n, g), atol=1e-13)


def test_single_iswap_path_matches_full_space_construction():
    """One path = the circuit with crossing gate j replaced by |i><j| (x) G_ij on (block-A
    endpoint, block-B endpoint), the term r = 2i + j read from the path id: the first crossing
    gate's two bits are the highest."""
    rows, cols, depth = 2, 4, 9
    n = rows * cols
    g = grid_circuit(rows, cols, depth, 21, two_qubit=ISWAP)
    mask = column_cut_mask(rows, cols, 2)
    cut = list(oracle.cut_gates(n, g, mask))
    k = oracle.num_cut(n, g, mask)
    assert k == 2 * len(cut) and 4 <= k <= 12
    G = _iswap_reference()
    bits = np.arange(1 << n, dtype=np.uint64)
    rng = np.random.default_rng(5)
    for path in [0, (1 << k) - 1] + [int(x) for x in rng.integers(0, 1 << k, 6)]:
        terms = {}
        for j, gi in enumerate(cut):
            r = (path >> (k - 2 * (j + 1))) & 3
            i, jj = r >> 1, r & 1
            a, b = int(g[gi]["q0"]), int(g[gi]["q1"])
            if not (mask >> a) & 1:
                a, b = b, a
            e = np.zeros((2, 2), complex)
            e[i, jj] = 1
            blk = G[2 * i:2 * i + 2, 2 * jj:2 * jj + 2]
            terms[gi] = (a, b, np.kron(e, blk))
        want = _brute(n, g, terms)
        got = oracle.path_sum(n, g, mask, [path], bits)
        np.testing.assert_allclose(got, want, atol=1e-14)


def test_mixed_cz_and_iswap_bits():
    """A circuit mixing crossing CZs (one bit) and crossing iSWAPs (two bits) still sums to the
    full state over all paths."""
    rows, cols, depth = 3, 3, 8
    n = rows * cols
    g = grid_circuit(rows, cols, depth, 7)
    g["kind"][np.flatnonzero(g["kind"] == CZ)[::2]] = ISWAP
    mask = column_cut_mask(rows, cols, 1)
    k = oracle.num_cut(n, g, mask)
    n_is = sum(1 for gi in oracle.cut_gates(n, g, mask) if g[gi]["kind"] == ISWAP)
    assert k == len(oracle.cut_gates(n, g, mask)) + n_is and n_is > 0
    bits = random_bitstrings(n, 300, 3)
    amps = oracle.path_sum(n, g, mask, np.arange(1 << k, dtype=np.uint64), bits)
    np.testing.assert_allclose(amps, oracle.full_state(n, g)[bits.astype(np.int64)], atol=1e-13)
