"""Pin of the crossing-gate order, i.e. which path bits decide which crossing gate.

Reading (Section 2: paths that share an x_p-bit prefix share their evolution up
to the checkpoint; Eq. (CZ) and Eq. (4way) give each crossing gate's terms):
the crossing gates are ordered by (clock cycle, smaller qubit id) and the
earliest takes the most significant path bits -- one bit for a CZ, two for an
iSWAP (term r = 2i + j, i the higher bit) -- so an aligned block of path ids is
a shared prefix.

The circuit below is written by hand so that list order and this order differ:
inside a cycle the crossing gates are listed with the larger smaller-qubit
first, one gate names its block-B endpoint first, and CZs and iSWAPs mix.  The
expected assignment is written out literally, and every single path is checked
against a full-space construction that reads the assignment from that literal
table (never from the oracle's own ordering).  A wrong sort key (list order,
larger qubit, q0) or cycles taken in reverse assigns some bits to other gates,
which changes single-path amplitudes by O(1).
"""
import numpy as np

import oracle
from workload import CZ, GATE_DTYPE, ISWAP

H, XH, YH, T = 0, 1, 2, 3

# 2 x 4 grid, qubit id r*4 + c:   0 1 2 3 / 4 5 6 7.  Block A = {0, 1, 2, 4}, block B = {3, 5, 6, 7}
# (a stepped cut, so that crossing gates can be ordered differently by their smaller and their
# larger qubit).  Crossing edges: 2-3, 1-5, 4-5, 2-6.
N = 8
MASK_A = (1 << 0) | (1 << 1) | (1 << 2) | (1 << 4)

# (cycle, kind, q0, q1); q1 unused for one-qubit gates.  List index in the comments.
GATES = [(0, H, q, 0) for q in range(N)] + [                  # 0..7
    (1, CZ, 2, 3),        # 8   crossing, smaller qubit 2, larger 3 (listed first)
    (1, ISWAP, 5, 1),     # 9   crossing, smaller qubit 1, larger 5 (block-B endpoint listed first)
    (1, CZ, 6, 7),        # 10  inside B
    (1, CZ, 0, 4),        # 11  inside A
    (2, XH, 1, 0), (2, YH, 2, 0), (2, T, 5, 0), (2, XH, 6, 0), (2, H, 0, 0), (2, YH, 7, 0),   # 12..17
    (3, CZ, 4, 5),        # 18  crossing, smaller qubit 4, larger 5 (listed first)
    (3, CZ, 6, 2),        # 19  crossing, smaller qubit 2, larger 6 (block-B endpoint listed first)
    (3, CZ, 0, 1),        # 20  inside A
    (3, CZ, 3, 7),        # 21  inside B
    (4, YH, 1, 0), (4, T, 2, 0), (4, XH, 5, 0), (4, YH, 6, 0), (4, T, 4, 0),               # 22..26
    (5, ISWAP, 3, 2),     # 27  crossing, the last one (block-B endpoint listed first)
    (5, ISWAP, 0, 4),     # 28  inside A
    (5, CZ, 6, 7),        # 29  inside B
    (6, XH, 2, 0), (6, T, 1, 0), (6, YH, 3, 0),                                              # 30..32
] + [(7, H, q, 0) for q in range(N)]                            # 33..40

# Each crossing gate with its block-A and block-B endpoints and the path bits it takes (high
# bit first), in the order of the reading.
EXPECTED = [
    (9, ISWAP, 1, 5, (6, 5)),    # cycle 1, smaller qubit 1
    (8, CZ, 2, 3, (4,)),         # cycle 1, smaller qubit 2
    (19, CZ, 2, 6, (3,)),        # cycle 3, smaller qubit 2
    (18, CZ, 4, 5, (2,)),        # cycle 3, smaller qubit 4
    (27, ISWAP, 2, 3, (1, 0)),   # cycle 5
]
K = 7


def _gates():
    rec = [(kind, 0, cyc, q0, q1) for cyc, kind, q0, q1 in GATES]
    return np.array(rec, dtype=GATE_DTYPE)


def _one_qubit(kind):
    s = 1 / np.sqrt(2)
    if kind == H:
        return np.array([[s, s], [s, -s]], dtype=complex)
    if kind == XH:
        return 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]])
    if kind == YH:
        return 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]])
    return np.diag([1, np.exp(1j * np.pi / 4)])


ISWAP_M = np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]], dtype=complex)
CZ_M = np.diag([1, 1, 1, -1]).astype(complex)


def _apply1(psi, q, m):
    out = psi.copy()
    for i in range(1 << N):
        if not (i >> q) & 1:
            j = i | (1 << q)
            out[i] = m[0, 0] * psi[i] + m[0, 1] * psi[j]
            out[j] = m[1, 0] * psi[i] + m[1, 1] * psi[j]
    return out


def _apply2(psi, a, b, m4):
    """4x4 m4 in the basis 2 x_a + x_b."""
    out = np.zeros_like(psi)
    for i in range(1 << N):
        col = 2 * ((i >> a) & 1) + ((i >> b) & 1)
        base = i & ~((1 << a) | (1 << b))
        for row in range(4):
            out[base | ((row >> 1) << a) | ((row & 1) << b)] += m4[row, col] * psi[i]
    return out


def _term(kind, r):
    """Eq. (4way) term r = 2i + j as a 4x4 matrix in the basis 2 x_A + x_B: |i><j| (x) G_ij
    (for a CZ only r = 0 and r = 3 occur: P0 (x) I and P1 (x) Z, Eq. (CZ))."""
    g = CZ_M if kind == CZ else ISWAP_M
    i, j = r >> 1, r & 1
    e = np.zeros((2, 2), complex)
    e[i, j] = 1
    return np.kron(e, g[2 * i:2 * i + 2, 2 * j:2 * j + 2])


def _single_path(path):
    table = {gi: (kind, a, b, bits) for gi, kind, a, b, bits in EXPECTED}
    psi = np.zeros(1 << N, complex)
    psi[0] = 1
    for gi, (cyc, kind, q0, q1) in enumerate(GATES):
        if gi in table:
            kind_t, a, b, bits = table[gi]
            assert kind_t == kind
            v = 0
            for bit in bits:
                v = 2 * v + ((path >> bit) & 1)
            r = 3 * v if kind == CZ else v
            psi = _apply2(psi, a, b, _term(kind, r))
        elif kind == CZ:
            psi = _apply2(psi, q0, q1, CZ_M)
        elif kind == ISWAP:
            psi = _apply2(psi, q0, q1, ISWAP_M)
        else:
            psi = _apply1(psi, q0, _one_qubit(kind))
    return psi


def test_expected_table_is_consistent():
    """The literal table covers each crossing gate once and the path bits 0..K-1 once."""
    g = GATES
    crossing = [i for i, (c, kd, a, b) in enumerate(g)
                if kd in (CZ, ISWAP) and ((MASK_A >> a) & 1) != ((MASK_A >> b) & 1)]
    assert sorted(e[0] for e in EXPECTED) == crossing
    assert sorted(b for e in EXPECTED for b in e[4]) == list(range(K))
    for gi, kind, a, b, _ in EXPECTED:
        assert g[gi][1] == kind and {a, b} == {g[gi][2], g[gi][3]}
        assert (MASK_A >> a) & 1 and not (MASK_A >> b) & 1


def test_path_bit_count():
    assert oracle.num_cut(N, _gates(), MASK_A) == K


def test_every_single_path_matches_literal_bit_assignment(oracle_lib):
    gates = _gates()
    bits = np.arange(1 << N, dtype=np.uint64)
    for path in range(1 << K):
        got = oracle.path_sum(N, gates, MASK_A, [path], bits)
        np.testing.assert_allclose(got, _single_path(path), atol=1e-14, err_msg=f"path {path}")


def test_literal_assignment_differs_from_wrong_orders():
    """The circuit separates the reading from the plausible mistakes: ordering by list position,
    by larger qubit, by the first-listed qubit, or cycles in reverse gives a different gate for some path bit, so the
    single-path check above would fail for them."""
    cross = [(gi, GATES[gi]) for gi, *_ in EXPECTED]
    right = [gi for gi, *_ in EXPECTED]
    by_list = sorted(gi for gi, _ in cross)
    by_larger = [gi for gi, _ in sorted(cross, key=lambda t: (t[1][0], max(t[1][2], t[1][3])))]
    by_q0 = [gi for gi, _ in sorted(cross, key=lambda t: (t[1][0], t[1][2]))]
    reversed_cycles = [gi for gi, _ in sorted(cross, key=lambda t: (-t[1][0], min(t[1][2], t[1][3])))]
    for wrong in (by_list, by_larger, by_q0, reversed_cycles):
        assert wrong != right
