"""Hand-built circuits whose last tree level has the shapes the folded leaf gather handles.

Only gate lists (no arithmetic of the method): a random grid circuit without its closing H
layer, then one cycle of CZs crossing the column cut between columns 1 and 2 in every row (one
tree level with `rows` branch bits), then a tail of gates chosen so that the last level mixes
sqrt(X)/sqrt(Y)/H on branch qubits, T and CZ phases after them (one CZ reaching a qubit that only
diagonal gates touch), and branch qubits that no non-diagonal gate touches after the crossing.
"""
import numpy as np

from workload import CZ, GATE_DTYPE, H, T, XH, YH, grid_circuit


def crossing_tail_circuit(rows=4, depth=8, seed=5):
    cols = 4
    base = grid_circuit(rows, cols, depth, seed)
    gates = [tuple(g) for g in base if g["cycle"] <= depth]
    q = lambda r, c: r * cols + c
    c1, c2, c3, c4 = depth + 1, depth + 2, depth + 3, depth + 4
    for r in range(rows):
        gates.append((CZ, 0, c1, q(r, 1), q(r, 2)))      # crossing: block A = columns 0-1
    # block A: sqrt(X), then CZ to the non-branch qubit (0,0), then H on (0,1); H, T, H on (1,1);
    # H on (2,1); nothing after the crossing on (3,1)
    gates += [(XH, 0, c2, q(0, 1), 0), (H, 0, c2, q(1, 1), 0), (H, 0, c2, q(2, 1), 0)]
    gates += [(CZ, 0, c3, q(0, 1), q(0, 0)), (T, 0, c3, q(1, 1), 0)]
    gates += [(H, 0, c4, q(0, 1), 0), (H, 0, c4, q(1, 1), 0)]
    # block B: sqrt(Y), T, H on (0,2); H, then CZ to the non-branch qubit (1,3) on (1,2); only a
    # T (diagonal) on (2,2); nothing on (3,2)
    gates += [(YH, 0, c2, q(0, 2), 0), (H, 0, c2, q(1, 2), 0), (T, 0, c2, q(2, 2), 0)]
    gates += [(T, 0, c3, q(0, 2), 0), (CZ, 0, c3, q(1, 2), q(1, 3))]
    gates += [(H, 0, c4, q(0, 2), 0)]
    # the other qubits of columns 0 and 3 end with an H (not part of the last level)
    gates += [(H, 0, c4, q(r, 0), 0) for r in range(1, rows)]
    gates += [(H, 0, c4, q(r, 3), 0) for r in range(rows) if r != 1]
    mask_a = 0
    for r in range(rows):
        mask_a |= (1 << q(r, 0)) | (1 << q(r, 1))
    gates.sort(key=lambda g: g[2])           # stable: list order within a cycle is kept
    return rows, cols, np.array(gates, dtype=GATE_DTYPE), mask_a


def two_level_tail_circuit(depth=8, seed=5):
    """Two crossing cycles at the end on a 4 x 4 grid (cut between columns 1 and 2): rows 0-1
    cross first, rows 2-3 two cycles later.  Between and after them: non-diagonal gates on
    some branch qubits only, T and CZ phases (one CZ reaching a non-branch qubit on each side),
    and branch qubits that no non-diagonal gate touches afterwards; so the last two tree levels
    fold together (4 path bits)."""
    rows, cols = 4, 4
    base = grid_circuit(rows, cols, depth, seed)
    gates = [tuple(g) for g in base if g["cycle"] <= depth]
    q = lambda r, c: r * cols + c
    c1, c2, c3, c4, c5, c6 = (depth + i for i in range(1, 7))
    gates += [(CZ, 0, c1, q(0, 1), q(0, 2)), (CZ, 0, c1, q(1, 1), q(1, 2))]
    gates += [(XH, 0, c2, q(0, 1), 0), (H, 0, c2, q(1, 1), 0), (YH, 0, c2, q(0, 2), 0), (T, 0, c2, q(1, 2), 0)]
    gates += [(CZ, 0, c3, q(0, 1), q(0, 0)), (CZ, 0, c3, q(2, 1), q(2, 2)), (CZ, 0, c3, q(3, 1), q(3, 2))]
    gates += [(H, 0, c4, q(0, 1), 0), (T, 0, c4, q(2, 1), 0), (H, 0, c4, q(3, 1), 0), (H, 0, c4, q(0, 2), 0),
              (YH, 0, c4, q(2, 2), 0)]
    gates += [(CZ, 0, c5, q(2, 2), q(2, 3)), (CZ, 0, c5, q(3, 2), q(3, 3))]
    gates += [(H, 0, c6, q(2, 2), 0)]
    gates += [(H, 0, c6, q(r, 0), 0) for r in (1, 2, 3)] + [(H, 0, c6, q(r, 3), 0) for r in (0, 1)]
    gates.sort(key=lambda g: g[2])
    mask_a = 0
    for r in range(rows):
        mask_a |= (1 << q(r, 0)) | (1 << q(r, 1))
    return rows, cols, np.array(gates, dtype=GATE_DTYPE), mask_a


def iswap_tail_circuit(drop_final_h=()):
    """2 x 4 grid, cut between columns 1 and 2, whose last two cycles each hold one crossing
    iSWAP (rows 0 and 1) after in-block iSWAPs and one-qubit gates: both trailing tree levels
    can be folded (two iSWAP gates).  Qubits in drop_final_h get no closing H, so their
    branch operators are not followed by a non-diagonal gate."""
    from workload import GATE_DTYPE, H, XH, YH, T, ISWAP, column_cut_mask
    g = [(H, 0, 0, q, 0) for q in range(8)]
    g += [(ISWAP, 0, 1, 0, 4), (ISWAP, 0, 1, 3, 7)] + [(T, 0, 1, q, 0) for q in (1, 2, 5, 6)]
    g += [(ISWAP, 0, 2, 1, 2), (XH, 0, 2, 0, 0), (YH, 0, 2, 4, 0), (T, 0, 2, 3, 0)]
    g += [(ISWAP, 0, 3, 5, 6), (T, 0, 3, 0, 0), (XH, 0, 3, 7, 0)]
    g += [(H, 0, 4, q, 0) for q in range(8) if q not in drop_final_h]
    return 2, 4, np.array(g, dtype=GATE_DTYPE), column_cut_mask(2, 4, 2)
