"""Find the seeded 7x8 path block whose paths carry nonzero terms, with the FP64 oracle.

The 7x8 benchmark block is an aligned block of 1024 path ids whose index is drawn from
SplitMix64(path seed).  Many draws give blocks in which every path's block-A state is exactly
zero: the projectors of the crossing CZs (Section 2, Eq. (CZ)) multiply to zero when a qubit
keeps a value fixed by one path bit until another projector asks for a different one, either
directly (workload.equal_bit_pairs) or through chains of gates over several qubits.  This script
takes the draws in order, skips those that equal_bit_pairs already rules out, computes with
the oracle's path sum the block-A norm of the state the block's paths share before its own
crossing cycles (zero: every path of the block is zero), and then the block-A norms of the
block's first and last path; the first draw with both norms nonzero is printed (the value of
`block_draw` in the 7x8 workload configuration).

Only block A decides whether a term is zero (block B sees unitaries), so the oracle runs on the
circuit without block B's own gates: same crossing CZs (so the same path bits), same block-A
program, block B reduced to the crossing Z's.  Runs only the oracle and the input generator;
about 4 minutes per path on 8 host cores.

    python tests/golden/find_live_block.py [first_draw]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workload import CONFIGS, CZ, SplitMix64, equal_bit_pairs, grid_circuit, is_live  # noqa: E402


def main():
    cfg = CONFIGS["grid7x8_d40"]
    gates = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    mask = cfg.cut_mask()
    n = cfg.n_qubits
    in_a = lambda q: (mask >> int(q)) & 1
    crossing = np.array([int(g["kind"]) == CZ and in_a(g["q0"]) != in_a(g["q1"]) for g in gates])
    keep = np.array([bool(in_a(g["q0"])) for g in gates]) | crossing
    reduced = gates[keep]
    k = oracle.num_cut(n, gates, mask)
    assert oracle.num_cut(n, reduced, mask) == k
    pairs = equal_bit_pairs(gates, mask)
    hi = k - cfg.block_bits
    # cycle of the crossing gate that decides the block's highest low bit (path bit block_bits - 1)
    cut = oracle.cut_gates(n, gates, mask)
    first_low_cycle = int(gates[cut[k - cfg.block_bits]]["cycle"])
    first = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    rng = SplitMix64(cfg.path_seed)
    for draw in range(first + 64):
        b = rng.next() >> (64 - hi)
        if draw < first:
            continue
        begin = b << cfg.block_bits
        if not is_live(begin, pairs):
            print(f"draw {draw}: block {b} has unequal bit pairs", flush=True)
            continue
        # first the gates up to the block's first crossing cycle (their block-A state is shared by
        # the whole block): a zero there rules the block out at about 70% of the cost
        t0 = time.time()
        pre = reduced[reduced["cycle"] < first_low_cycle]
        kp = oracle.num_cut(n, pre, mask)
        _, npre, _ = oracle.path_sum(n, pre, mask, np.array([begin >> (k - kp)], dtype=np.uint64),
                                     np.zeros(1, dtype=np.uint64), norms=True)
        if not npre[0] > 0:
            print(f"draw {draw}: block {b}, shared prefix has block-A norm 0 ({time.time() - t0:.0f} s)", flush=True)
            continue
        ids = np.array([begin, begin + (1 << cfg.block_bits) - 1], dtype=np.uint64)
        _, na, _ = oracle.path_sum(n, reduced, mask, ids, np.zeros(1, dtype=np.uint64), norms=True)
        print(f"draw {draw}: block {b}, block-A norms {na.tolist()} ({time.time() - t0:.0f} s)", flush=True)
        if np.all(na > 0):
            print(f"block_draw = {draw}")
            return
    raise SystemExit("no block found")


if __name__ == "__main__":
    main()
