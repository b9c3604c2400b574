"""Write FP64 oracle amplitudes of the 7x8 block workload to tests/golden/grid7x8_d40_paths.npz.

Workload: the 7x8 grid (56 qubits), depth 1+40+1, vertical cut into two
28-qubit blocks (35 crossing CZs), the seeded live aligned block of 1024 path
ids the benchmark runs (workload.workload_block; Section 5 and Appendix H: the
56-qubit run with a 28+28 cut).  The oracle's O2 path sum evolves both 28-qubit blocks in FP64 (4 GiB
each) for every listed path, so only a few paths are stored:

* an aligned sub-block of 8 paths inside the block, at a seeded offset (it
  shares every path bit but the last three, so the last tree levels fan out);
  each of its paths is stored on its own, and the sub-block's sum is their sum
  in id order, which is the path sum of Section 2 over those ids;
* the block's last path id, whose low ten bits all differ from the sub-block's
  first id (a different branch at every level below the shared prefix);

each on the first 4096 of the workload's bitstrings.  Runs only the oracle and
the seeded input generator; about 6 minutes per path on 8 host cores.

    python tests/golden/make_grid7x8_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workload import CONFIGS, SplitMix64, grid_circuit, random_bitstrings, workload_block  # noqa: E402

OUT = os.path.join(HERE, "grid7x8_d40_paths.npz")
N_BITS = 4096
SUB_SEED = 4004          # seed of the sub-block offset inside the 1024-path block


def main():
    cfg = CONFIGS["grid7x8_d40"]
    gates = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed)
    mask = cfg.cut_mask()
    k = oracle.num_cut(cfg.n_qubits, gates, mask)
    begin, count = workload_block(cfg.name)
    sub = (SplitMix64(SUB_SEED).next() >> 57) * 8          # 0, 8, ..., 1016
    ids = [begin + sub + i for i in range(8)] + [begin + count - 1]
    bits = random_bitstrings(cfg.n_qubits, N_BITS, cfg.bits_seed)
    amps = np.zeros((len(ids), N_BITS), dtype=np.complex128)
    for i, p in enumerate(ids):
        t0 = time.time()
        amps[i] = oracle.path_sum(cfg.n_qubits, gates, mask, np.array([p], dtype=np.uint64), bits)
        print(f"path {i + 1}/{len(ids)} (id {p}): {time.time() - t0:.0f} s", flush=True)
    sub_sum = np.zeros(N_BITS, dtype=np.complex128)
    for i in range(8):
        sub_sum += amps[i]
    for i in range(len(ids)):
        assert np.abs(amps[i]).max() > 0, f"path {int(ids[i])} has a zero term"
    np.savez(OUT, k=np.int64(k), block_begin=np.uint64(begin), block_count=np.int64(count),
             ids=np.array(ids, dtype=np.uint64), bitstrings=bits, amps=amps, sub_block_sum=sub_sum,
             n_qubits=np.int64(cfg.n_qubits), mask_a=np.uint64(mask))
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
