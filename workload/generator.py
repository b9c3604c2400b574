"""Seeded random grid circuits, bitstring sets and path blocks.

Conventions (fixed here because the paper leaves them open):

* Qubit id on an R x C grid is ``r*C + c`` (row-major, as in the qubit-grid
  printouts of the paper's simulation logs, Appendix D).
* Gate kinds: 0 = H, 1 = X^1/2, 2 = Y^1/2, 3 = T, 4 = CZ (Section 1 names
  this gate set), 5 = iSWAP (the harder variant of Section 7).  Records are 8 bytes: kind u8, pad u8, cycle u16, q0 u16,
  q1 u16 (q1 unused for one-qubit gates).
* Cycle 0 is a layer of H on every qubit.  Cycles 1..D each apply one of
  eight CZ layouts; layout (c mod 8) is chosen so that every nearest-
  neighbour edge appears once in any 8 consecutive cycles and horizontal and
  vertical layouts alternate (Section 1; Section 6, second bullet list).
* One-qubit gates: a qubit that had a CZ in cycle c-1 and has none in cycle
  c receives one gate in cycle c: T if it has had no one-qubit gate yet
  (besides the opening H), otherwise X^1/2 or Y^1/2, different from its
  previous one; after a T the choice is uniform.  Draws are made in
  ascending qubit order within a cycle, one SplitMix64 draw per uniform
  choice (top bit 0 -> X^1/2, 1 -> Y^1/2).
* Cycle D+1 is a layer of H on every qubit.
* Within a cycle the list holds the CZs first (in layout order) and then the
  one-qubit gates in ascending qubit order; the two sets touch disjoint
  qubits, so the order inside a cycle does not change the circuit.

Random numbers come from SplitMix64 (Steele, Lea and Flood, 2014): the state
advances by 0x9E3779B97F4A7C15 and each output is the state passed through
the published two-multiply finaliser.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

H, XH, YH, T, CZ, ISWAP = 0, 1, 2, 3, 4, 5
GATE_NAMES = {H: "H", XH: "X^1/2", YH: "Y^1/2", T: "T", CZ: "CZ", ISWAP: "iSWAP"}

GATE_DTYPE = np.dtype([("kind", np.uint8), ("pad", np.uint8), ("cycle", np.uint16),
                       ("q0", np.uint16), ("q1", np.uint16)])
assert GATE_DTYPE.itemsize == 8

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1


class SplitMix64:
    """Sequential SplitMix64 stream (scalar, exact 64-bit arithmetic)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * _M1) & _MASK64
        z = ((z ^ (z >> 27)) * _M2) & _MASK64
        return z ^ (z >> 31)


def splitmix64_array(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the stream seeded with ``seed``."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + idx * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return z


# CZ layout table: layout index -> (orientation, a, b).
#   "H"(a, b): edges (r, c)-(r, c+1) with c = a (mod 2) and r = b (mod 2)
#   "V"(a, b): edges (r, c)-(r+1, c) with r = a (mod 2) and c = b (mod 2)
_LAYOUTS = [("H", 0, 0), ("V", 0, 0), ("H", 1, 1), ("V", 1, 1),
            ("H", 0, 1), ("V", 0, 1), ("H", 1, 0), ("V", 1, 0)]


def cz_pattern_edges(rows: int, cols: int, pattern: int):
    """Edges (q0, q1), q0 < q1, of CZ layout ``pattern`` (0..7)."""
    orient, a, b = _LAYOUTS[pattern % 8]
    edges = []
    if orient == "H":
        for r in range(rows):
            if r % 2 != b:
                continue
            for c in range(cols - 1):
                if c % 2 == a:
                    edges.append((r * cols + c, r * cols + c + 1))
    else:
        for r in range(rows - 1):
            if r % 2 != a:
                continue
            for c in range(cols):
                if c % 2 == b:
                    edges.append((r * cols + c, (r + 1) * cols + c))
    return edges


def grid_circuit(rows: int, cols: int, depth: int, seed: int, two_qubit: int = CZ) -> np.ndarray:
    """Random circuit of depth 1+depth+1 on a rows x cols grid (see module doc).

    two_qubit = ISWAP gives the harder benchmark variant of the section on two-qubit gates:
    every CZ of the same circuit replaced by an iSWAP (same layouts, same one-qubit gates)."""
    n = rows * cols
    if n > 64:
        raise ValueError("at most 64 qubits")
    rng = SplitMix64(seed)
    gates = []
    for q in range(n):
        gates.append((H, 0, 0, q, 0))
    last = [None] * n          # last one-qubit gate kind after the opening H
    prev_cz = [False] * n
    for c in range(1, depth + 1):
        edges = cz_pattern_edges(rows, cols, c % 8)
        cur_cz = [False] * n
        for (a, b) in edges:
            gates.append((two_qubit, 0, c, a, b))
            cur_cz[a] = cur_cz[b] = True
        for q in range(n):
            if prev_cz[q] and not cur_cz[q]:
                if last[q] is None:
                    g = T
                elif last[q] == T:
                    g = XH if (rng.next() >> 63) == 0 else YH
                else:
                    g = YH if last[q] == XH else XH
                gates.append((g, 0, c, q, 0))
                last[q] = g
        prev_cz = cur_cz
    for q in range(n):
        gates.append((H, 0, depth + 1, q, 0))
    return np.array(gates, dtype=GATE_DTYPE)


def random_bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct uniform n-qubit bitstrings (bit q = qubit q), as uint64.

    Draw i is output i of SplitMix64(seed) masked to n bits; repeats are
    skipped and drawing continues until ``count`` distinct values are found.
    """
    if n_qubits < 64 and count > (1 << n_qubits):
        raise ValueError("more distinct bitstrings requested than exist")
    mask = np.uint64(_MASK64 if n_qubits >= 64 else (1 << n_qubits) - 1)
    out = np.empty(0, dtype=np.uint64)
    seen = set()
    start = 0
    while out.size < count:
        chunk = max(1024, 2 * (count - out.size))
        draws = splitmix64_array(seed, chunk, start) & mask
        start += chunk
        keep = []
        for v in draws.tolist():
            if v not in seen:
                seen.add(v)
                keep.append(v)
                if out.size + len(keep) == count:
                    break
        out = np.concatenate([out, np.array(keep, dtype=np.uint64)])
    return out


def path_block(k: int, block_bits: int, seed: int):
    """A seeded aligned block of 2^block_bits path ids: returns (begin, count)."""
    if block_bits > k:
        raise ValueError("block larger than the path space")
    hi_bits = k - block_bits
    b = 0 if hi_bits == 0 else SplitMix64(seed).next() >> (64 - hi_bits)
    return b << block_bits, 1 << block_bits


def equal_bit_pairs(gates: np.ndarray, mask_a: int):
    """Pairs (u, v) of path bits that every path with a nonzero term sets equal, for circuits whose
    crossing two-qubit gates are all CZs (an empty list otherwise).

    Path bits follow the crossing CZs in (cycle, smaller qubit) order, the first CZ taking the
    highest bit (k-1).  A crossing CZ's path bit s puts the projector onto |s> on its block-A
    endpoint (Section 2, Eq. (CZ)).  When a block-A qubit meets two crossing CZs with only
    diagonal gates (T, CZ) on it in between, the two projectors multiply, and the path's term is
    zero unless both bits are equal: such paths are skipped (the paper's zero blocks, Section 2),
    and a benchmark path block must avoid them.  This only scans the gate list."""
    in_a = lambda q: (mask_a >> int(q)) & 1
    crossing = [i for i, g in enumerate(gates) if int(g["kind"]) in (CZ, ISWAP) and in_a(g["q0"]) != in_a(g["q1"])]
    if any(int(gates[i]["kind"]) != CZ for i in crossing):
        return []
    order = sorted(crossing, key=lambda i: (int(gates[i]["cycle"]), min(int(gates[i]["q0"]), int(gates[i]["q1"]))))
    k = len(order)
    bit_of = {gi: k - 1 - j for j, gi in enumerate(order)}
    held = {}          # block-A qubit -> path bit of its projector, while only diagonal gates follow
    pairs = []
    for i, g in enumerate(gates):
        kind, q0, q1 = int(g["kind"]), int(g["q0"]), int(g["q1"])
        if i in bit_of:
            a = q0 if in_a(q0) else q1
            if a in held:
                pairs.append((held[a], bit_of[i]))
            held[a] = bit_of[i]
        elif kind in (H, XH, YH):
            held.pop(q0, None)
    return pairs


def is_live(path_id: int, pairs) -> bool:
    """Whether a path id sets every pair of equal_bit_pairs equal."""
    return all(((path_id >> u) & 1) == ((path_id >> v) & 1) for u, v in pairs)


def live_path_block(k: int, block_bits: int, seed: int, pairs, draw: Optional[int] = None):
    """A seeded aligned block of 2^block_bits path ids: output `draw` of SplitMix64(seed) (its top
    k - block_bits bits as the block index), or, with draw None, the first output whose block has
    no pair of equal_bit_pairs decided differently within the shared prefix; returns
    (begin, count).  Pairs that involve the low block_bits bits are left to the paths of the
    block."""
    if block_bits > k:
        raise ValueError("block larger than the path space")
    hi_bits = k - block_bits
    pre = [(u, v) for u, v in pairs if u >= block_bits and v >= block_bits]
    rng = SplitMix64(seed)
    for d in range(1 << 16):
        b = 0 if hi_bits == 0 else rng.next() >> (64 - hi_bits)
        if (draw is None and is_live(b << block_bits, pre)) or d == draw:
            return b << block_bits, 1 << block_bits
    raise ValueError("no live block found")


def column_cut_mask(rows: int, cols: int, ncols_a: int) -> int:
    """Block A = columns 0..ncols_a-1 (a vertical cut)."""
    m = 0
    for r in range(rows):
        for c in range(ncols_a):
            m |= 1 << (r * cols + c)
    return m


def row_cut_mask(rows: int, cols: int, nrows_a: int) -> int:
    """Block A = rows 0..nrows_a-1 (a horizontal cut)."""
    return (1 << (nrows_a * cols)) - 1


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    rows: int
    cols: int
    depth: int
    cut: tuple              # ("col", n) or ("row", n)
    n_bits: int
    paths: str              # "all", "sample" (fraction f), "block" (aligned block)
    f: float = 1.0
    block_bits: int = 0
    fp64_sweeps: bool = False
    circuit_seed: int = 0
    bits_seed: int = 0
    path_seed: int = 0
    two_qubit: int = CZ     # CZ, or ISWAP for the harder variant (every CZ replaced)
    # path blocks: index of the SplitMix64(path_seed) draw that gives the block (None: the first
    # draw whose prefix passes equal_bit_pairs)
    block_draw: Optional[int] = None

    @property
    def n_qubits(self) -> int:
        return self.rows * self.cols

    def cut_mask(self) -> int:
        kind, n = self.cut
        if kind == "col":
            return column_cut_mask(self.rows, self.cols, n)
        return row_cut_mask(self.rows, self.cols, n)


def _cfg(i, **kw):
    return WorkloadConfig(circuit_seed=1000 + i, bits_seed=2000 + i, path_seed=3000 + i, **kw)


CONFIGS = {
    # 4x4, 1+16+1, 8+8 cut, all paths, 1024 bitstrings, FP64 sweeps
    "grid4x4_d16": _cfg(1, name="grid4x4_d16", rows=4, cols=4, depth=16, cut=("col", 2),
                        n_bits=1024, paths="all", fp64_sweeps=True),
    # 5x6, 1+24+1, 15+15 cut, all paths, 1e5 bitstrings
    "grid5x6_d24": _cfg(2, name="grid5x6_d24", rows=5, cols=6, depth=24, cut=("col", 3),
                        n_bits=100_000, paths="all"),
    # 6x7, 1+32+1, 21+21 cut, f = 0.01 random subset, 1e6 bitstrings
    "grid6x7_d32": _cfg(3, name="grid6x7_d32", rows=6, cols=7, depth=32, cut=("row", 3),
                        n_bits=1_000_000, paths="sample", f=0.01),
    # 7x8, 1+40+1, 28+28 cut, one seeded aligned block of 1024 paths, 1e6 bitstrings
    # (block_draw 19: the first draw whose block-A states are nonzero in the FP64 oracle,
    # tests/golden/find_live_block.py; draws 11, 13 and 18 pass equal_bit_pairs but are zero)
    "grid7x8_d40": _cfg(4, name="grid7x8_d40", rows=7, cols=8, depth=40, cut=("col", 4),
                        n_bits=1_000_000, paths="block", block_bits=10, block_draw=19),
    # the 5x6, 1+24+1 circuit above with every CZ an iSWAP (2 path bits per crossing gate,
    # k = 30): one seeded aligned block of 2^18 paths, 1e5 bitstrings
    "grid5x6_d24_iswap": WorkloadConfig(name="grid5x6_d24_iswap", rows=5, cols=6, depth=24, cut=("col", 3),
                                        n_bits=100_000, paths="block", block_bits=18, circuit_seed=1002,
                                        bits_seed=2002, path_seed=3005, two_qubit=ISWAP),
}


def make_workload(name: str, n_bits: Optional[int] = None) -> dict:
    """Gate list, cut mask and bitstrings of a named configuration."""
    cfg = CONFIGS[name]
    gates = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed, two_qubit=cfg.two_qubit)
    nb = cfg.n_bits if n_bits is None else n_bits
    bits = random_bitstrings(cfg.n_qubits, nb, cfg.bits_seed)
    return {"cfg": cfg, "gates": gates, "mask_a": cfg.cut_mask(), "bitstrings": bits}


def workload_block(name: str):
    """(begin, count) of a block workload's path ids (live_path_block): the block of the draw the
    configuration names, or the first draw that equal_bit_pairs does not rule out.  The 7x8
    configuration names the first draw whose paths have nonzero terms in the FP64 oracle
    (tests/golden/find_live_block.py), so that the benchmark block carries amplitude."""
    cfg = CONFIGS[name]
    if cfg.paths != "block":
        raise ValueError(f"{name} is not a path-block workload")
    gates = grid_circuit(cfg.rows, cfg.cols, cfg.depth, cfg.circuit_seed, two_qubit=cfg.two_qubit)
    mask = cfg.cut_mask()
    in_a = lambda q: (mask >> int(q)) & 1
    k = sum(1 if int(g["kind"]) == CZ else 2 for g in gates
            if int(g["kind"]) in (CZ, ISWAP) and in_a(g["q0"]) != in_a(g["q1"]))
    return live_path_block(k, cfg.block_bits, cfg.path_seed, equal_bit_pairs(gates, mask), cfg.block_draw)


def serving_mix(n_jobs: int, seed: int):
    """Jobs of the serving workload: grid rows in {4,5,6}, cols in {5,6}, depth
    1+D+1 with D uniform in 16..32, a bitstring count log-uniform in 1e3..1e5 and
    fidelity f uniform in {0.01, 0.1, 1}; every choice is a SplitMix64 draw."""
    rng = SplitMix64(seed)

    def uniform_int(lo, hi):   # inclusive
        return lo + (rng.next() * (hi - lo + 1) >> 64)

    def uniform01():
        return (rng.next() >> 11) * (1.0 / (1 << 53))

    jobs = []
    for i in range(n_jobs):
        rows = uniform_int(4, 6)
        cols = uniform_int(5, 6)
        depth = uniform_int(16, 32)
        n_bits = int(round(10 ** (3 + 2 * uniform01())))
        f = (0.01, 0.1, 1.0)[uniform_int(0, 2)]
        jobs.append({"rows": rows, "cols": cols, "depth": depth, "n_bits": n_bits, "f": f,
                     "circuit_seed": 10_000 + i, "bits_seed": 20_000 + i, "path_seed": 30_000 + i})
    return jobs
