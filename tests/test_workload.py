"""Host-side checks of the seeded input generators."""
import numpy as np
import pytest

from workload import (CONFIGS, CZ, H, T, XH, YH, SplitMix64, cz_pattern_edges, grid_circuit,
                      make_workload, path_block, random_bitstrings, splitmix64_array)


def test_splitmix64_known_outputs():
    # first outputs for seed 0 and seed 1234567 of the published SplitMix64
    r = SplitMix64(0)
    assert [r.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                             0x06C45D188009454F]
    r = SplitMix64(1234567)
    assert r.next() == 6457827717110365317
    np.testing.assert_array_equal(splitmix64_array(1234567, 2),
                                  np.array([6457827717110365317, 3203168211198807973],
                                           dtype=np.uint64))


@pytest.mark.parametrize("rows,cols", [(4, 4), (5, 6), (6, 7), (7, 8), (3, 5)])
def test_layouts_are_matchings_covering_every_edge_once(rows, cols):
    all_edges = set()
    for r in range(rows):
        for c in range(cols):
            q = r * cols + c
            if c + 1 < cols:
                all_edges.add((q, q + 1))
            if r + 1 < rows:
                all_edges.add((q, q + cols))
    seen = []
    for pat in range(8):
        e = cz_pattern_edges(rows, cols, pat)
        qs = [q for ed in e for q in ed]
        assert len(qs) == len(set(qs)), "a layout must be a matching"
        seen.extend(e)
    assert sorted(seen) == sorted(all_edges)


def test_layouts_alternate_horizontal_and_vertical():
    for pat in range(8):
        e = cz_pattern_edges(4, 4, pat)
        horizontal = all(b - a == 1 for a, b in e)
        assert horizontal == (pat % 2 == 0)


def test_generator_rules():
    g = grid_circuit(5, 6, 24, seed=1002)
    n = 30
    assert all(int(x["kind"]) == H and int(x["cycle"]) == 0 for x in g[:n])
    assert all(int(x["kind"]) == H and int(x["cycle"]) == 25 for x in g[-n:])
    last = {}
    cz_in = {}
    for x in g:
        c = int(x["cycle"])
        if int(x["kind"]) == CZ:
            cz_in.setdefault(c, set()).update((int(x["q0"]), int(x["q1"])))
    for x in g[n:-n]:
        c, k, q = int(x["cycle"]), int(x["kind"]), int(x["q0"])
        if k == CZ:
            continue
        assert c >= 2
        assert q in cz_in.get(c - 1, set()) and q not in cz_in.get(c, set())
        if q not in last:
            assert k == T
        elif last[q] != T:
            assert k != last[q] and k in (XH, YH)
        else:
            assert k in (XH, YH)
        last[q] = k


def test_generator_is_deterministic():
    a = grid_circuit(6, 7, 32, seed=5)
    b = grid_circuit(6, 7, 32, seed=5)
    c = grid_circuit(6, 7, 32, seed=6)
    assert a.tobytes() == b.tobytes()
    assert a.tobytes() != c.tobytes()


def test_bitstrings_distinct_and_in_range():
    b = random_bitstrings(16, 1024, 2001)
    assert b.size == 1024 and np.unique(b).size == 1024
    assert int(b.max()) < 1 << 16
    b2 = random_bitstrings(56, 5000, 2004)
    assert np.unique(b2).size == 5000 and int(b2.max()) < 1 << 56
    np.testing.assert_array_equal(random_bitstrings(16, 1024, 2001), b)


def test_path_block():
    begin, count = path_block(35, 10, 3004)
    assert count == 1024 and begin % 1024 == 0 and begin + count <= 1 << 35


def test_named_configs():
    w = make_workload("grid4x4_d16")
    assert w["bitstrings"].size == 1024
    assert bin(w["mask_a"]).count("1") == 8 and w["mask_a"] & 1
    for name, cfg in CONFIGS.items():
        assert bin(cfg.cut_mask()).count("1") * 2 == cfg.n_qubits, name
