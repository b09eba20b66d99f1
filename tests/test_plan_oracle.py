"""Pins for the divide-and-conquer tile split and the packed pair index (Section IV-B, Table I)."""
import os

import pytest

import oracle
from oracle import plan

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_paper_8x8_quadrants():
    g = {r[0]: [int(x) for x in r[1:]] for r in _read("quadtree_8x8.txt")}
    n = g["n"][0]
    assert plan.level1_pair_counts(n) == g["level1"]
    leaves = plan.quadtree_leaves(n, 1)
    assert len(leaves) == g["total"][0]
    assert sorted(leaves) == [(i, j) for i in range(n) for j in range(i + 1, n)]
    # the empty bottom-left quadrant produces no leaf
    assert not any(i >= 4 and j < 4 for i, j in leaves)


@pytest.mark.parametrize("row", _read("table1_pair_counts.txt"))
def test_table1_pair_counts(row):
    _, n, pairs = row[0], int(row[1]), int(row[2])
    assert n * (n - 1) // 2 == pairs
    assert oracle.packed_index(n - 2, n - 1, n) == pairs - 1
    T = 64
    assert sum(len(plan.tile_pairs(bi, bj, T, n)) for bi, bj in plan.quadtree_leaves(n, T)) == pairs


@pytest.mark.parametrize("n", [0, 1, 2, 3, 8, 17, 255, 256, 257])
@pytest.mark.parametrize("T", [1, 4, 64])
def test_leaves_cover_every_pair_once(n, T):
    seen = []
    for bi, bj in plan.quadtree_leaves(n, T):
        assert bi <= bj
        tp = plan.tile_pairs(bi, bj, T, n)
        assert tp, "empty leaf"
        seen.extend(tp)
    assert len(seen) == len(set(seen)) == n * (n - 1) // 2


def test_packed_index_is_dense_row_major():
    n = 13
    pi, pj = oracle.all_pairs(n)
    assert [oracle.packed_index(i, j, n) for i, j in zip(pi, pj)] == list(range(pi.size))


def _golden_loads(name):
    rows = [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and not l.startswith("#")]
    return [(int(a), int(b)) for a, b in rows]


def test_lru_hand_worked_example():
    count, loads = plan.lru_loads(4, 1, 2)
    assert loads == _golden_loads("lru_n4_T1_S2.txt") and count == 8


@pytest.mark.parametrize("n,T", [(4096, 256), (700, 128), (300, 64), (1000, 7), (2, 64)])
def test_lru_bounds(n, T):
    nb = (n + T - 1) // T
    leaves = plan.quadtree_leaves(n, T)
    for S in range(1 if nb == 1 else 2, nb + 3):
        count, loads = plan.lru_loads(n, T, S)
        assert nb <= count <= 2 * len(leaves)
        if S >= nb:
            assert count == nb  # everything fits: each block loaded exactly once
        assert sorted({b for b, _ in loads}) == list(range(nb))  # every block is loaded
        assert all(0 <= s < S for _, s in loads)
