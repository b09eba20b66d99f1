"""Reference for the divide-and-conquer split of the pair matrix -- TEST INFRASTRUCTURE ONLY.

Section IV-B: the workload of all pairs (i, j), i < j, is an upper-triangular
matrix; it is split into four quadrants, each split again recursively, and
quadrants holding no pair are skipped.  Here the recursion runs over blocks of
``T`` items and stops at single blocks, so a leaf is the tile of pairs
(rows of block bi) x (columns of block bj), bi <= bj.  Quadrants are visited
top-left, top-right, bottom-left, bottom-right.
"""
from __future__ import annotations


def has_work(r0: int, r1: int, c0: int, c1: int, n: int) -> bool:
    """True iff some pair i < j < n has r0 <= i < r1 and c0 <= j < c1 (item units)."""
    r1 = min(r1, n)
    c1 = min(c1, n)
    if r0 >= r1 or c0 >= c1:
        return False
    # smallest i is r0; the largest j must exceed it and be at least c0
    return max(c0, r0 + 1) <= c1 - 1


def quadtree_leaves(n: int, T: int):
    """Leaf tiles (bi, bj) of the recursive quadrant split, in visiting order."""
    nb = (n + T - 1) // T
    side = 1
    while side < max(nb, 1):
        side *= 2
    out = []

    def rec(b_r0, b_c0, size):
        if not has_work(b_r0 * T, (b_r0 + size) * T, b_c0 * T, (b_c0 + size) * T, n):
            return
        if size == 1:
            out.append((b_r0, b_c0))
            return
        h = size // 2
        rec(b_r0, b_c0, h)
        rec(b_r0, b_c0 + h, h)
        rec(b_r0 + h, b_c0, h)
        rec(b_r0 + h, b_c0 + h, h)

    if n >= 2:
        rec(0, 0, side)
    return out


def tile_pairs(bi: int, bj: int, T: int, n: int):
    """All pairs i < j of tile (bi, bj)."""
    return [(i, j) for i in range(bi * T, min(n, (bi + 1) * T))
            for j in range(bj * T, min(n, (bj + 1) * T)) if i < j]


def level1_pair_counts(n: int):
    """Pair counts of the four first-level quadrants (TL, TR, BL, BR) of an n x n matrix."""
    side = 1
    while side < n:
        side *= 2
    h = side // 2
    quads = [(0, h, 0, h), (0, h, h, side), (h, side, 0, h), (h, side, h, side)]
    return [sum(1 for i in range(r0, min(r1, n)) for j in range(c0, min(c1, n)) if i < j)
            for (r0, r1, c0, c1) in quads]


def lru_loads(n: int, T: int, slots: int):
    """Block loads of a device cache of ``slots`` block slots visiting the leaves in order.

    Section IV-A (first-level device cache): a job (i, j) needs both items in the
    cache; on a miss the least-recently-used slot is evicted and refilled from the
    next level.  Here the cached unit is a block of T items and a job is a leaf tile
    (bi, bj).  The block a tile still needs is never the one evicted for its other
    block.  Returns (number of loads, list of (block, slot) loads in order).
    """
    if slots < 1 or (slots < 2 and (n + T - 1) // T > 1):
        raise ValueError("a tile of two blocks needs two slots")
    holder = [None] * slots   # slot -> block
    last = [-1] * slots       # slot -> time of last use
    where = {}                # block -> slot
    loads = []
    clock = 0
    for bi, bj in quadtree_leaves(n, T):
        need = [bi] if bi == bj else [bi, bj]
        for b in need:
            clock += 1
            if b in where:
                last[where[b]] = clock
                continue
            keep = {where[o] for o in need if o != b and o in where}
            free = [s for s in range(slots) if holder[s] is None]
            if free:
                s = free[0]
            else:
                s = min((s for s in range(slots) if s not in keep), key=lambda s: last[s])
                del where[holder[s]]
            holder[s] = b
            where[b] = s
            last[s] = clock
            loads.append((b, s))
    return len(loads), loads
