"""Pins of the oracle's depth fallback (Sec. 3: a degenerate tree is replaced
by one of logarithmic depth).  Reading: a cell tree over c leaves is replaced
by the balanced tree when some positive-weight leaf lies more than
2 ceil(log2 c) internal nodes deep; the balanced tree splits [lo, hi] at
mid = ceil((lo + hi) / 2)."""
import math

import numpy as np


def comb_weights(c):
    """c weights 2^(c-1), ..., 2, 1: in one cell their fixed-point lower
    bounds share ever longer prefixes of ones (C_i / W has the repeating
    pattern of C_i in c bits), so the levels fall by one per boundary and
    the radix tree is a comb: leaf c-1 lies c-1 internal nodes deep."""
    return np.array([1 << (c - 1 - k) for k in range(c)], np.uint32)


def depth_of_cell(f, a, b):
    """Internal nodes below node a's child 1 on the deepest path to a leaf of
    [a, b] with positive weight (Alg. 2 with u = U_i)."""
    deepest = 0
    for i in range(a, b + 1):
        if i + 1 <= b and f.key[i + 1] == f.key[i]:
            continue
        j, steps = int(f.child[a, 1]), 0
        while j >= 0:
            steps += 1
            j = int(f.child[j, 0] if f.key[i] < f.key[j] else f.child[j, 1])
        deepest = max(deepest, steps)
    return deepest


def test_hand_built_balanced_tree(orc):
    """Eight weights 128, 64, ..., 1 in one cell.  Before: the comb
    node 0 -> 1 -> 2 -> ... -> 7, each node's child 0 the leaf on its left.
    Its deepest leaf lies 7 > 2 ceil(log2 8) = 6 nodes deep, so the cell is
    rebuilt: split(0, 7) = node 4; split(0, 3) = node 2 with split(0, 1) =
    node 1 (leaves 0, 1) and split(2, 3) = node 3 (leaves 2, 3); split(4, 7)
    = node 6 with node 5 (leaves 4, 5) and node 7 (leaves 6, 7).  Node 0
    keeps child 0 = ~0 (distribution start) and gets child 1 = node 4."""
    f = orc.forest(comb_weights(8), m=1)
    comb = [[~0, 1]] + [[~(j - 1), j + 1] for j in range(1, 7)] + [[~6, ~7]]
    assert f.child.tolist() == comb
    g, rebuilt = orc.balance(f)
    assert rebuilt == 1
    expect = [[~0, 4], [~0, ~1], [1, 3], [~2, ~3], [2, 6], [~4, ~5], [5, 7], [~6, ~7]]
    assert g.child.tolist() == expect
    assert np.array_equal(g.key, f.key) and np.array_equal(g.table, f.table)


def test_criterion_at_its_edge(orc):
    """A comb of c leaves is c-1 nodes deep: rebuilt exactly when
    c - 1 > 2 ceil(log2 c), i.e. for c = 8 and c = 10, not for c = 7 or 9."""
    for c, want in [(5, 0), (7, 0), (8, 1), (9, 0), (10, 1), (20, 1)]:
        f = orc.forest(comb_weights(c), m=1)
        assert depth_of_cell(f, 0, c - 1) == c - 1
        g, rebuilt = orc.balance(f)
        assert rebuilt == want, c
        if want:
            assert depth_of_cell(g, 0, c - 1) == math.ceil(math.log2(c))
        else:
            assert np.array_equal(g.child, f.child)


def test_balanced_forest_searches_like_binary_search(orc):
    """After the fallback every search equals binary search (the rebuilt
    trees are search trees over the same keys), at every critical u, in a
    batch of comb, zero-run and random distributions; rebuilt cells have
    balanced depth."""
    rng = np.random.default_rng(5)
    ws = [np.tile(comb_weights(24), 3), comb_weights(31)]
    z = comb_weights(16).astype(np.uint64)
    z[3:6] = 0  # zero weights inside the comb
    ws.append(z.astype(np.uint32))
    ws.append(rng.integers(1, 2 ** 32, 500, dtype=np.uint64).astype(np.uint32))
    sizes = [w.size for w in ws]
    eo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cells = [2, 1, 1, 125]
    co = np.concatenate([[0], np.cumsum(cells)]).astype(np.int64)
    w = np.concatenate(ws)
    f = orc.forest(w, elem_off=eo, cell_off=co)
    g, rebuilt = orc.balance(f)
    assert rebuilt >= 4  # the three combs of 24, the comb of 31, the zero-run comb
    for d in range(len(ws)):
        C = orc.prefix(ws[d])
        Wd = int(C[-1])
        keys = [-((-int(c) << 64) // Wd) for c in C[:-1] if int(c) < Wd]
        u = set([0, 2 ** 64 - 1])
        for k in keys:
            u.update([k, max(k - 1, 0), min(k + 1, 2 ** 64 - 1)])
        u = np.array(sorted(u), np.uint64)
        i_ref, _ = orc.search(ws[d], u, want_x=False)
        assert np.array_equal(orc.descend(g, u, d), i_ref), d
    # rebuilt cells are balanced, the others untouched
    for d in range(len(ws)):
        for gg in range(int(co[d]), int(co[d + 1])):
            a = int(f.table[gg])
            if a < 0:
                continue
            b = a
            while b + 1 < eo[d + 1] and f.key[b + 1] != np.uint64(2 ** 64 - 1) and \
                    (int(f.key[b + 1]) * int(cells[d])) >> 64 == gg - co[d]:
                b += 1
            c = b - a + 1
            if not np.array_equal(g.child[a + 1:b + 1], f.child[a + 1:b + 1]) or \
                    g.child[a, 1] != f.child[a, 1]:
                assert depth_of_cell(f, a, b) > 2 * math.ceil(math.log2(c))
                assert depth_of_cell(g, a, b) <= math.ceil(math.log2(c))


def test_ordinary_forests_are_left_alone(orc):
    """Random weights with a guide table of n/4 cells: no cell tree is
    degenerate, the forest is unchanged."""
    rng = np.random.default_rng(6)
    w = rng.integers(1, 2 ** 32, 1 << 14, dtype=np.uint64).astype(np.uint32)
    f = orc.forest(w, m=1 << 12)
    g, rebuilt = orc.balance(f)
    assert rebuilt == 0 and np.array_equal(g.child, f.child)
