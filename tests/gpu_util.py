"""Helpers shared by the GPU parity tests (host side only)."""
import math
import sys

import numpy as np

TWO64 = 1 << 64


def note(msg):
    """Name the case on stdout before its GPU work starts."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def random_weights(rng, n, zero_frac=0.0, skew=False):
    if skew:
        w = np.floor(np.exp(rng.uniform(0, math.log(2 ** 32 - 1), n))).astype(np.uint64)
    else:
        w = rng.integers(1, 2 ** 32, n, dtype=np.uint64)
    if zero_frac > 0:
        w[rng.random(n) < zero_frac] = 0
    if w.sum() == 0:
        w[rng.integers(0, n)] = 1
    return w.astype(np.uint32)


def critical_u(key, W, m, extra=0, rng=None):
    """Uniforms at and around every lower bound and every cell edge, plus 0 and
    2^64-1 (the places where an off-by-one in the search would show)."""
    key = np.asarray(key, np.uint64)
    real = key[key != np.uint64(TWO64 - 1)]
    c = [np.uint64(0), np.uint64(TWO64 - 1)]
    parts = [real, real - np.uint64(1), real + np.uint64(1)]
    g = np.arange(m + 1, dtype=object)
    edges = np.array([-((-(int(x) << 64)) // m) for x in g[: min(m + 1, 5000)]], dtype=object)
    edges = edges[(edges > 0) & (edges < TWO64)].astype(np.uint64)
    parts += [edges, edges - np.uint64(1)]
    u = np.concatenate([np.array(c, np.uint64)] + [p.astype(np.uint64) for p in parts])
    if extra and rng is not None:
        u = np.concatenate([u, rng.integers(0, 2 ** 64, extra, dtype=np.uint64)])
    return u


X_TOL = 1e-12  # x in FP64 from exact integers: a few ulps (the bar is 1e-6)


def assert_samples(idx_gpu, x_gpu, idx_ref, x_ref):
    idx_gpu = np.asarray(idx_gpu)
    bad = np.nonzero(idx_gpu != idx_ref)[0]
    assert bad.size == 0, f"{bad.size} indices differ, first at {bad[:5]}"
    if x_ref is not None:
        err = np.abs(np.asarray(x_gpu) - x_ref)
        assert err.max() <= X_TOL, f"max |x - x_ref| = {err.max()}"


CELL_BOUNDS = 5  # lower bounds a guide cell record holds
CELL_KEYS = CELL_BOUNDS + 2  # keys of a record: k[0] .. k[CELL_BOUNDS + 1]


def _cells_of(key, x, eo, co):
    """Global guide cell of leaf x with key `key`: co_d + floor(key * m_d / 2^64)."""
    d = np.searchsorted(eo, x, side="right") - 1
    m = (co[d + 1] - co[d]).astype(np.uint64)
    kh, kl = key >> np.uint64(32), key & np.uint64(0xFFFFFFFF)
    hi = (kh * m + ((kl * m) >> np.uint64(32))) >> np.uint64(32)
    return co[d] + hi.astype(np.int64)


def expected_cells(ref):
    """The keys and aux field each 64-byte guide cell record must hold, derived
    from the oracle forest (the record is described in include/rtforest.h)."""
    MAX = np.uint64(TWO64 - 1)
    key, child, table = ref.key, ref.child, ref.table.astype(np.int64)
    eo, co = ref.elem_off.astype(np.int64), ref.cell_off.astype(np.int64)
    n, m = key.size, table.size
    node = table >= 0
    a = np.where(node, table, ~table)  # first node a, or covering leaf i
    end = eo[np.searchsorted(eo, a, side="right")]  # end of a's distribution
    g = np.arange(m, dtype=np.int64)
    K = np.zeros((m, CELL_KEYS), np.uint64)
    prev = np.where(key[a] == 0, np.uint64(0), key[np.maximum(a - 1, 0)])
    nxt = np.where(a + 1 < end, key[np.minimum(a + 1, n - 1)], MAX)
    K[:, 0] = np.where(node, prev, key[a])
    K[:, 1] = np.where(node, key[a], nxt)
    opened = node.copy()
    cnt = np.ones(m, np.int64)
    for t in range(1, CELL_BOUNDS + 1):
        x = a + t
        xc = np.minimum(x, n - 1)
        kx = key[xc]
        live = (x < end) & (kx != MAX)
        cx = np.where(live, _cells_of(np.where(live, kx, 0), xc, eo, co), -1)
        incell = opened & live & (cx == g)
        closing = opened & ~incell
        K[:, t + 1] = np.where(incell, kx, np.where(closing, np.where(live, kx, MAX), np.uint64(0)))
        cnt += incell
        opened &= incell
    aux = np.where(node, np.where(opened, child[a, 1], ~cnt), table).astype(np.int32)
    return K, aux


def assert_forest(f, ref, what=""):
    key, child, table, W, (ckeys, cc1) = f.export(with_cells=True)
    assert np.array_equal(W, ref.W), f"{what} totals differ"
    bk = np.nonzero(key != ref.key)[0]
    assert bk.size == 0, f"{what} {bk.size} keys differ, first at {bk[:5]}"
    bc = np.nonzero((child != ref.child).any(axis=1))[0]
    assert bc.size == 0, f"{what} {bc.size} node records differ, first at {bc[:5]}: " \
        f"gpu {child[bc[:3]].tolist()} ref {ref.child[bc[:3]].tolist()}"
    bt = np.nonzero(table != ref.table)[0]
    assert bt.size == 0, f"{what} {bt.size} table entries differ, first at {bt[:5]}"
    ek, ec1 = expected_cells(ref)
    bx = np.nonzero((ckeys != ek).any(axis=1) | (cc1 != ec1))[0]
    assert bx.size == 0, f"{what} {bx.size} cell records differ, first at {bx[:5]}: " \
        f"gpu {ckeys[bx[:2]].tolist()} {cc1[bx[:2]].tolist()} ref {ek[bx[:2]].tolist()} " \
        f"{ec1[bx[:2]].tolist()}"


def expected_wide(ref):
    """The collapsed records rtf_forest_widen must write, derived from the
    oracle forest: (node indices j, int64 rows [len(j), 5] holding k, kc0,
    kc1 and the reference pairs (r0, r1), (r2, r3) as int32 pairs)."""
    MAX = np.uint64(TWO64 - 1)
    key, child, table = ref.key, ref.child, ref.table.astype(np.int64)
    eo, co = ref.elem_off.astype(np.int64), ref.cell_off.astype(np.int64)
    _, aux = expected_cells(ref)
    j = np.nonzero(key != MAX)[0]
    g = _cells_of(key[j], j, eo, co)
    deep = (table[g] >= 0) & (aux[g] >= 0) & (table[g] != j)
    j = j[deep]
    rows = np.zeros((j.size, 5), np.int64)
    rows[:, 0] = key[j].view(np.int64)
    refs = []
    for s in (0, 1):
        c = child[j, s].astype(np.int64)
        inner = c >= 0
        cc = np.where(inner, c, 0)
        rows[:, 1 + s] = np.where(inner, key[cc], np.uint64(0)).view(np.int64)
        refs.append(np.where(inner, child[cc, 0], c).astype(np.int32))
        refs.append(np.where(inner, child[cc, 1], c).astype(np.int32))
    pair = lambda a, b: (b.astype(np.int64) << 32) | (a.astype(np.int64) & 0xFFFFFFFF)  # noqa: E731
    rows[:, 3] = pair(refs[0], refs[1])
    rows[:, 4] = pair(refs[2], refs[3])
    return j, rows


def assert_wide(f, ref, what=""):
    j, rows = expected_wide(ref)
    got = f.wide_view().cpu().numpy()[j, :5]
    bad = np.nonzero((got != rows).any(axis=1))[0]
    assert bad.size == 0, f"{what} {bad.size} of {j.size} collapsed records differ, first nodes " \
        f"{j[bad[:5]]}: gpu {got[bad[:2]].tolist()} ref {rows[bad[:2]].tolist()}"
    return j.size


def alg2_reads(ref, u, d=0):
    """Reads Alg. 2 makes for each uniform of distribution d on the oracle
    forest: the guide entry plus one per node visited."""
    key, child, table = ref.key, ref.child, ref.table.astype(np.int64)
    co, m = int(ref.cell_off[d]), int(ref.cell_off[d + 1] - ref.cell_off[d])
    u = np.asarray(u, np.uint64)
    g = ((u.astype(object) * m) >> 64).astype(np.int64)
    j = table[co + g]
    reads = np.ones(u.size, np.int64)
    act = j >= 0
    while act.any():
        ja = j[act]
        reads[act] += 1
        j[act] = np.where(u[act] < key[ja], child[ja, 0], child[ja, 1])
        act = j >= 0
    return reads


def forest_depth(ref):
    """The deepest search of the oracle forest (what rtf_forest_depth
    reports): Alg. 2's reads for u = U_i over the leaves with positive
    weight, every distribution."""
    MAX = np.uint64(TWO64 - 1)
    best = 0
    eo = ref.elem_off
    for d in range(eo.size - 1):
        if int(ref.W[d]) == 0:
            continue
        k = ref.key[eo[d]:eo[d + 1]]
        nxt = np.append(k[1:], MAX)
        live = (k != MAX) & ((nxt != k) | (nxt == MAX))
        if live.any():
            best = max(best, int(alg2_reads(ref, k[live], d).max()))
    return best
