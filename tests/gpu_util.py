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


def expected_cells(ref):
    """The repeated keys and child each guide cell record must hold, derived
    from the oracle forest (see the cell record in include/rtforest.h)."""
    MAX = np.uint64(TWO64 - 1)
    key, child, table, eo = ref.key, ref.child, ref.table.astype(np.int64), ref.elem_off
    node = table >= 0
    a = np.where(node, table, ~table)  # first node a, or covering leaf i
    end = eo[np.searchsorted(eo, a, side="right")]
    nxt_ok = (a + 1 < end)
    nxt = np.where(nxt_ok, key[np.minimum(a + 1, key.size - 1)], MAX)
    nxt = np.where(nxt == MAX, MAX, nxt)
    prev = np.where(key[a] == 0, np.uint64(0), key[np.maximum(a - 1, 0)])
    k0 = np.where(node, prev, key[a])
    k1 = np.where(node, key[a], nxt)
    k2 = np.where(node, nxt, np.uint64(0))
    c1 = np.where(node, child[a, 1], table).astype(np.int32)
    return np.stack([k0, k1, k2], axis=1).astype(np.uint64), c1


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
