"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: expected values come from the
paper's printed figures, from exact rational arithmetic in Python integers,
from closed forms, from brute force, or from the paper's Alg. 1 run under
random schedules against the recursive definition.
"""
from fractions import Fraction
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
TWO64 = 1 << 64


# --------------------------------------------------------------------------
# exact helpers (Python integers; independent of the C oracle)
# --------------------------------------------------------------------------
def exact_prefix(w):
    C = [0]
    for x in w:
        C.append(C[-1] + int(x))
    return C


def exact_index(C, u):
    """The i with C_i * 2^64 <= u * W < C_{i+1} * 2^64 (P_i <= xi < P_{i+1})."""
    W = C[-1]
    uw = int(u) * W
    found = [i for i in range(len(C) - 1) if C[i] * TWO64 <= uw < C[i + 1] * TWO64]
    assert len(found) == 1
    return found[0]


def exact_lower_bound(C, i):
    W = C[-1]
    return -((-(C[i] << 64)) // W)  # ceil(C_i 2^64 / W)


def critical_u(C, m):
    W = C[-1]
    n = len(C) - 1
    cand = {0, TWO64 - 1}
    for i in range(n):
        if C[i] < W:
            U = exact_lower_bound(C, i)
            cand.update({U - 1, U, U + 1})
    for g in range(m + 1):
        e = -((-(g << 64)) // m)
        cand.update({e - 1, e, e + 1})
    return np.array(sorted(c for c in cand if 0 <= c < TWO64), dtype=np.uint64)


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


# --------------------------------------------------------------------------
# Fig. radix_forest: the worked forest (Sec. 3.2)
# --------------------------------------------------------------------------
def load_forest_figure():
    bars, cells, labels, edges = {}, [], {}, []
    with open(os.path.join(HERE, "golden", "radix_forest_fig.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            if t[0] == "bar":
                bars[int(t[1])] = (float(t[2]), float(t[3]))
            elif t[0] == "cellline":
                cells.append(float(t[1]))
            elif t[0] == "label":
                labels[int(t[1])] = t[2]
            elif t[0] == "edge":
                edges.append((t[1], t[2]))
    return bars, cells, labels, edges


def figure_weights():
    """Integer weights read off the figure's bars: the bars tile a span of
    11.7 units and every boundary lies on a multiple of 11.7/113."""
    bars, _, _, _ = load_forest_figure()
    x0, x1 = -0.5, 11.2
    span = x1 - x0
    ends = [bars[i][1] for i in range(12)]
    cdf113 = [(e - x0) / span * 113 for e in ends]
    ints = [round(c) for c in cdf113]
    assert max(abs(c - k) for c, k in zip(cdf113, ints)) < 1e-6
    assert ints[-1] == 113
    w = np.diff([0] + ints).astype(np.uint32)
    return w


def test_figure_input_reading():
    w = figure_weights()
    assert w.tolist() == [5, 1, 3, 2, 6, 6, 7, 6, 28, 2, 14, 33]
    # the figure's generator draws multiples of 1/64, the first seven small
    assert all(x <= 8 for x in w[:7])
    _, cells, _, _ = load_forest_figure()
    assert len(cells) == 12
    for k, c in enumerate(cells):
        assert abs(c - (-0.5 + k * 11.7 / 12)) < 1e-9


def test_figure_forest_edges(orc):
    w = figure_weights()
    f = orc.forest(w, m=12)
    _, _, labels, edges = load_forest_figure()
    drawn = set()
    for a, b in edges:
        drawn.add((int(a), ("leaf", int(b[1:])) if b.startswith("l") else ("node", int(b))))
    C = exact_prefix(w)
    cell = [(exact_lower_bound(C, i) * 12) >> 64 for i in range(12)]
    first = {i for i in range(12) if i == 0 or cell[i] != cell[i - 1]}
    built = set()
    for j in range(12):
        for s in (0, 1):
            if s == 0 and j in first:
                continue  # left child of a cell's first node is not drawn
            c = int(f.child[j, s])
            built.add((j, ("leaf", ~c) if c < 0 else ("node", c)))
    assert built == drawn


def test_figure_leaf_labels(orc):
    """Each leaf's printed digits are a prefix of its lower bound in binary."""
    w = figure_weights()
    f = orc.forest(w, m=12)
    _, _, labels, _ = load_forest_figure()
    for i, lab in labels.items():
        digits = lab.split(".")[1]
        bits = format(int(f.key[i]), "064b")
        assert bits.startswith(digits), (i, lab, bits[:12])


def test_figure_keys_and_table(orc):
    w = figure_weights()
    f = orc.forest(w, m=12)
    C = exact_prefix(w)
    assert [int(k) for k in f.key] == [exact_lower_bound(C, i) for i in range(12)]
    assert int(f.W[0]) == 113
    # guide table from the Cutpoint definition in exact rationals: cell g
    # holds the first interval whose lower bound falls in it, else only the
    # interval covering it from the left is there (complemented reference)
    for g in range(12):
        lo, hi = Fraction(g, 12), Fraction(g + 1, 12)
        inside = [i for i in range(12) if lo <= Fraction(C[i], 113) < hi]
        if inside:
            assert f.table[g] == inside[0]
        else:
            cover = [i for i in range(12) if Fraction(C[i], 113) < lo < Fraction(C[i + 1], 113)]
            assert len(cover) == 1 and f.table[g] == ~cover[0]


SENT = 65  # level of a boundary that no merge crosses


def test_figure_levels_from_labels(orc):
    """Levels of Fig. radix_forest read off the drawing.

    A leaf's printed digits are its lower bound's binary prefix down to the
    split above it, so two neighbours in one cell first differ at printed
    digit p, which is bit 64 - p of the 0.64 keys: level 65 - p (Sec. 3.1).
    Neighbours in different cells (by the drawn cell lines) are SENT."""
    w = figure_weights()
    _, cells, labels, _ = load_forest_figure()
    bars, _, _, _ = load_forest_figure()
    # the cell of a leaf is the cell line interval its bar's left end lies in
    width = cells[1] - cells[0]
    cell = [int((bars[i][0] - cells[0]) // width + 1e-9) for i in range(12)]
    cell[0] = 0
    expect = []
    for b in range(11):
        if cell[b] != cell[b + 1]:
            expect.append(SENT)
            continue
        da, db = labels[b].split(".")[1], labels[b + 1].split(".")[1]
        p = next(k for k in range(min(len(da), len(db))) if da[k] != db[k]) + 1
        expect.append(65 - p)
    assert expect == [60, 59, 61, SENT, 62, SENT, SENT, 61, SENT, SENT, SENT]
    assert orc.levels(w, 12).tolist() == expect


@pytest.mark.parametrize("seed", range(8))
def test_levels_brute_force(orc, seed):
    """Levels against a bit-string comparison of exact keys: the first
    differing binary digit of U_b and U_{b+1} (Sec. 3.1), SENT where the
    cells differ (Sec. 3.2) and from the last positive weight on."""
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(2, 200))
    w = random_weights(rng, n, zero_frac=[0, 0.3, 0.6, 0.1][seed % 4], skew=seed % 2 == 0)
    if seed % 3 == 1:
        w[-3:] = 0
        if w.sum() == 0:
            w[0] = 5
    C = exact_prefix(w)
    last = max(i for i in range(n) if w[i] > 0)
    for m in {1, 3, n, 4 * n}:
        lvl = orc.levels(w, m)
        for b in range(n - 1):
            if b + 1 > last:
                assert lvl[b] == SENT, (b, m)
                continue
            Ua, Ub = exact_lower_bound(C, b), exact_lower_bound(C, b + 1)
            # cells of the keys: floor(U m / 2^64), exact in rationals
            ga = math.floor(Fraction(Ua, TWO64) * m)
            gb = math.floor(Fraction(Ub, TWO64) * m)
            if ga != gb:
                assert lvl[b] == SENT, (b, m)
                continue
            sa, sb = format(Ua, "064b"), format(Ub, "064b")
            diff = [k for k in range(64) if sa[k] != sb[k]]
            assert lvl[b] == (64 - diff[0] if diff else 0), (b, m, sa, sb)


# --------------------------------------------------------------------------
# Fig. results_sine64: monotonic mapping of a regular grid (Sec. 2.6)
# --------------------------------------------------------------------------
def test_sine64_printed_histograms(orc):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "sine64_monotone.txt"))
            if not l.startswith("#")]
    target = np.array([float(r[1]) for r in rows])
    printed = {2 ** 9: np.array([float(r[2]) for r in rows]),
               2 ** 11: np.array([float(r[3]) for r in rows])}
    i = np.arange(64)
    p = np.sin(np.pi * i / 64) ** 2 / 32
    # the plotted target is p_i = sin^2(pi i / 64) / 32 to the printed digits
    assert np.abs(p - target).max() <= 5e-7
    q, _ = orc.quantize(p.astype(np.float32))
    for N, pr in printed.items():
        b = int(math.log2(N))
        u = np.arange(N, dtype=np.uint64) << np.uint64(64 - b)
        idx, _ = orc.search(q, u)
        c = np.bincount(idx, minlength=64)
        got = np.array([float("%.6f" % (cc / N)) for cc in c])
        # P_32 = 31/64 and P_33 = 33/64 are exact ties for the grid; which side
        # a tie point falls on depends on rounding, so bins 31..33 are pinned
        # by their total only
        ties = [31, 32, 33]
        other = [k for k in range(64) if k not in ties]
        assert np.array_equal(got[other], pr[other])
        assert c[ties].sum() == round(pr[ties].sum() * N)


# --------------------------------------------------------------------------
# binary search (Sec. 2.2) vs linear search (Sec. 2.1) vs exact definition
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(12))
def test_search_brute_force_small(orc, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 65))
    w = random_weights(rng, n, zero_frac=[0, 0.3, 0.6][seed % 3], skew=seed % 2 == 1)
    C = exact_prefix(w)
    m = int(rng.integers(1, 3 * n + 1))
    u = critical_u(C, m)
    idx, x = orc.search(w, u)
    lin = orc.linear_search(w, u)
    ref = np.array([exact_index(C, uu) for uu in u], np.int32)
    assert np.array_equal(idx, ref)
    assert np.array_equal(lin, ref)
    assert np.all(w[idx] > 0)
    # x against exact rationals: x = (i + (u W / 2^64 - C_i) / w_i) / n
    for s in range(0, u.size, max(1, u.size // 50)):
        i = int(idx[s])
        ex = (i + (Fraction(int(u[s]) * C[-1], TWO64) - C[i]) / int(w[i])) / n
        assert abs(x[s] - float(ex)) <= 4 * np.spacing(max(float(ex), 1e-300)) + 1e-300


def test_oracle_prefix_exact(orc):
    rng = np.random.default_rng(5)
    w = random_weights(rng, 1000)
    assert [int(c) for c in orc.prefix(w)] == exact_prefix(w)


def test_monotone_mapping(orc):
    """u1 < u2 implies i1 <= i2 and x1 <= x2 (the mapping is monotone)."""
    rng = np.random.default_rng(7)
    w = random_weights(rng, 5000, zero_frac=0.2, skew=True)
    u = np.sort(rng.integers(0, 2 ** 64, 200000, dtype=np.uint64))
    idx, x = orc.search(w, u)
    assert np.all(np.diff(idx) >= 0)
    assert np.all(np.diff(x) >= 0)
    n = w.size
    assert np.all(x >= idx / n) and np.all(x <= (idx + 1) / n)


def test_equal_weights_closed_form(orc):
    """Equal weights: i = floor(u n / 2^64) and x = u / 2^64."""
    rng = np.random.default_rng(8)
    for n in (1, 3, 1000, 4097):
        w = np.full(n, 12345, np.uint32)
        u = rng.integers(0, 2 ** 64, 2000, dtype=np.uint64)
        idx, x = orc.search(w, u)
        ref = np.array([(int(uu) * n) >> 64 for uu in u])
        assert np.array_equal(idx, ref)
        xi = np.array([float(Fraction(int(uu), TWO64)) for uu in u])
        assert np.abs(x - xi).max() <= 1e-15


def test_regular_grid_closed_form(orc):
    """Grid u_k = k 2^(64-b): count of bin i is ceil(2^b C_{i+1}/W) - ceil(2^b C_i/W)."""
    rng = np.random.default_rng(9)
    w = random_weights(rng, 300, zero_frac=0.1, skew=True)
    C = exact_prefix(w)
    W = C[-1]
    b = 14
    u = np.arange(1 << b, dtype=np.uint64) << np.uint64(64 - b)
    idx, _ = orc.search(w, u)
    c = np.bincount(idx, minlength=w.size)
    ceil = lambda a: -((-a) // W)
    ref = [ceil(C[i + 1] << b) - ceil(C[i] << b) for i in range(w.size)]
    assert c.tolist() == ref


def test_zero_total_is_an_error(orc):
    with pytest.raises(orc.OracleError):
        orc.search(np.zeros(5, np.uint32), np.array([1], np.uint64))
    with pytest.raises(orc.OracleError):
        orc.forest(np.zeros(5, np.uint32), m=4)


# --------------------------------------------------------------------------
# forest + Alg. 2 == binary search (Sec. 4: identical mapping)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(16))
def test_forest_descent_equals_search(orc, seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(1, 400))
    w = random_weights(rng, n, zero_frac=[0, 0.25, 0.7, 0][seed % 4], skew=seed % 3 == 0)
    if seed % 5 == 0:
        w[-min(n - 1, 7):] = 0  # trailing zero weights
        if w.sum() == 0:
            w[0] = 3
    C = exact_prefix(w)
    for m in {1, 2, max(1, n // 7), n, 3 * n, 1 << 12}:
        f = orc.forest(w, m=m)
        u = critical_u(C, m)
        got = orc.descend(f, u)
        ref, _ = orc.search(w, u)
        assert np.array_equal(got, ref), (n, m)


@pytest.mark.parametrize("seed", range(10))
def test_alg1_random_schedules_match_definition(orc, seed):
    """Alg. 1 under arbitrary interleavings builds the forest of the definition."""
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(1, 600))
    w = random_weights(rng, n, zero_frac=[0, 0.3, 0.8][seed % 3], skew=seed % 2 == 0)
    if seed % 4 == 3:
        w[-3:] = 0
        if w.sum() == 0:
            w[0] = 1
    for m in {1, max(1, n // 10), n, 2 * n + 1}:
        f = orc.forest(w, m=m)
        for sched in range(3):
            key, child = orc.alg1(w, m, seed=1 + 7919 * sched + seed)
            assert np.array_equal(key, f.key)
            assert np.array_equal(child, f.child), (n, m, sched)


def forest_checks(w, f, m):
    """Structural invariants of a forest (Sec. 3.1, 3.2)."""
    n = w.size
    C = exact_prefix(w)
    W = C[-1]
    n_eff = max(i for i in range(n) if w[i] > 0) + 1
    key = [int(k) for k in f.key]
    cell = [(key[i] * m) >> 64 for i in range(n_eff)]
    first = [i for i in range(n_eff) if i == 0 or cell[i] != cell[i - 1]]
    seen_leaf = [0] * n
    depth_max = 0
    for a in first:
        # left child of a cell's first node: the interval on its left
        assert f.child[a, 0] == (~a if a == 0 else ~(a - 1))
        b = a
        while b + 1 < n_eff and cell[b + 1] == cell[a]:
            b += 1
        # walk the cell's tree: every subtree covers a contiguous leaf range
        stack = [(int(f.child[a, 1]), a, b, 1)]
        while stack:
            ref, lo, hi, dep = stack.pop()
            depth_max = max(depth_max, dep)
            if ref < 0:
                assert lo == hi == ~ref
                seen_leaf[~ref] += 1
                continue
            j = ref
            assert lo < j <= hi  # node j splits between leaf j-1 and j
            stack.append((int(f.child[j, 0]), lo, j - 1, dep + 1))
            stack.append((int(f.child[j, 1]), j, hi, dep + 1))
    assert seen_leaf[:n_eff] == [1] * n_eff
    for j in range(n_eff, n):
        assert f.child[j, 0] == ~j and f.child[j, 1] == ~j
        assert key[j] == TWO64 - 1
    assert depth_max <= 66 + int((w == 0).sum())
    assert key[:n_eff] == [exact_lower_bound(C, i) for i in range(n_eff)]
    assert int(f.W[0]) == W


@pytest.mark.parametrize("seed", range(20))
def test_forest_invariants(orc, seed):
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(1, 300))
    w = random_weights(rng, n, zero_frac=[0, 0.2, 0.5, 0.9][seed % 4], skew=seed % 2 == 1)
    if seed % 3 == 2:
        w[:2] = 0
        w[-2:] = 0
        if w.sum() == 0:
            w[n // 2] = 9
    for m in {1, max(1, n // 3), n, 3 * n}:
        forest_checks(w, orc.forest(w, m=m), m)


def test_batched_forest_is_per_distribution(orc):
    """Many distributions at once (Sec. 5) equal separate builds, offset."""
    rng = np.random.default_rng(11)
    sizes = [1, 5, 64, 3, 200, 17]
    cells = [1, 7, 64, 2, 150, 40]
    ws = [random_weights(rng, s, zero_frac=0.2) for s in sizes]
    eo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    co = np.concatenate([[0], np.cumsum(cells)]).astype(np.int64)
    fb = orc.forest(np.concatenate(ws), elem_off=eo, cell_off=co)
    for d, (w, m) in enumerate(zip(ws, cells)):
        f1 = orc.forest(w, m=m)
        a, b = eo[d], eo[d + 1]
        assert np.array_equal(fb.key[a:b], f1.key)
        sh = lambda r: np.where(r >= 0, r + a, ~(~r + a))
        assert np.array_equal(fb.child[a:b], sh(f1.child))
        assert np.array_equal(fb.table[co[d]:co[d + 1]], sh(f1.table))
        u = rng.integers(0, 2 ** 64, 500, dtype=np.uint64)
        ref, _ = orc.search(w, u)
        assert np.array_equal(orc.descend(fb, u, d), ref)


# --------------------------------------------------------------------------
# quantisation rule
# --------------------------------------------------------------------------
def test_quantize_properties(orc):
    rng = np.random.default_rng(12)
    v = rng.random(10000).astype(np.float32)
    v[::97] = 0
    q, s = orc.quantize(v)
    mx = float(v.max())
    assert q[np.argmax(v)] == 2 ** 32 - 1
    assert np.all(q[v == 0] == 0) and np.all(q[v > 0] >= 1)
    # within half a unit (plus rounding of the scale) of the exact scaled value
    exact = v.astype(np.float64) * (2 ** 32 - 1) / mx
    assert np.all(np.abs(q - exact) <= 0.5 + 1e-6 * np.maximum(exact, 1))
    order = np.argsort(v, kind="stable")
    assert np.all(np.diff(q[order].astype(np.int64)) >= 0)
    # exact power-of-two scaling of the input does not change the result
    q2, _ = orc.quantize(v * np.float32(0.25))
    assert np.array_equal(q, q2)
    # -0.0 is a zero weight: it neither sets the maximum nor gets mass
    qz, sz = orc.quantize(np.array([-0.0, 0.5, -0.0, 0.25], np.float32))
    assert qz.tolist() == [0, 2 ** 32 - 1, 0, 2 ** 31] and sz[0] == (2 ** 32 - 1) / 0.5
    tiny = np.array([1e-30, 1.0], np.float32)
    assert orc.quantize(tiny)[0].tolist() == [1, 2 ** 32 - 1]
    with pytest.raises(orc.OracleError):
        orc.quantize(np.array([1.0, -1.0], np.float32))
    with pytest.raises(orc.OracleError):
        orc.quantize(np.array([1.0, np.nan], np.float32))


# --------------------------------------------------------------------------
# gradient of the continuous position (index held fixed)
# --------------------------------------------------------------------------
def x_of_weights(v, i, xi):
    """x = (i + (xi * sum(v) - sum_{k<i} v_k) / v_i) / n in FP64."""
    cs = np.concatenate([[0.0], np.cumsum(v)])
    return (i + (xi * cs[-1] - cs[i]) / v[i]) / v.size


def test_grad_matches_central_differences(orc):
    rng = np.random.default_rng(13)
    n, S = 40, 300
    v = (0.1 + rng.random(n)).astype(np.float32)
    q, s = orc.quantize(v)
    wv = q.astype(np.float64) / s[0]  # the real weights the kernel sees
    u = rng.integers(0, 2 ** 64, S, dtype=np.uint64)
    g = rng.standard_normal(S)
    idx, _ = orc.search(q, u)
    xi = np.array([float(Fraction(int(uu), TWO64)) for uu in u])
    grad = orc.grad(q, s[0], u, g)
    h = 1e-6
    fd = np.zeros(n)
    for k in range(n):
        vp, vm = wv.copy(), wv.copy()
        vp[k] += h
        vm[k] -= h
        lp = sum(g[t] * x_of_weights(vp, idx[t], xi[t]) for t in range(S))
        lm = sum(g[t] * x_of_weights(vm, idx[t], xi[t]) for t in range(S))
        fd[k] = (lp - lm) / (2 * h)
    assert np.abs(grad - fd).max() <= 1e-5 * np.abs(fd).max()
    # x is 0-homogeneous in the weights: sum_k v_k dL/dv_k = 0
    assert abs(np.dot(wv, grad)) <= 1e-9 * np.abs(wv * grad).sum()


def test_grad_matches_per_sample_closed_form(orc):
    """dx_s/dv_k = (xi_s - [k < i_s] - [k == i_s] frac_s) / (n v_{i_s})."""
    rng = np.random.default_rng(14)
    n, S = 25, 60
    v = (0.05 + rng.random(n)).astype(np.float32)
    v[3] = 0
    q, s = orc.quantize(v)
    wv = q.astype(np.float64) / s[0]
    u = rng.integers(0, 2 ** 64, S, dtype=np.uint64)
    g = rng.standard_normal(S)
    idx, x = orc.search(q, u)
    ref = np.zeros(n)
    for t in range(S):
        i = int(idx[t])
        xi = float(Fraction(int(u[t]), TWO64))
        frac = x[t] * n - i
        for k in range(n):
            d = xi - (1.0 if k < i else 0.0) - (frac if k == i else 0.0)
            ref[k] += g[t] * d / (n * wv[i])
    grad = orc.grad(q, s[0], u, g)
    assert np.abs(grad - ref).max() <= 1e-9 * np.abs(ref).max()
