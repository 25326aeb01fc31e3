"""Pins of the oracle's Alias Method (Sec. 2.6, Fig. alias_map) and of the
quadratic error of Fig. convergence, on the CPU.  Nothing here compares the
oracle with itself: the table is checked against the mass every item must
receive, the sampler against exact rational arithmetic on the definition of
Fig. alias_map_details and against the closed-form counts of a regular grid."""
import math
from fractions import Fraction

import numpy as np
import pytest

TWO64 = 1 << 64


def item_mass(t, n):
    """Mass each item receives from the table: its own cell's kept part plus
    the remainders of the cells aliasing it (capacity W per cell)."""
    W = t.W
    got = [0] * n
    for j in range(n):
        got[j] += int(t.thr[j])
        if int(t.thr[j]) < W:
            got[int(t.alias[j])] += W - int(t.thr[j])
    return got


@pytest.mark.parametrize("seed", range(6))
def test_alias_table_gives_every_item_its_mass(orc, seed):
    """Walker's table must give item i exactly the fraction w_i / W of the
    unit interval: with cells of capacity W that is w_i * n, exactly."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    w = rng.integers(0, 2 ** 32, n, dtype=np.uint64)
    if seed % 2:
        w[rng.random(n) < 0.3] = 0  # zero weights: never sampled
    if seed == 4:
        w = (np.floor(np.exp(rng.uniform(0, 22, n)))).astype(np.uint64)  # heavy skew
    if w.sum() == 0:
        w[0] = 1
    w = w.astype(np.uint32)
    t = orc.alias_build(w)
    assert t.W == int(w.astype(np.uint64).sum())
    assert np.all(t.thr <= np.uint64(t.W))
    assert np.all((t.alias >= 0) & (t.alias < n))
    full = t.thr == np.uint64(t.W)
    assert np.array_equal(t.alias[full], np.arange(n)[full])  # a full cell keeps no alias
    assert item_mass(t, n) == [int(x) * n for x in w]
    # a zero weight's cell is entirely its alias's and it is no one's alias
    z = w == 0
    assert np.all(t.thr[z] == 0)
    assert not np.isin(np.nonzero(z)[0], t.alias[~full]).any()


def test_alias_equal_weights_closed_form(orc):
    """Equal weights: every cell is its own item's, and the mapping is
    i = floor(xi n)."""
    n = 37
    t = orc.alias_build(np.full(n, 12345, np.uint32))
    assert np.all(t.thr == np.uint64(t.W)) and np.array_equal(t.alias, np.arange(n))
    u = np.random.default_rng(3).integers(0, 2 ** 64, 5000, dtype=np.uint64)
    want = np.array([(int(x) * n) >> 64 for x in u])
    assert np.array_equal(orc.alias_sample(t, u), want)


def rational_alias(t, n, xi):
    """Fig. alias_map_details: xi in [j/n, (j+1)/n) maps to j when its
    position in the cell is below q_j = thr_j / W, else to alias(j)."""
    j = math.floor(xi * n)
    f = xi * n - j
    return j if f < Fraction(int(t.thr[j]), t.W) else int(t.alias[j])


@pytest.mark.parametrize("seed", range(4))
def test_alias_sample_matches_exact_rationals(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 40))
    w = rng.integers(0, 1000, n).astype(np.uint32)
    w[0] += 1
    t = orc.alias_build(w)
    u = list(rng.integers(0, 2 ** 64, 400, dtype=np.uint64))
    # the points where the mapping jumps: cell edges and split points
    for j in range(n):
        for num in (Fraction(j, n), Fraction(j, n) + Fraction(int(t.thr[j]), t.W * n)):
            c = math.ceil(num * TWO64)
            for d in (-1, 0, 1):
                if 0 <= c + d < TWO64:
                    u.append(np.uint64(c + d))
    u = np.array(u, np.uint64)
    got = orc.alias_sample(t, u)
    want = [rational_alias(t, n, Fraction(int(x), TWO64)) for x in u]
    assert list(got) == want


def test_alias_regular_grid_closed_form(orc):
    """A regular grid of G = 2^b points over n = 2^a cells puts G/n points in
    each cell at relative positions l / (G/n); the cell's own item takes the
    ceil(thr_j G / (n W)) of them below its split point, the alias the rest."""
    rng = np.random.default_rng(7)
    a, b = 6, 14
    n, G = 1 << a, 1 << b
    w = rng.integers(0, 2 ** 20, n).astype(np.uint32)
    w[5] = 0
    t = orc.alias_build(w)
    u = np.arange(G, dtype=np.uint64) << np.uint64(64 - b)
    c = np.bincount(orc.alias_sample(t, u), minlength=n)
    per = G // n
    want = np.zeros(n, np.int64)
    for j in range(n):
        own = -((-int(t.thr[j]) * per) // t.W)  # ceil
        want[j] += own
        want[int(t.alias[j])] += per - own
    assert np.array_equal(c, want)
    assert c[5] == 0


def test_alias_is_not_monotone(orc):
    """Fig. alias_map_details: reordering the intervals breaks monotonicity."""
    w = np.array([5, 1, 3, 2, 6, 6, 7, 6, 28, 2, 14, 33], np.uint32)  # Fig. radix_forest's weights
    t = orc.alias_build(w)
    u = np.sort(np.random.default_rng(1).integers(0, 2 ** 64, 20000, dtype=np.uint64))
    idx = orc.alias_sample(t, u)
    assert np.any(np.diff(idx) < 0)
    # while the inverse mapping is monotone on the same uniforms
    i_inv, _ = orc.search(w, u)
    assert np.all(np.diff(i_inv) >= 0)


def test_alias_zero_total_is_an_error(orc):
    with pytest.raises(orc.OracleError):
        orc.alias_build(np.zeros(5, np.uint32))


def test_quadratic_error_definition(orc):
    """e = sum_i (p_i - c_i / N)^2 (Fig. convergence), by hand."""
    assert orc.quadratic_error([0.5, 0.5], [3, 1], 4) == pytest.approx(0.125, abs=0)
    assert orc.quadratic_error([0.25, 0.75], [1, 3], 4) == 0.0
    assert orc.quadratic_error([1.0, 0.0, 0.0], [0, 2, 0], 2) == pytest.approx(2.0, abs=0)


def test_sine64_alias_converges_slower_on_a_grid(orc):
    """Fig. results_sine64: on the sin^2 density of 64 bins the alias mapping of
    a regular grid has a larger quadratic error than the inverse mapping (for
    the printed N = 2^9 and 2^11 and beyond)."""
    i = np.arange(64)
    p = np.sin(np.pi * i / 64) ** 2 / 32
    q, _ = orc.quantize(p.astype(np.float32))
    t = orc.alias_build(q)
    pq = q / q.astype(np.float64).sum()
    for b in (9, 11, 13):
        N = 1 << b
        u = np.arange(N, dtype=np.uint64) << np.uint64(64 - b)
        i_inv, _ = orc.search(q, u)
        e_inv = orc.quadratic_error(pq, np.bincount(i_inv, minlength=64), N)
        e_alias = orc.quadratic_error(pq, np.bincount(orc.alias_sample(t, u), minlength=64), N)
        assert e_inv < e_alias, (b, e_inv, e_alias)
