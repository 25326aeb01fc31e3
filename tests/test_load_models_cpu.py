"""Host models of loads per sample used by bench.py's load-count
measurement, checked on small forests of the oracle against cases whose
counts follow from the definitions."""
import numpy as np

import bench
from gpu_util import TWO64, expected_cells


def test_equal_weights_counts(orc):
    """n equal weights with m = n: every cell holds exactly one lower bound, so
    Alg. 2 reads the guide entry and node a (2 loads), the record lookup one
    record, and the Cutpoint bisection spans [g-1, g+1] (2 key loads)."""
    n = 64
    w = np.full(n, 7, np.uint32)
    ref = orc.forest(w, m=n)
    K, aux = expected_cells(ref)
    rng = np.random.default_rng(1)
    u = rng.integers(0, TWO64, 5000, dtype=np.uint64)
    g = ((u.astype(object) * n) >> 64).astype(np.int64)
    a = bench.loads_forest_alg2(ref.key, ref.child, ref.table, n, u)
    assert np.all(a == 2)
    r = bench.loads_forest_records(ref.key, ref.child, ref.table, K, aux, n, u)
    assert np.all(r == 1)
    c = bench.loads_cutpoint(ref.key, ref.table, n, u)
    inner = (g > 0) & (g < n - 1)
    assert np.all(c[inner] == 3) and np.all(c >= 2)


def test_alg2_count_is_path_length(orc):
    """The Alg. 2 count equals one plus the number of nodes on the path the
    oracle's descent takes (walked here one step at a time)."""
    rng = np.random.default_rng(2)
    w = rng.integers(0, 1000, 3000).astype(np.uint32)
    m = 300
    ref = orc.forest(w, m=m)
    u = rng.integers(0, TWO64, 2000, dtype=np.uint64)
    got = bench.loads_forest_alg2(ref.key, ref.child, ref.table, m, u)
    for s, us in enumerate(u.tolist()):
        j = int(ref.table[(us * m) >> 64])
        steps = 1
        while j >= 0:
            steps += 1
            j = int(ref.child[j, 0]) if us < int(ref.key[j]) else int(ref.child[j, 1])
        assert got[s] == steps


def test_load_stats_groups():
    loads = np.array([1] * 63 + [9] + [2] * 64, np.int64)
    st = bench.load_stats(loads)
    assert st["max"] == 9 and st["avg64"] == (9 + 2) / 2 and st["avg32"] == (1 + 9 + 2 + 2) / 4


def test_table1_trends(orc):
    """The paper's load-count table (Table 1, Sec. 4) on its three high-dynamic-range
    densities at n = m = 2^16 (the paper does not state its n and m): the
    Cutpoint maxima equal the printed 6 and 7 for the two periodic densities
    (they do not depend on n), and as the paper reports, the radix forest
    lowers the average and the synchronised-group average while raising the
    maximum."""
    from paper_1901_05423_amd import workloads as wl
    rng = np.random.default_rng(3)
    n = 1 << 16
    u = rng.integers(0, TWO64, 1 << 16, dtype=np.uint64)
    printed_cp_max = {"mod32_pow25": 6, "mod64_pow35": 7}
    for fam in wl.TABLE1_FAMILIES:
        q, _ = orc.quantize(wl.table1_weights(fam, n))
        ref = orc.forest(q, m=n)
        cp = bench.load_stats(bench.loads_cutpoint(ref.key, ref.table, n, u))
        fo = bench.load_stats(bench.loads_forest_alg2(ref.key, ref.child, ref.table, n, u))
        assert fo["avg"] < cp["avg"], fam
        assert fo["avg32"] < cp["avg32"], fam
        if fam in printed_cp_max:
            assert cp["max"] == printed_cp_max[fam], fam
            assert fo["max"] > cp["max"], fam
