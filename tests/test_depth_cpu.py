"""The deepest search of a forest, on the oracle's forests: the maximum of
Alg. 2's reads over all uniforms is attained at the lower bounds U_i of the
leaves with positive weight (what rtf_forest_depth computes), and it stays
within 68 - floor(log2 m) whatever the weights, while the chains that runs of
zero weights form make the trees themselves arbitrarily deep (the degenerate
trees of Sec. 3 exist but no search reaches into them)."""
import math

import numpy as np
import pytest

from gpu_util import TWO64, alg2_reads, critical_u, forest_depth, random_weights


def height(ref):
    """Structural height: the deepest leaf below its cell's guide entry,
    zero-weight leaves included."""
    key, child, table = ref.key, ref.child, ref.table
    best = 0
    for t in table:
        if t < 0:
            continue
        stack = [(int(t), 2)]
        while stack:
            j, dep = stack.pop()
            best = max(best, dep)
            for c in child[j]:
                if c >= 0 and c != j:
                    stack.append((int(c), dep + 1))
    return best


@pytest.mark.parametrize("seed", range(10))
def test_depth_is_attained_at_lower_bounds(orc, seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(2, 3000))
    w = random_weights(rng, n, zero_frac=[0.0, 0.5, 0.9][seed % 3], skew=seed % 2 == 0)
    for m in {1, 3, max(1, n // 7), n}:
        ref = orc.forest(w, m=m)
        u = np.concatenate([critical_u(ref.key, int(ref.W[0]), m),
                            rng.integers(0, TWO64, 20000, dtype=np.uint64)])
        assert forest_depth(ref) == int(alg2_reads(ref, u).max())


@pytest.mark.parametrize("m", [1, 3, 1000, 4096])
def test_depth_bound_with_long_zero_runs(orc, m):
    """Thousands of zero weights in a row (equal keys): the trees hold chains
    as long as the runs, the searches stay under the bound."""
    rng = np.random.default_rng(m)
    w = random_weights(rng, 20000, skew=True)
    w[100:6100] = 0
    w[9000:9500] = 0
    ref = orc.forest(w, m=m)
    dep = forest_depth(ref)
    assert dep <= 68 - int(math.floor(math.log2(m)))
    if m <= 3:
        assert height(ref) > 5000 > dep


def test_depth_bound_skewed_cells(orc):
    """Weights spread over 32 binary orders of magnitude, few cells: the
    deepest cells of the paper's load-count densities."""
    from paper_1901_05423_amd import workloads as wl
    for fam in wl.TABLE1_FAMILIES:
        q, _ = orc.quantize(wl.table1_weights(fam, 1 << 14))
        for m in (1, 64, 1 << 14):
            ref = orc.forest(q, m=m)
            assert forest_depth(ref) <= 68 - int(math.floor(math.log2(m)))
