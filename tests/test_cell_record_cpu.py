"""The 64-byte guide cell record, checked on the CPU: records derived from the
oracle forest (the layout the GPU build must write) resolve every sample to
the oracle's binary-search index, through the record alone or through the
tree descent the record points to (Alg. 2 with the guide entry of Sec. 3.2)."""
import numpy as np
import pytest

from gpu_util import CELL_BOUNDS, CELL_KEYS, TWO64, critical_u, expected_cells, random_weights


def model_sample(ref, K, aux, u):
    """Resolve uniforms of one distribution the way the sampling kernel does."""
    key, child, table = ref.key, ref.child, ref.table
    m = table.size
    out = np.empty(u.size, np.int64)
    for s, us in enumerate(u.tolist()):
        g = (us * m) >> 64
        t = int(table[g])
        if t < 0:
            out[s] = ~t
            continue
        a = int(aux[g])
        if a < 0 or us < int(K[g, CELL_KEYS - 1]):
            lim = ~a if a < 0 else CELL_BOUNDS
            j = sum(1 for q in range(1, lim + 1) if int(K[g, q]) <= us)
            out[s] = t - 1 + j
            continue
        j = a
        while j >= 0:
            j = int(child[j, 0]) if us < int(key[j]) else int(child[j, 1])
        out[s] = ~j
    return out


CASES = [
    # (n, m, zero_frac, skew): cells from nearly empty to hundreds of leaves
    (1000, 1000, 0.0, False),
    (5000, 1000, 0.0, False),   # about 5 leaves per cell: both record paths
    (20000, 1000, 0.0, False),  # about 20 per cell: mostly descents
    (5000, 400, 0.1, False),    # dense cells: descents from aux
    (3000, 6000, 0.3, True),    # sparse, skewed, zero runs: covered cells
    (2048, 1, 0.0, False),      # one cell: a single tree
    (7, 64, 0.0, False),
]


@pytest.mark.parametrize("n,m,zf,skew", CASES)
def test_records_resolve_like_binary_search(orc, n, m, zf, skew):
    rng = np.random.default_rng(n * 7 + m)
    w = random_weights(rng, n, zero_frac=zf, skew=skew)
    ref = orc.forest(w, m=m)
    K, aux = expected_cells(ref)
    u = np.concatenate([critical_u(ref.key, ref.W[0], m, rng=rng),
                        rng.integers(0, TWO64, 4000, dtype=np.uint64)])
    want, _ = orc.search(w, u, want_x=False)
    got = model_sample(ref, K, aux, u)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} samples differ, first u={u[bad[:3]]}"


def test_record_paths_all_taken(orc):
    """The cases above exercise covered cells, records that hold the whole
    cell, and cells whose tree is descended from aux."""
    rng = np.random.default_rng(5)
    ref = orc.forest(random_weights(rng, 5000), m=1000)
    K, aux = expected_cells(ref)
    node = ref.table >= 0
    assert (node & (aux < 0)).any() and (node & (aux >= 0)).any()
    ref2 = orc.forest(random_weights(rng, 3000, zero_frac=0.3, skew=True), m=6000)
    assert (ref2.table < 0).any()
