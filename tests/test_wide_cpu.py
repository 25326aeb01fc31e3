"""The collapsed 4-ary records (two binary levels per record, Sec. 5) and the
key tracking of the descent, checked on the CPU: records derived from the
oracle forest (the layout rtf_forest_widen must write) resolve every sample
to the oracle's binary-search index, the descent meets the sampled interval's
two bounds U_i and U_{i+1} (so the position needs no further read unless i is
its cell's last leaf), and it reads about half the records of the binary
descent."""
import numpy as np
import pytest

from gpu_util import (CELL_BOUNDS, CELL_KEYS, TWO64, critical_u, expected_cells, expected_wide,
                      random_weights)

MAX = TWO64 - 1


def unpack(rows):
    r = {}
    for q, (lo, hi) in enumerate(((3, 0), (3, 1), (4, 0), (4, 1))):
        v = (rows[:, lo] >> (32 * hi)) & 0xFFFFFFFF
        r[q] = np.where(v >= 1 << 31, v - (1 << 32), v).astype(np.int64)
    return r


def model(ref, K, aux, wide, u, collapsed):
    """Resolve uniforms of one distribution the way the sampling kernel does:
    (index, lower key, upper key, records read after the cell record, whether
    the upper key had to be read after the descent)."""
    key, child, table = ref.key, ref.child, ref.table
    m, n = table.size, key.size
    out = []
    for us in u.tolist():
        g = (us * m) >> 64
        t = int(table[g])
        if t < 0:
            out.append((~t, None, None, 0, False))
            continue
        a = int(aux[g])
        if a < 0 or us < int(K[g, CELL_KEYS - 1]):
            lim = ~a if a < 0 else CELL_BOUNDS
            j = sum(1 for q in range(1, lim + 1) if int(K[g, q]) <= us)
            out.append((t - 1 + j, None, None, 0, False))
            continue
        klo, khi, reads, jn = int(K[g, CELL_KEYS - 1]), None, 0, a
        while jn >= 0:
            reads += 1
            if collapsed:
                k, kc0, kc1, r = wide[jn]
                right = us >= k
                if right:
                    klo = k
                else:
                    khi = k
                g0, g1 = (r[2], r[3]) if right else (r[0], r[1])
                kc = kc1 if right else kc0
                if g0 == g1:
                    jn = g0
                    continue
                if us >= kc:
                    klo, jn = kc, g1
                else:
                    khi, jn = kc, g0
            else:
                k = int(key[jn])
                if us >= k:
                    klo, jn = k, int(child[jn, 1])
                else:
                    khi, jn = k, int(child[jn, 0])
        i = ~jn
        late = khi is None
        if late:
            khi = int(key[i + 1]) if i + 1 < n else MAX
        out.append((i, klo, khi, reads, late))
    return out


CASES = [
    (5000, 400, 0.1, False),
    (20000, 1000, 0.0, False),
    (3000, 6000, 0.3, True),
    (2048, 1, 0.0, False),
    (4000, 3, 0.5, True),
]


@pytest.mark.parametrize("n,m,zf,skew", CASES)
def test_collapsed_records_resolve_like_binary_search(orc, n, m, zf, skew):
    rng = np.random.default_rng(n * 3 + m)
    w = random_weights(rng, n, zero_frac=zf, skew=skew)
    ref = orc.forest(w, m=m)
    K, aux = expected_cells(ref)
    j, rows = expected_wide(ref)
    r = unpack(rows)
    wide = {int(j[q]): (int(rows[q, 0]) % TWO64, int(rows[q, 1]) % TWO64,
                        int(rows[q, 2]) % TWO64, [int(r[t][q]) for t in range(4)])
            for q in range(j.size)}
    u = np.concatenate([critical_u(ref.key, ref.W[0], m, rng=rng),
                        rng.integers(0, TWO64, 3000, dtype=np.uint64)])
    want, _ = orc.search(w, u, want_x=False)
    key = [int(k) for k in ref.key]
    binary = model(ref, K, aux, wide, u, collapsed=False)
    wide_m = model(ref, K, aux, wide, u, collapsed=True)
    for res in (binary, wide_m):
        got = np.array([x[0] for x in res])
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"{bad.size} samples differ, first u={u[bad[:3]]}"
        for (i, klo, khi, _, _) in res:
            if klo is not None:  # a descent: the bounds it met are the interval's
                assert klo == key[i]
                assert khi == (key[i + 1] if i + 1 < n else MAX)
    rb = sum(x[3] for x in binary)
    rw = sum(x[3] for x in wide_m)
    if rb > 100:
        assert rw <= 0.65 * rb, (rw, rb)
    # the upper key is read after the descent only for a cell's last leaf
    for (i, klo, _, _, late) in binary:
        if late:
            g_i = (key[i] * m) >> 64
            assert i + 1 >= n or key[i + 1] == MAX or ((key[i + 1] * m) >> 64) != g_i
