"""GPU parity of the Alias Method (Sec. 2.6), the comparison mapping of the
quality study: tables bit for bit against the oracle's Vose construction,
indices against the oracle's exact sampling rule, 2D pairs, and the
quadratic error of Fig. convergence on Hammersley points for both mappings
(counts computed on the GPU equal counts from the oracle's indices)."""
import numpy as np
import pytest

from gpu_util import note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1901_05423_amd as rtf
    rtf.lib()
    return rtf


def offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def test_alias_tables_and_samples_batched(rtf, orc):
    note("alias: batched tables and samples")
    rng = np.random.default_rng(91)
    ws = [np.array([5], np.uint32), np.full(17, 3, np.uint32),
          rng.integers(0, 2 ** 32, 1000, dtype=np.uint64).astype(np.uint32),
          rng.integers(1, 2 ** 12, 4096, dtype=np.uint64).astype(np.uint32),
          np.array([0, 0, 9, 0, 1], np.uint32)]
    ws[2][::7] = 0
    w = np.concatenate(ws)
    eo = offsets([x.size for x in ws])
    t = rtf.alias_build(to_dev(w), to_dev(eo))
    thr, alias, W = t.export()
    counts = [1000, 0, 50000, 70000, 3000]
    so = offsets(counts)
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    u[:8] = [0, 2 ** 64 - 1, 1, 2 ** 63, 2 ** 63 - 1, 12345, 2 ** 62, 3 * 2 ** 62]
    idx = rtf.alias_sample(t, to_dev(u), to_dev(so)).cpu().numpy()
    for d, wd in enumerate(ws):
        ref = orc.alias_build(wd)
        a, b = eo[d], eo[d + 1]
        assert int(W[d]) == ref.W, d
        assert np.array_equal(thr[a:b], ref.thr), d
        assert np.array_equal(alias[a:b], ref.alias), d
        s0, s1 = so[d], so[d + 1]
        assert np.array_equal(idx[s0:s1], orc.alias_sample(ref, u[s0:s1])), d


def test_alias_zero_total(rtf):
    note("alias: zero total")
    import torch
    w = to_dev(np.array([1, 2, 0, 0], np.uint32))
    eo = to_dev(np.array([0, 2, 4], np.int64))
    t = rtf.alias_build(w, eo)
    with pytest.raises(rtf.RtfError):
        t.export()
    so = to_dev(np.array([0, 3, 6], np.int64))
    idx = rtf.alias_sample(t, to_dev(np.arange(6, dtype=np.uint64) << np.uint64(60)), so)
    torch.cuda.synchronize()
    assert (idx.cpu().numpy()[3:] == -1).all()


def test_alias_2d_marginal_longer_than_rows(rtf):
    """A marginal with more items than there are row tables: a pair whose row
    has no table gets (-1, -1) instead of reading past the offsets."""
    note("alias: 2D with a marginal longer than the rows")
    import torch
    w = to_dev(np.array([1, 1, 1, 1, 5, 6, 7, 8], np.uint32))  # marginal of 4, two rows of 2
    eo = to_dev(np.array([0, 4, 6, 8], np.int64))
    t = rtf.alias_build(w, eo)
    u2 = to_dev((np.arange(2048, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)))
    rc = rtf.alias_sample_2d(t, u2).cpu().numpy()
    torch.cuda.synchronize()
    # marginal items 2 and 3 (half the mass) have no row table
    assert ((rc[:, 0] == -1) | (rc[:, 0] < 2)).all()
    assert ((rc[:, 0] == -1) == (rc[:, 1] == -1)).all()
    assert 0 < (rc[:, 0] == -1).sum() < rc.shape[0]
    ok = rc[:, 0] >= 0
    assert ((rc[ok, 1] >= 0) & (rc[ok, 1] < 2)).all()


def small_map(rng, R, C):
    from paper_1901_05423_amd import workloads as wl
    img, marg = wl.map_2d(rng, rows=R, cols=C, spots=2)
    return img, marg


def test_alias_2d_and_quadratic_error(rtf, orc):
    """A 64 x 96 map sampled with 2^12 Hammersley points through the forest
    (the inverse mapping) and the alias tables: GPU pairs equal the oracle's
    (binary search per component; alias rule per component), and the
    quadratic error e = sum (p_i - c_i / N)^2 from GPU counts equals the
    oracle's.  At this size the inverse mapping already has the smaller e."""
    note("alias: 2D pairs and the quadratic error, 64 x 96, N = 2^12")
    import torch
    from paper_1901_05423_amd import workloads as wl
    rng = np.random.default_rng(93)
    R, C = 64, 96
    img, marg = small_map(rng, R, C)
    v = np.concatenate([marg, img.ravel()])
    eo = np.concatenate([[0, R], R + C * np.arange(1, R + 1)]).astype(np.int64)
    q, _ = orc.quantize(v, eo)
    qd, eod = to_dev(q), to_dev(eo)
    N = 1 << 12
    u2 = wl.hammersley_u64(N)
    u2d = to_dev(u2)
    f = rtf.build_batched(qd, eod, eod)
    t = rtf.alias_build(qd, eod)
    rc_inv, _ = rtf.sample_2d(f, u2d, want_xy=False)
    rc_al = rtf.alias_sample_2d(t, u2d)
    torch.cuda.synchronize()
    rc_inv, rc_al = rc_inv.cpu().numpy(), rc_al.cpu().numpy()
    # the oracle's pairs
    marg_t = orc.alias_build(q[:R])
    rows_t = [orc.alias_build(q[R + r * C:R + (r + 1) * C]) for r in range(R)]
    r_inv, _ = orc.search(q[:R], u2[:, 0], want_x=False)
    r_al = orc.alias_sample(marg_t, u2[:, 0])
    c_inv = np.array([orc.search(q[R + r * C:R + (r + 1) * C], u2[s:s + 1, 1], want_x=False)[0][0]
                      for s, r in enumerate(r_inv)], np.int32)
    c_al = np.array([orc.alias_sample(rows_t[r], u2[s:s + 1, 1])[0] for s, r in enumerate(r_al)],
                    np.int32)
    assert np.array_equal(rc_inv[:, 0], r_inv) and np.array_equal(rc_inv[:, 1], c_inv)
    assert np.array_equal(rc_al[:, 0], r_al) and np.array_equal(rc_al[:, 1], c_al)
    # exact probabilities of the quantised map
    qm = q[:R].astype(np.float64)
    rows = q[R:].astype(np.float64).reshape(R, C)
    p = (qm / qm.sum())[:, None] * rows / rows.sum(axis=1, keepdims=True)
    e = {}
    for name, rc in (("inverse", rc_inv), ("alias", rc_al)):
        cnt = np.bincount(rc[:, 0].astype(np.int64) * C + rc[:, 1], minlength=R * C)
        e[name] = orc.quadratic_error(p.ravel(), cnt, N)
    assert e["inverse"] < e["alias"], e
