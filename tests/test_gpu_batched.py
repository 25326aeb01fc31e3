"""GPU parity for many distributions at once (Sec. 5): batched builds and
samples, the two-dimensional inversion, and the adjoint of x."""
import ctypes

import numpy as np
import pytest

from gpu_util import assert_forest, assert_samples, note, random_weights, to_dev

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


def check_batched(rtf, orc, ws, cells, sample_counts, seed, tile=0):
    rng = np.random.default_rng(seed)
    w = np.concatenate(ws)
    eo = offsets([a.size for a in ws])
    co = offsets(cells)
    f = rtf.build_batched(to_dev(w), to_dev(eo), to_dev(co), tile=tile)
    f.check()
    assert f.desc.tile == (tile or 2048)
    ref = orc.forest(w, elem_off=eo, cell_off=co)
    assert_forest(f, ref, f"D={len(ws)}")
    so = offsets(sample_counts)
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
    idx, x = idx.cpu().numpy(), x.cpu().numpy()
    idx_only, none = rtf.sample_batched(f, to_dev(so), to_dev(u), want_x=False)
    assert none is None and np.array_equal(idx_only.cpu().numpy(), idx)
    for d, wd in enumerate(ws):
        a, b = so[d], so[d + 1]
        if a == b:
            continue
        i_ref, x_ref = orc.search(wd, u[a:b])
        assert_samples(idx[a:b], x[a:b], i_ref, x_ref)
    return f


# the build tiles the tuner chooses from (0: the default, 2048 elements)
TILES = [0, 1024]


@pytest.mark.parametrize("tile", TILES)
def test_batched_random_sizes(rtf, orc, tile):
    note(f"batched D=60 random sizes tile={tile}")
    rng = np.random.default_rng(21)
    sizes = rng.integers(1, 6000, 60)
    sizes[:5] = [1, 1, 2, 4096, 4097]
    ws = [random_weights(rng, int(s), zero_frac=[0, 0.3, 0.95][k % 3], skew=k % 2 == 0)
          for k, s in enumerate(sizes)]
    for k in (7, 19):
        ws[k][-3:] = 0  # trailing zeros inside the batch
        if ws[k].sum() == 0:
            ws[k][0] = 1
    cells = [max(1, int(s * r)) for s, r in zip(sizes, rng.uniform(0.01, 3, 60))]
    counts = rng.integers(0, 3000, 60)
    counts[3] = 0
    counts[10:13] = 0
    check_batched(rtf, orc, ws, cells, counts, 1, tile)


@pytest.mark.parametrize("tile", TILES)
def test_batched_tile_straddling(rtf, orc, tile):
    """Distributions that start and end at and around the edges of 1024- and
    2048-element tiles."""
    note(f"batched straddling tiles tile={tile}")
    rng = np.random.default_rng(22)
    sizes = [4095, 1, 4096, 2, 8190, 1, 1, 1, 12289, 3, 4096, 4096, 1023, 1, 1024, 2047, 1025]
    ws = [random_weights(rng, s, zero_frac=0.1) for s in sizes]
    cells = [s for s in sizes]
    cells[4] = 1
    cells[8] = 50000
    check_batched(rtf, orc, ws, cells, [500] * len(sizes), 2, tile)


def test_batched_zero_distribution(rtf, orc):
    note("batched with an all-zero distribution")
    import paper_1901_05423_amd as rtfm
    rng = np.random.default_rng(23)
    ws = [random_weights(rng, 100), np.zeros(50, np.uint32), random_weights(rng, 70)]
    w = np.concatenate(ws)
    eo, co = offsets([100, 50, 70]), offsets([100, 50, 70])
    f = rtf.build_batched(to_dev(w), to_dev(eo), to_dev(co))
    with pytest.raises(rtfm.RtfError):
        f.check()
    so = offsets([10, 10, 10])
    u = rng.integers(0, 2 ** 64, 30, dtype=np.uint64)
    idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
    idx = idx.cpu().numpy()
    assert (idx[10:20] == -1).all() and np.isnan(x.cpu().numpy()[10:20]).all()
    for d in (0, 2):
        i_ref, _ = orc.search(ws[d], u[10 * d:10 * d + 10])
        assert np.array_equal(idx[10 * d:10 * d + 10], i_ref)


@pytest.mark.parametrize("tile", TILES)
def test_batched_many_tiny(rtf, orc, tile):
    """Thousands of tiny distributions with a few uniforms each, so that a
    chunk of the sampling kernel spans more distributions than it can stage
    and its lanes walk the offsets; some get no uniform at all."""
    note(f"batched D=3000 tiny tile={tile}")
    rng = np.random.default_rng(25)
    sizes = rng.integers(1, 6, 3000)
    ws = [random_weights(rng, int(s)) for s in sizes]
    counts = rng.integers(0, 4, 3000)
    counts[1000:1100] = 300  # a stretch that chunks can stage
    check_batched(rtf, orc, ws, [int(s) for s in sizes], counts, 4, tile)


def dist_records(f):
    """The per-distribution parameter records as the build stored them, 64
    bytes each: W, the reciprocal v, the global prefix G0, first element, n,
    first cell, m, then the 32-bit normalisation shift and the flags."""
    import torch
    off = f.desc.dists - f.ws.data_ptr()
    return f.ws[off:off + 64 * f.D].view(torch.int64).view(f.D, 8).cpu().numpy().view(np.uint64)


def expected_params(w, eo, co):
    """The same records from their definitions, in Python integers: W the sum
    of the distribution's weights, s = clz64(W), v = floor((2^128 - 1) /
    (W << s)) - 2^64 (the 2-by-1 reciprocal of Moller and Granlund), G0 the
    sum of all weights before the distribution."""
    rows, G = [], 0
    for d in range(len(eo) - 1):
        W = int(w[eo[d]:eo[d + 1]].astype(np.uint64).sum())
        s = 64 - W.bit_length()
        v = ((1 << 128) - 1) // (W << s) - (1 << 64)
        rows.append([W, v, G, int(eo[d]), int(eo[d + 1] - eo[d]), int(co[d]),
                     int(co[d + 1] - co[d]), s])
        G += W
    return rows


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("D", [1, 700, 2500])
def test_dist_params_against_definition(rtf, D, tile):
    """Each distribution's total, reciprocal, normalisation and global prefix,
    bit for bit: one distribution of 2^20 weights (its own parameter path),
    up to 1024 distributions (one thread each in the scan block) and more (a
    kernel of their own).  The weights span every magnitude from 1 to
    2^32 - 1, so the totals cover 1 to about 2^51, W = 1 (v = 2^64 - 1) among
    them."""
    note(f"parameters D={D} tile={tile}")
    rng = np.random.default_rng(90 + D)
    sizes = rng.integers(1, 3000, D) if D > 1 else [1 << 20]
    ws = []
    for k, sz in enumerate(sizes):
        bits = int(rng.integers(1, 33)) if D > 1 else 32
        ws.append(rng.integers(0, 2 ** bits, int(sz), dtype=np.uint64).astype(np.uint32))
        if ws[-1].sum() == 0:
            ws[-1][0] = 1
    specials = [[1], [3], [2 ** 32 - 1], [1, 0, 0], [2 ** 31, 2 ** 31], [2 ** 32 - 1] * 2999]
    for k, sp in enumerate(specials if D > 1 else []):
        ws[k] = np.array(sp, np.uint32)
    w = np.concatenate(ws)
    eo = offsets([a.size for a in ws])
    co = offsets([max(1, a.size // 4) for a in ws])
    if D == 1:
        f = rtf.build(to_dev(w), int(co[-1]), tile=tile)
    else:
        f = rtf.build_batched(to_dev(w), to_dev(eo), to_dev(co), tile=tile)
    f.check()
    got = dist_records(f)
    want = expected_params(w, eo, co)
    for d in range(D):
        g = [int(x) for x in got[d, :7]] + [int(got[d, 7]) & 0xFFFFFFFF]
        assert g == want[d], f"distribution {d}: {g} != {want[d]}"


def test_batched_staged_cells(rtf, orc):
    """Batches with several samples per cell run the kernel that stages a
    distribution's cells in LDS: distributions of at most 1024 cells staged,
    one of 2000 cells read from global memory, a tiny one, a zero one."""
    note("batched staged cells")
    rng = np.random.default_rng(24)
    ws = [random_weights(rng, 3000, zero_frac=0.2), random_weights(rng, 5000, skew=True),
          random_weights(rng, 100), random_weights(rng, 4096)]
    ws[3][-50:] = 0
    check_batched(rtf, orc, ws, [700, 2000, 1, 1024], [300000, 200000, 5, 400003], 3)
    # with a distribution of zero total weight among them
    import paper_1901_05423_amd as rtfm
    ws = [ws[0], np.zeros(50, np.uint32), ws[3]]
    w = np.concatenate(ws)
    eo, co = offsets([3000, 50, 4096]), offsets([700, 16, 1024])
    f = rtf.build_batched(to_dev(w), to_dev(eo), to_dev(co))
    with pytest.raises(rtfm.RtfError):
        f.check()
    so = offsets([100000, 20000, 100000])
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
    idx, x = idx.cpu().numpy(), x.cpu().numpy()
    assert (idx[so[1]:so[2]] == -1).all() and np.isnan(x[so[1]:so[2]]).all()
    for d in (0, 2):
        i_ref, x_ref = orc.search(ws[d], u[so[d]:so[d + 1]])
        assert_samples(idx[so[d]:so[d + 1]], x[so[d]:so[d + 1]], i_ref, x_ref)


@pytest.mark.parametrize("ratio,tile", [(0.25, 0), (1.0, 0), (0.125, 1024)])
def test_c4_batched_uneven_full(rtf, orc, ratio, tile):
    """10,000 distributions, sizes log-uniform in [16, 65536], uniform or
    Pareto(1.2) weights, ceil(64 n_d / 1000) uniforms each; guide cells
    m_d = ratio n_d and the build tile as the tuner may pick them."""
    import torch
    from paper_1901_05423_amd import workloads as wl
    note(f"C4 batched D=10000 ratio={ratio} tile={tile}")
    r = wl.rng(wl.C4_BATCHED)
    v, eo, so = wl.batched_uneven(r)
    u = wl.uniforms(r, int(so[-1]))
    q_ref, s_ref = orc.quantize(v, eo)
    q, s = rtf.quantize(to_dev(v), to_dev(eo))
    assert np.array_equal(q.cpu().numpy(), q_ref)
    assert np.array_equal(s.cpu().numpy(), s_ref)
    note(f"C4 n_total={eo[-1]} S={so[-1]}: building")
    eod = to_dev(eo)
    cod = rtf.cells_like(eod, ratio)
    f = rtf.build_batched(q, eod, cod, tile=tile)
    f.check()
    ref = orc.forest(q_ref, elem_off=eo, cell_off=cod.cpu().numpy())
    note("C4 oracle forest done")
    assert_forest(f, ref, "C4")
    idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
    idx, x = idx.cpu().numpy(), x.cpu().numpy()
    note("C4 comparing samples")
    i_ref = np.empty_like(idx)
    x_ref = np.empty_like(x)
    for d in range(eo.size - 1):
        a, b = so[d], so[d + 1]
        i_ref[a:b], x_ref[a:b] = orc.search(q_ref[eo[d]:eo[d + 1]], u[a:b])
    assert_samples(idx, x, i_ref, x_ref)
    torch.cuda.synchronize()


def quantised_map(orc, img, marginal):
    R, C = img.shape
    v = np.concatenate([marginal, img.ravel()])
    eo = np.concatenate([[0, R], R + C * np.arange(1, R + 1)]).astype(np.int64)
    q, _ = orc.quantize(v, eo)
    return v, q, eo


def check_2d(rtf, orc, img, marginal, pairs, seed, zero_rows=False, ratio=1.0, tile=0):
    rng = np.random.default_rng(seed)
    R, C = img.shape
    v, q_ref, eo = quantised_map(orc, img, marginal)
    q, _ = rtf.quantize(to_dev(v), to_dev(eo))
    assert np.array_equal(q.cpu().numpy(), q_ref)
    eod = to_dev(eo)
    cod = rtf.cells_like(eod, ratio)
    f = rtf.build_batched(q, eod, cod, tile=tile)
    if zero_rows:  # an all-zero row is a distribution without mass
        import paper_1901_05423_amd as rtfm
        with pytest.raises(rtfm.RtfError):
            f.check()
    else:
        f.check()
    u2 = rng.integers(0, 2 ** 64, 2 * pairs, dtype=np.uint64)
    rc, xy = rtf.sample_2d(f, to_dev(u2))
    rc, xy = rc.cpu().numpy(), xy.cpu().numpy()
    rc_only, none = rtf.sample_2d(f, to_dev(u2), want_xy=False)
    assert none is None and np.array_equal(rc_only.cpu().numpy(), rc)
    r_ref, y_ref = orc.search(q_ref[:R], u2[0::2])
    assert_samples(rc[:, 0], xy[:, 0], r_ref, y_ref)
    c_ref = np.empty(pairs, np.int32)
    x_ref = np.empty(pairs)
    order = np.argsort(r_ref, kind="stable")
    rows, starts = np.unique(r_ref[order], return_index=True)
    bounds = list(starts) + [pairs]
    for k, row in enumerate(rows):
        sel = order[bounds[k]:bounds[k + 1]]
        lo = R + int(row) * C
        c_ref[sel], x_ref[sel] = orc.search(q_ref[lo:lo + C], u2[1::2][sel])
    assert_samples(rc[:, 1], xy[:, 1], c_ref, x_ref)
    return f, q_ref, eo, cod.cpu().numpy()


def test_2d_small_map(rtf, orc):
    note("2D 96x130")
    from paper_1901_05423_amd import workloads as wl
    img, marg = wl.map_2d(np.random.default_rng(31), rows=96, cols=130, spots=3)
    img[5] = 0  # an empty row is never picked
    marg = img.astype(np.float64).sum(axis=1).astype(np.float32)
    check_2d(rtf, orc, img, marg, 200000, 3, zero_rows=True)


def test_2d_two_pairs_per_lane(rtf, orc):
    """More pairs than the sampling grid has lanes (4M), an odd count: every
    lane takes two interleaved pairs per step and the last step is ragged."""
    note("2D 64x300, 9M pairs")
    from paper_1901_05423_amd import workloads as wl
    img, marg = wl.map_2d(np.random.default_rng(41), rows=64, cols=300, spots=2)
    check_2d(rtf, orc, img, marg, 9_000_001, 5)


@pytest.mark.parametrize("ratio,tile", [(0.25, 0), (1.0, 0), (0.25, 1024)])
def test_c3_2d_full_map(rtf, orc, ratio, tile):
    """4096 x 4096 log-normal(0, 1.5) map with 8 hot spots: forest of the
    marginal plus 4096 rows bit-exact at m_d = ratio n_d with the build tile
    the tuner may pick, 2^20 pairs checked."""
    from paper_1901_05423_amd import workloads as wl
    note(f"C3 2D 4096x4096 ratio={ratio} tile={tile}")
    img, marg = wl.map_2d(wl.rng(wl.C3_MAP_2D))
    f, q_ref, eo, co = check_2d(rtf, orc, img, marg, 1 << 20, 4, ratio=ratio, tile=tile)
    note("C3 samples match; comparing forest")
    assert_forest(f, orc.forest(q_ref, elem_off=eo, cell_off=co), "C3")


def check_grad(rtf, orc, D, n, per, check_dists, seed, ratio=1.0):
    import torch
    import paper_1901_05423_amd as rtfm
    from paper_1901_05423_amd import workloads as wl
    r = wl.rng(seed)
    z_h = wl.logits(r, D, n)
    u_h = wl.uniforms(r, D * per)
    z = torch.from_numpy(z_h).to("cuda:0").requires_grad_(True)
    v = torch.nn.functional.softplus(z).reshape(-1)
    eo = to_dev(np.arange(D + 1, dtype=np.int64) * n)
    so = to_dev(np.arange(D + 1, dtype=np.int64) * per)
    u = to_dev(u_h)
    x = rtfm.RTFSample.apply(v, u, eo, so, ratio)
    L = torch.sin(7.0 * x).sum()
    L.backward()
    gz = z.grad.detach().double().cpu().numpy()
    x_h = x.detach().cpu().numpy()
    v_h = v.detach().cpu().numpy()
    sig = 1.0 / (1.0 + np.exp(-z_h.astype(np.float64)))
    for d in check_dists:
        q, s = orc.quantize(v_h[d * n:(d + 1) * n])
        uu = u_h[d * per:(d + 1) * per]
        i_ref, x_ref = orc.search(q, uu)
        assert np.abs(x_h[d * per:(d + 1) * per] - x_ref).max() <= 1e-12
        g = 7.0 * np.cos(7.0 * x_ref)
        ref = orc.grad(q, s[0], uu, g) * sig[d]
        got = gz[d]
        err = np.abs(got - ref)
        assert err.max() <= 1e-4 * np.abs(ref).max(), (d, err.max(), np.abs(ref).max())
        assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)


def test_grad_small(rtf, orc):
    note("grad D=6 n=4096 2^16 each")
    check_grad(rtf, orc, 6, 4096, 1 << 16, range(6), 105)


def test_grad_uneven_raw(rtf, orc):
    """rtf_backward directly on an uneven batch, against the oracle."""
    note("grad uneven raw")
    import torch
    rng = np.random.default_rng(41)
    sizes = [1, 300, 4096, 5000, 17]
    vs = [(0.01 + rng.random(s)).astype(np.float32) for s in sizes]
    vs[2][100] = 0
    v = np.concatenate(vs)
    eo = offsets(sizes)
    counts = [100, 0, 30000, 20000, 5]
    so = offsets(counts)
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    g = rng.standard_normal(int(so[-1]))
    q, s = rtf.quantize(to_dev(v), to_dev(eo))
    eod = to_dev(eo)
    f = rtf.build_batched(q, eod, eod)
    ud, sod = to_dev(u), to_dev(so)
    idx, _ = rtf.sample_batched(f, sod, ud)
    gw = rtf.backward(f, ud, idx, to_dev(g), s, sample_off=sod).cpu().numpy()
    q_h, s_h = q.cpu().numpy(), s.cpu().numpy()
    for d in range(len(sizes)):
        a, b = eo[d], eo[d + 1]
        ref = orc.grad(q_h[a:b], s_h[d], u[so[d]:so[d + 1]], g[so[d]:so[d + 1]])
        got = gw[a:b]
        # a one-weight distribution has gradient exactly 0 (x = xi for any
        # weight); there the bar is absolute
        scale = max(np.abs(ref).max(), 1.0)
        assert np.abs(got - ref).max() <= 1e-9 * scale, d
    torch.cuda.synchronize()


def raw_grad(rtf, orc, vs, counts, seed):
    """rtf_backward on distributions vs with counts[d] uniforms each, every
    distribution against the oracle."""
    import torch
    rng = np.random.default_rng(seed)
    v = np.concatenate(vs).astype(np.float32)
    eo = offsets([x.size for x in vs])
    so = offsets(counts)
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    g = rng.standard_normal(int(so[-1]))
    eod = to_dev(eo)
    if len(vs) > 1:
        q, s = rtf.quantize(to_dev(v), eod)
        f = rtf.build_batched(q, eod, eod)
        sod = to_dev(so)
        ud = to_dev(u)
        idx, _ = rtf.sample_batched(f, sod, ud)
        gw = rtf.backward(f, ud, idx, to_dev(g), s, sample_off=sod).cpu().numpy()
    else:
        q, s = rtf.quantize(to_dev(v))
        f = rtf.build(q, v.size)
        ud = to_dev(u)
        idx, _ = rtf.sample(f, ud)
        gw = rtf.backward(f, ud, idx, to_dev(g), s).cpu().numpy()
    q_h, s_h = q.cpu().numpy(), s.cpu().numpy()
    for d in range(len(vs)):
        a, b = eo[d], eo[d + 1]
        ref = orc.grad(q_h[a:b], s_h[d], u[so[d]:so[d + 1]], g[so[d]:so[d + 1]])
        scale = max(np.abs(ref).max(), 1.0)
        assert np.abs(gw[a:b] - ref).max() <= 1e-9 * scale, d
    torch.cuda.synchronize()


def test_grad_block_paths(rtf, orc):
    """The three ways a scatter block runs: samples of one distribution of at
    most 4096 weights (partial sums staged in LDS, here with zero runs and
    trailing zeros, whose keys are all ones), of one larger distribution
    (keys read per sample), and of several distributions."""
    note("grad block paths")
    rng = np.random.default_rng(43)
    small = (0.01 + rng.random(3000)).astype(np.float32)
    small[500:700] = 0
    small[-40:] = 0
    raw_grad(rtf, orc, [small], [300000], 1)
    big = (0.01 + rng.random(10000)).astype(np.float32)
    big[-3:] = 0
    raw_grad(rtf, orc, [big], [300000], 2)
    mixed = [small, big, (0.5 + rng.random(100)).astype(np.float32), np.ones(4096, np.float32)]
    raw_grad(rtf, orc, mixed, [262149, 140000, 7, 131072], 3)


def test_grad_one_large_distribution(rtf, orc):
    """One distribution of 2^22 weights and 2^24 samples: the combining pass
    spreads it over 1024 chunks, each block adding the carry of the chunks
    after it."""
    note("grad one distribution n=2^22 S=2^24")
    rng = np.random.default_rng(47)
    v = (0.01 + rng.random(1 << 22)).astype(np.float32)
    v[1000:1100] = 0
    v[-5:] = 0
    raw_grad(rtf, orc, [v], [1 << 24], 4)


def test_grad_chunk_straddling(rtf, orc):
    """Distributions that begin and end at and around the combining pass's
    chunk edges (4096 elements), several inside one chunk and one over many."""
    note("grad chunk straddling")
    rng = np.random.default_rng(53)
    sizes = [4096, 4095, 1, 2, 8192 + 3, 1, 70000, 17, 4096 * 3 - 24, 5]
    vs = [(0.01 + rng.random(sz)).astype(np.float32) for sz in sizes]
    counts = [int(c) for c in rng.integers(0, 50000, len(sizes))]
    counts[3] = 0
    raw_grad(rtf, orc, vs, counts, 6)


def test_c5_grad_full(rtf, orc):
    """256 distributions of 4096 softplus(N(0,1)) weights, 2^20 uniforms each,
    1024 guide cells each (the sampling kernel stages them in LDS),
    L = sum sin(7x): dL/dlogits of 4 distributions checked against the oracle."""
    note("C5 grad D=256 n=4096 2^20 each")
    check_grad(rtf, orc, 256, 4096, 1 << 20, [0, 1, 128, 255], 5, ratio=0.25)


@pytest.fixture(scope="module")
def million_tiny(orc):
    """2^20 distributions of 1 to 8 float32 weights (one in ten zero, every
    distribution with mass), their oracle quantisation and guide offsets."""
    rng = np.random.default_rng(31)
    D = 1 << 20
    sizes = rng.integers(1, 9, D)
    eo = offsets(sizes)
    n = int(eo[-1])
    v = (1.0 - rng.random(n)).astype(np.float32)
    v[rng.random(n) < 0.1] = 0.0
    v[eo[:-1][np.add.reduceat(v, eo[:-1]) == 0]] = 0.5
    q_ref, s_ref = orc.quantize(v, eo)
    co = offsets(np.maximum(1, sizes // 2))
    return v, eo, co, q_ref, s_ref, rng


@pytest.mark.parametrize("tile", TILES)
def test_batched_million_tiny(rtf, orc, million_tiny, tile):
    """2^20 distributions of 1 to 8 weights each (4.7M weights): far more
    distributions than one block of any kernel holds, so the quantisation's
    blocks span hundreds of distributions each (global atomics), the
    parameters go through k_dist_finish, tiles hold hundreds of distribution
    starts, and sampling chunks walk the offsets.  Quantised weights, totals,
    forest and cell records bit-exact; the samples of 3000 distributions
    (the first, the last, and random ones) checked one by one."""
    import torch
    v, eo, co, q_ref, s_ref, rng0 = million_tiny
    note(f"batched D=2^20 tiny tile={tile}")
    rng = np.random.default_rng(32 + tile)
    D = eo.size - 1
    eod = to_dev(eo)
    q, s = rtf.quantize(to_dev(v), eod)
    assert np.array_equal(q.cpu().numpy(), q_ref)
    assert np.array_equal(s.cpu().numpy(), s_ref)
    f = rtf.build_batched(q, eod, to_dev(co), tile=tile)
    f.check()
    assert_forest(f, orc.forest(q_ref, elem_off=eo, cell_off=co), "D=2^20")
    counts = rng.integers(0, 4, D)
    so = offsets(counts)
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
    idx, x = idx.cpu().numpy(), x.cpu().numpy()
    for d in np.unique(np.concatenate([[0, D - 1], rng.integers(0, D, 3000)])):
        a, b = so[d], so[d + 1]
        if a < b:
            i_ref, x_ref = orc.search(q_ref[eo[d]:eo[d + 1]], u[a:b])
            assert_samples(idx[a:b], x[a:b], i_ref, x_ref)
    torch.cuda.synchronize()


def test_batched_offsets_out_of_rule(rtf, orc):
    """Sample offsets that break the rules (decreasing, not ending at S) give
    unspecified indices but bounded work: the call returns, every sample gets
    an index of some distribution (or -1) and an x in [0, 1]; both sampling
    kernels (LDS-staged cells and chunks) and the batched quantisation are
    run this way.  Valid offsets afterwards still give the oracle's answers."""
    import torch
    note("batched offsets out of rule")
    rng = np.random.default_rng(41)
    sizes = [3000, 50, 4096, 7, 1000]
    ws = [random_weights(rng, s) for s in sizes]
    w = np.concatenate(ws)
    eo, co = offsets(sizes), offsets([700, 10, 1024, 2, 250])
    f = rtf.build_batched(to_dev(w), to_dev(eo), to_dev(co))
    f.check()
    nmax = max(sizes)
    for S in (200000, 3000):  # many samples per cell (staged cells), few (chunks)
        u = rng.integers(0, 2 ** 64, S, dtype=np.uint64)
        for so in (np.array([0, S, S // 2, S // 3, 5, 1], np.int64),
                   np.array([0, 10, 20, 30, 40, 50], np.int64),
                   np.array([S, 0, S, 0, S, 0], np.int64)):
            idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
            torch.cuda.synchronize()
            idx, x = idx.cpu().numpy(), x.cpu().numpy()
            assert ((idx >= -1) & (idx < nmax)).all()
            ok = idx >= 0
            assert ((x[ok] >= 0) & (x[ok] <= 1)).all()
        so = offsets([S // 5] * 4 + [S - 4 * (S // 5)])
        idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
        idx, x = idx.cpu().numpy(), x.cpu().numpy()
        for d in range(5):
            i_ref, x_ref = orc.search(ws[d], u[so[d]:so[d + 1]])
            assert_samples(idx[so[d]:so[d + 1]], x[so[d]:so[d + 1]], i_ref, x_ref)
    v = (1.0 - rng.random(w.size)).astype(np.float32)
    for bad in (np.array([0, 9000, 100, 5000, 2, 1], np.int64), np.array([0, 1, 2, 3, 4, 5], np.int64)):
        q, s = rtf.quantize(to_dev(v), to_dev(bad))
        torch.cuda.synchronize()
        assert q.numel() == v.size and s.numel() == 5


def test_build_offsets_out_of_rule(rtf, orc):
    """Build offsets that break the rules (not increasing, not starting at 0,
    not ending at the totals) are reported by rtf_check as
    RTF_ERR_INVALID_ARG; the build and sampling on its forest stay in bounds
    and return.  The same workspace then builds valid offsets correctly."""
    import torch
    import paper_1901_05423_amd as rtfm
    note("build offsets out of rule")
    rng = np.random.default_rng(43)
    sizes = [500, 300, 900, 1200]
    ws = [random_weights(rng, s) for s in sizes]
    w = np.concatenate(ws)
    n, D = w.size, len(sizes)
    eo_ok, co_ok = offsets(sizes), offsets([100, 100, 100, 100])
    bad_cases = [
        (np.array([0, 500, 300, 1800, n], np.int64), co_ok),   # not increasing
        (eo_ok, np.array([0, 100, 100, 300, 400], np.int64)),  # repeated cell offset
        (np.array([7, 500, 800, 1700, n], np.int64), co_ok),   # not starting at 0
        (np.array([0, 500, 800, 1700, n - 1], np.int64), co_ok),  # not ending at n_total
    ]
    wd = to_dev(w)
    so = offsets([1000] * D)
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    for eo, co in bad_cases:
        nb = rtf.lib().rtf_workspace_bytes_batched(D, n, int(co_ok[-1]))
        wsp = torch.empty(nb, dtype=torch.uint8, device="cuda")
        desc = rtfm.rtf_forest()
        eod, cod = to_dev(eo), to_dev(co)
        rtfm._check(rtf.lib().rtf_build_batched(rtfm._ptr(wd), rtfm._ptr(eod), rtfm._ptr(cod), D, n,
                                                int(co_ok[-1]), rtfm._ptr(wsp), nb, rtfm._stream(),
                                                ctypes.byref(desc)), "rtf_build_batched")
        f = rtfm.Forest(wsp, desc, wd.device)
        with pytest.raises(rtfm.RtfError) as e:
            f.check()
        assert e.value.code == rtf.RTF_ERR_INVALID_ARG
        idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
        torch.cuda.synchronize()
        assert (idx.cpu().numpy() >= -1).all()
    check_batched(rtf, orc, ws, [100] * D, [1000] * D, 5)
