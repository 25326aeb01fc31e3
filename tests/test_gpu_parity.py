"""GPU parity: one distribution, built and sampled through the C ABI, against
the CPU oracle.  Forests, guide tables and indices bit-exact; x within 1e-12
(the method's bar is 1e-6)."""
import numpy as np
import pytest

from gpu_util import (X_TOL, assert_forest, assert_samples, critical_u, note, random_weights,
                      to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1901_05423_amd as rtf
    rtf.lib()
    return rtf


def build_and_compare(rtf, orc, w, m, S_extra=20000, seed=0, baselines=True, tile=0):
    rng = np.random.default_rng(seed)
    f = rtf.build(to_dev(w), m, tile=tile)
    f.check()
    assert f.desc.tile == (tile or 2048)
    ref = orc.forest(w, m=m)
    assert_forest(f, ref, f"n={w.size} m={m}")
    u = critical_u(ref.key, int(ref.W[0]), m, extra=S_extra, rng=rng)
    ud = to_dev(u)
    i_ref, x_ref = orc.search(w, u)
    idx, x = rtf.sample(f, ud)
    assert_samples(idx.cpu().numpy(), x.cpu().numpy(), i_ref, x_ref)
    idx_only, none = rtf.sample(f, ud, want_x=False)
    assert none is None and np.array_equal(idx_only.cpu().numpy(), i_ref)
    if baselines:
        for fn in (rtf.sample_bsearch, rtf.sample_cutpoint_bsearch):
            bi, bx = fn(f, ud)
            assert_samples(bi.cpu().numpy(), bx.cpu().numpy(), i_ref, x_ref)
    return f


def test_c1_uniform_1k(rtf, orc):
    """n=1024 uniform(0,1] weights, quantised on the GPU, m=1024, 2^16 uniforms."""
    import torch
    from paper_1901_05423_amd import workloads as wl
    note("C1 n=1024 m=1024 S=65536")
    r = wl.rng(wl.C1_UNIFORM_1K)
    v = wl.weights_uniform(r, 1024)
    u = wl.uniforms(r, 1 << 16)
    q_ref, s_ref = orc.quantize(v)
    q, s = rtf.quantize(to_dev(v))
    assert np.array_equal(q.cpu().numpy(), q_ref)
    assert s.cpu().numpy()[0] == s_ref[0]
    f = rtf.build(q, 1024)
    assert_forest(f, orc.forest(q_ref, m=1024))
    idx, x = rtf.sample(f, to_dev(u))
    i_ref, x_ref = orc.search(q_ref, u)
    assert_samples(idx.cpu().numpy(), x.cpu().numpy(), i_ref, x_ref)
    torch.cuda.synchronize()


CASES = [
    # (n, m, zero_frac, skew, trailing_zeros)
    (1, 1, 0.0, False, 0),
    (1, 5, 0.0, False, 0),
    (2, 1, 0.0, False, 0),
    (3, 2, 0.5, True, 0),
    (17, 17, 0.0, False, 3),
    (100, 1, 0.0, True, 0),
    (100, 300, 0.3, False, 0),
    (4095, 4095, 0.0, False, 0),
    (4096, 4096, 0.0, True, 0),
    (4097, 4097, 0.2, False, 5),
    (3 * 4096 + 5, 1, 0.0, False, 0),
    (3 * 4096 + 5, 7, 0.0, True, 0),
    (3 * 4096 + 5, 3 * (3 * 4096 + 5), 0.1, False, 0),
    (70001, 70001, 0.0, False, 0),
    (70001, 65536, 0.9, True, 40),
    (70001, 100, 0.5, False, 0),
    (200003, 200003, 0.0, True, 0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_m%d_z%g_s%d_t%d" % (
    c[0], c[1], c[2], c[3], c[4]))
def test_forest_and_samples(rtf, orc, case):
    n, m, zf, skew, trail = case
    note(f"single n={n} m={m} zeros={zf} skew={skew} trailing={trail}")
    rng = np.random.default_rng(n * 7919 + m)
    w = random_weights(rng, n, zero_frac=zf, skew=skew)
    if trail:
        w[-trail:] = 0
        if w.sum() == 0:
            w[0] = 5
    build_and_compare(rtf, orc, w, m, seed=n + m)


def test_leading_zero_runs_and_duplicates(rtf, orc):
    """Long runs of zero weights make runs of equal keys (ties in the levels)."""
    note("zero runs n=50000")
    rng = np.random.default_rng(99)
    n = 50000
    w = random_weights(rng, n)
    w[:3000] = 0
    w[10000:14000] = 0
    w[20000:20100] = 0
    w[-5000:] = 0
    for m in (1, 1000, n):
        build_and_compare(rtf, orc, w, m, seed=m)


def test_single_heavy_interval(rtf, orc):
    """One interval covering most cells: long guide-table runs."""
    note("heavy interval n=20000")
    rng = np.random.default_rng(5)
    w = random_weights(rng, 20000, skew=False) // 1000
    w[1234] = 4000000000
    w[17] = 4000000000
    build_and_compare(rtf, orc, w, 20000)
    build_and_compare(rtf, orc, w, 3 * 20000 + 1)


def test_zero_total_is_reported(rtf, orc):
    note("all-zero weights")
    import paper_1901_05423_amd as rtfm
    w = np.zeros(100, np.uint32)
    f = rtf.build(to_dev(w), 10)
    with pytest.raises(rtfm.RtfError) as e:
        f.check()
    assert e.value.code == rtfm.RTF_ERR_ZERO_TOTAL
    idx, x = rtf.sample(f, to_dev(np.array([0, 5, 2 ** 63], np.uint64)))
    assert (idx.cpu().numpy() == -1).all() and np.isnan(x.cpu().numpy()).all()


def test_quantize_value_errors(rtf, orc):
    note("quantize negative")
    import torch
    import paper_1901_05423_amd as rtfm
    st = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    v = np.array([1.0, 2.0, -1.0, 0.0], np.float32)
    q, _ = rtf.quantize(to_dev(v), status=st)
    assert int(st.item()) & (1 << rtfm.RTF_ERR_VALUE)
    assert q.cpu().numpy()[2] == 0


def test_quantize_parity_batched(rtf, orc):
    note("quantize batched")
    rng = np.random.default_rng(3)
    sizes = [1, 4096, 17, 5000, 3, 40000]
    v = np.concatenate([rng.random(s).astype(np.float32) * 10 ** rng.uniform(-3, 3)
                        for s in sizes])
    v[::31] = 0
    eo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    q_ref, s_ref = orc.quantize(v, eo)
    q, s = rtf.quantize(to_dev(v), to_dev(eo))
    assert np.array_equal(q.cpu().numpy(), q_ref)
    assert np.array_equal(s.cpu().numpy(), s_ref)


@pytest.mark.parametrize("batched", [False, True])
def test_quantize_negative_zero(rtf, orc, batched):
    """-0.0 passes the sign test but is a zero weight: it must neither set a
    distribution's maximum nor raise an error."""
    import torch
    note(f"quantize -0.0 batched={batched}")
    rng = np.random.default_rng(5)
    sizes = [5000, 3, 70000, 1, 9]
    v = np.concatenate([rng.random(s).astype(np.float32) for s in sizes])
    v[::3] = -0.0
    v[4] = np.float32(-0.0)
    eo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    st = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    if batched:
        q_ref, s_ref = orc.quantize(v, eo)
        q, s = rtf.quantize(to_dev(v), to_dev(eo), status=st)
    else:
        q_ref, s_ref = orc.quantize(v)
        q, s = rtf.quantize(to_dev(v), status=st)
    assert int(st.item()) == 0
    assert np.array_equal(s.cpu().numpy(), s_ref)
    assert np.array_equal(q.cpu().numpy(), q_ref)


@pytest.mark.parametrize("n", [1, 4096, 4097, (1 << 20) + 3])
def test_quantize_single_scale_extremes(rtf, orc, n):
    """One distribution's scale, which the apply pass writes while its other
    blocks still read the maximum: bit for bit against the oracle for the
    largest float maximum (the smallest scale, about 1.3e-29), a subnormal
    maximum, an ordinary one and all-zero weights (scale 0), each quantised
    twice into the same buffers (the second call starts from the first's
    scale)."""
    import torch
    note(f"quantise one distribution n={n}")
    rng = np.random.default_rng(n)
    base = rng.random(n).astype(np.float32)
    cases = {
        "flt_max": base * np.float32(3.4028235e38),
        "subnormal": (base * np.float32(1e-40)).astype(np.float32),
        "ordinary": base,
        "zero": np.zeros(n, np.float32),
    }
    cases["flt_max"][n // 2] = np.float32(3.4028235e38)
    q = torch.empty(n, dtype=torch.uint32, device="cuda:0")
    s = torch.empty(1, dtype=torch.float64, device="cuda:0")
    for name, v in cases.items():
        q_ref, s_ref = orc.quantize(v)
        vd = to_dev(v)
        for _ in range(2):
            rtf.quantize(vd, out=(q, s))
            torch.cuda.synchronize()
            assert s.cpu().numpy()[0] == s_ref[0], name
            assert np.array_equal(q.cpu().numpy(), q_ref), name


def test_deterministic_rebuild(rtf, orc):
    note("determinism n=300000")
    rng = np.random.default_rng(11)
    w = random_weights(rng, 300000, zero_frac=0.05, skew=True)
    wd = to_dev(w)
    f1 = rtf.build(wd, 300000)
    a = f1.export()
    for _ in range(5):
        f2 = rtf.build(wd, 300000)
        b = f2.export()
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_c2_zipf_2e20_full_forest(rtf, orc):
    """n=2^20, p_i ~ (i+1)^-1.1 permuted, m=n: forest bit-exact, 2^22 uniforms."""
    import torch
    from paper_1901_05423_amd import workloads as wl
    note("C2 zipf n=2^20 m=2^20")
    r = wl.rng(wl.C2_ZIPF_1M)
    n = 1 << 20
    v = wl.weights_zipf(r, n)
    u = wl.uniforms(r, 1 << 22)
    q_ref, _ = orc.quantize(v)
    q, _ = rtf.quantize(to_dev(v))
    assert np.array_equal(q.cpu().numpy(), q_ref)
    f = rtf.build(q, n)
    assert_forest(f, orc.forest(q_ref, m=n), "C2")
    idx, x = rtf.sample(f, to_dev(u))
    i_ref, x_ref = orc.search(q_ref, u)
    assert_samples(idx.cpu().numpy(), x.cpu().numpy(), i_ref, x_ref)
    torch.cuda.synchronize()


# The benchmark sizes the guide table with the autotuner, which picks among
# these ratios m/n (paper_1901_05423_amd/tune.py); every candidate is checked
# at full size for the uniform workload, the usual picks for the Zipf one.
# The tuner also picks the build tile; both tiles are checked at the usual
# ratio.
H24_CASES = [("uniform", r, 0) for r in (0.25, 0.125, 0.5, 1.0, 2.0)] + \
            [("zipf", r, 0) for r in (0.25, 0.125, 1.0)] + \
            [("uniform", 0.25, 1024), ("zipf", 0.25, 1024)]


@pytest.mark.parametrize("kind,ratio,tile", H24_CASES)
def test_h24_full_size(rtf, orc, kind, ratio, tile):
    """The benchmark's workload and launch configuration: n = 2^24, m = ratio n,
    all S = 2^26 uniforms sampled in one call as the benchmark does.  Forest,
    guide table and cell records bit-exact against the oracle's; every 16th
    sample (2^22 of them) checked one by one."""
    import torch
    from paper_1901_05423_amd import workloads as wl
    n = 1 << 24
    m = max(1, int(round(ratio * n)))
    note(f"H24 {kind} n=2^24 m={m} tile={tile} S=2^26")
    r = wl.rng(wl.H24_UNIFORM if kind == "uniform" else wl.H24_ZIPF)
    v = wl.weights_uniform(r, n) if kind == "uniform" else wl.weights_zipf(r, n)
    u = wl.uniforms(r, 1 << 26)
    q_ref, _ = orc.quantize(v)
    q, _ = rtf.quantize(to_dev(v))
    assert np.array_equal(q.cpu().numpy(), q_ref)
    note("H24 quantised weights match; building")
    f = rtf.build(q, m, tile=tile)
    f.check()
    ref = orc.forest(q_ref, m=m)
    note("H24 oracle forest done; comparing")
    assert_forest(f, ref, "H24")
    note("H24 forest matches; sampling")
    ud = to_dev(u)
    idx, x = rtf.sample(f, ud)
    sel = slice(0, None, 16)
    i_ref, x_ref = orc.search(q_ref, u[sel])
    assert_samples(idx[sel].cpu().numpy(), x[sel].cpu().numpy(), i_ref, x_ref)
    # the index-only instance and both same-GPU baselines at the same size
    idx2, _ = rtf.sample(f, ud, want_x=False)
    assert torch.equal(idx2, idx)
    for fn in (rtf.sample_bsearch, rtf.sample_cutpoint_bsearch):
        bi, bx = fn(f, ud)
        assert torch.equal(bi, idx) and float((bx - x).abs().max()) <= X_TOL
    torch.cuda.synchronize()


@pytest.mark.parametrize("seed", range(24))
def test_random_shapes(rtf, orc, seed):
    """Random sizes, guide sizes and zero patterns against the oracle."""
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.choice([rng.integers(1, 300), rng.integers(300, 9000),
                        rng.integers(9000, 120000)]))
    ratio = float(rng.choice([0.01, 0.3, 1.0, 1.0, 2.5]))
    m = max(1, int(n * ratio))
    zf = float(rng.choice([0.0, 0.0, 0.2, 0.7, 0.97]))
    note(f"random seed={seed} n={n} m={m} zeros={zf}")
    w = random_weights(rng, n, zero_frac=zf, skew=bool(seed % 2))
    if seed % 5 == 4:
        w[-int(rng.integers(1, n + 1)):] = 0
        if w.sum() == 0:
            w[0] = 7
    build_and_compare(rtf, orc, w, m, S_extra=5000, seed=seed, baselines=seed % 3 == 0)


def test_single_tree_large(rtf, orc):
    """m = 1 and m = 2: one or two trees over 300k leaves, so most nodes'
    subtrees leave their tile and the fix-up kernel finishes them."""
    note("single tree n=300000")
    rng = np.random.default_rng(31)
    w = random_weights(rng, 300000, skew=True)
    build_and_compare(rtf, orc, w, 1, S_extra=50000, seed=1)
    build_and_compare(rtf, orc, w, 2, S_extra=50000, seed=2)
    # a few hundred trees: tiles with a handful of deferred nodes (fixed by
    # whole waves) beside tiles with dozens (fixed one thread per node)
    build_and_compare(rtf, orc, w, 64, S_extra=20000, seed=5)
    build_and_compare(rtf, orc, w, 600, S_extra=20000, seed=6)


def test_many_deferrals(rtf, orc):
    """Cells of several tiles each: every tile defers the nodes whose
    subtrees leave it, tens of thousands in all, more than the fix-up's
    waves take one at a time, so its one-thread-per-node path runs too."""
    note("many deferrals n=2^22")
    rng = np.random.default_rng(33)
    w = random_weights(rng, 1 << 22)
    build_and_compare(rtf, orc, w, 512, S_extra=20000, seed=7, baselines=False)
    build_and_compare(rtf, orc, w, 2048, S_extra=20000, seed=8, baselines=False)


def test_deferral_overflow(rtf, orc):
    """Long runs of equal keys (zero weights) inside one cell make every node
    of a tile defer, which overflows the per-tile list."""
    note("deferral overflow n=40000")
    rng = np.random.default_rng(32)
    w = random_weights(rng, 40000)
    for a in range(1000, 40000, 5000):
        w[a:a + 3000] = 0
    build_and_compare(rtf, orc, w, 4, S_extra=20000, seed=3)
    build_and_compare(rtf, orc, w, 40000, S_extra=20000, seed=4)


@pytest.mark.parametrize("family", ["pow20", "mod32_pow25", "mod64_pow35"])
def test_table1_densities(rtf, orc, family):
    """The high-dynamic-range densities of the paper's load-count table,
    quantised: bit-exact forest and samples at m = n and m = n/4."""
    from paper_1901_05423_amd import workloads as wl
    note(f"table-1 density {family} n=65536")
    n = 1 << 16
    q, _ = orc.quantize(wl.table1_weights(family, n))
    build_and_compare(rtf, orc, q, n, S_extra=40000, seed=11)
    build_and_compare(rtf, orc, q, n // 4, S_extra=40000, seed=12)


EXTREMES = np.array([0, 1, 2, 3, 1 << 31, (1 << 32) - 2, (1 << 32) - 1], np.uint64)


def adversarial(kind, n, rng):
    """Weight families that stress ties and degenerate trees: extreme values
    side by side, blocks of repeated values and zeros, one positive weight."""
    if kind == "extremes":
        w = EXTREMES[rng.integers(0, EXTREMES.size, n)]
    elif kind == "runs":
        parts, left = [], n
        while left > 0:
            ln = int(min(left, rng.integers(1, 3000)))
            parts.append(np.full(ln, [0, 0, 1, 7, (1 << 32) - 1][rng.integers(0, 5)], np.uint64))
            left -= ln
        w = np.concatenate(parts)
    else:  # one positive weight, at a tile edge or inside a tile
        w = np.zeros(n, np.uint64)
        w[int(rng.choice([0, 2047, 2048, n // 2, n - 1]) % n)] = int(rng.integers(1, 1 << 32))
    if w.sum() == 0:
        w[0] = 1
    return w.astype(np.uint32)


@pytest.mark.parametrize("kind", ["extremes", "runs", "single"])
@pytest.mark.parametrize("seed", range(4))
def test_adversarial_weights(rtf, orc, kind, seed):
    """Extreme values side by side, long blocks of equal weights and zeros,
    a single positive weight; sizes spanning several 2048-leaf tiles, guide
    tables from one cell to 3n."""
    rng = np.random.default_rng(7000 + 10 * seed + len(kind))
    n = int(rng.integers(1, 20000))
    m = max(1, int(n * float(rng.choice([0.001, 0.25, 1.0, 3.0]))))
    note(f"adversarial {kind} seed={seed} n={n} m={m}")
    w = adversarial(kind, n, rng)
    build_and_compare(rtf, orc, w, m, S_extra=5000, seed=seed, baselines=seed == 0)


@pytest.mark.parametrize("case", CASES[::2], ids=lambda c: "n%d_m%d" % (c[0], c[1]))
def test_tile_1024(rtf, orc, case):
    """The same forests built in 1024-element tiles of 256 threads (the
    other tile the tuner may pick): bit for bit the oracle's."""
    n, m, zf, skew, trail = case
    note(f"tile 1024 n={n} m={m} zeros={zf} skew={skew} trailing={trail}")
    rng = np.random.default_rng(n * 7919 + m)
    w = random_weights(rng, n, zero_frac=zf, skew=skew)
    if trail:
        w[-trail:] = 0
        if w.sum() == 0:
            w[0] = 5
    build_and_compare(rtf, orc, w, m, seed=n + m, baselines=False, tile=1024)


def test_tile_1024_deferrals(rtf, orc):
    """Tiles of 1024 with long zero runs and one heavy tree: deferred nodes
    near every tile edge and tiles that defer more than they can list."""
    note("tile 1024 zero runs and one tree")
    rng = np.random.default_rng(77)
    w = random_weights(rng, 50000)
    w[:3000] = 0
    w[10000:14000] = 0
    w[-5000:] = 0
    for m in (1, 2, 1000, 50000):
        build_and_compare(rtf, orc, w, m, seed=m, baselines=False, tile=1024)


def test_tile_rejected(rtf):
    import paper_1901_05423_amd as rtfm
    with pytest.raises(rtfm.RtfError):
        rtf.build(to_dev(np.ones(100, np.uint32)), 100, tile=512)
