"""rtf_forest_import: sampling on a forest the GPU did not build.

The oracle's forest (the recursive definition) is turned into the library's
records on the host -- node records from its keys and children, guide cell
records from its keys, guide entries and trees as the record layout defines
them -- imported, and sampled; the indices and positions must equal the
oracle's binary search at every critical u.  This checks the sampling
kernels independently of the GPU build.  A GPU-built forest exported and
imported again samples as the original does."""
import numpy as np
import pytest

from gpu_util import TWO64, assert_samples, critical_u, expected_cells, note, random_weights, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1901_05423_amd as rtf
    rtf.lib()
    return rtf


def oracle_records(ref):
    """The library's raw node and cell records for an oracle forest."""
    n, m = ref.key.size, ref.table.size
    nodes = np.zeros((n, 2), np.uint64)
    nodes[:, 0] = ref.key
    nodes[:, 1] = np.ascontiguousarray(ref.child.astype(np.int32)).view(np.uint64).reshape(n)
    K, aux = expected_cells(ref)
    cells = np.zeros((m, 8), np.uint64)
    cells[:, :7] = K
    pair = np.zeros((m, 2), np.int32)
    pair[:, 0] = ref.table
    pair[:, 1] = aux
    cells[:, 7] = pair.view(np.uint64).reshape(m)
    return nodes, cells


def offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


@pytest.mark.parametrize("ratio", [1.0, 0.25])
def test_import_oracle_forest_single(rtf, orc, ratio):
    note(f"import: oracle forest, one distribution, m = {ratio} n")
    rng = np.random.default_rng(101)
    n = 50000
    w = random_weights(rng, n, zero_frac=0.1)
    w[-7:] = 0  # trailing zeros
    m = max(1, int(round(ratio * n)))
    ref = orc.forest(w, m=m)
    nodes, cells = oracle_records(ref)
    f = rtf.forest_import(nodes, cells, ref.W)
    u = critical_u(ref.key, int(ref.W[0]), m, extra=100000, rng=rng)
    idx, x = rtf.sample(f, to_dev(u))
    i_ref, x_ref = orc.search(w, u)
    assert_samples(idx.cpu().numpy(), x.cpu().numpy(), i_ref, x_ref)


def test_import_oracle_forest_batched(rtf, orc):
    note("import: oracle forest, batched")
    rng = np.random.default_rng(102)
    ws = [random_weights(rng, s, zero_frac=z) for s, z in
          [(1, 0.0), (700, 0.2), (4096, 0.0), (3000, 0.5), (17, 0.0)]]
    w = np.concatenate(ws)
    eo = offsets([a.size for a in ws])
    co = offsets([max(1, a.size // 4) for a in ws])
    ref = orc.forest(w, elem_off=eo, cell_off=co)
    nodes, cells = oracle_records(ref)
    f = rtf.forest_import(nodes, cells, ref.W, eo, co)
    counts = [500, 20000, 30000, 20000, 100]
    so = offsets(counts)
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
    idx, x = idx.cpu().numpy(), x.cpu().numpy()
    for d, wd in enumerate(ws):
        a, b = so[d], so[d + 1]
        i_ref, x_ref = orc.search(wd, u[a:b])
        assert_samples(idx[a:b], x[a:b], i_ref, x_ref)


def test_export_import_round_trip(rtf, orc):
    note("import: GPU forest exported and imported")
    import torch
    rng = np.random.default_rng(103)
    w = random_weights(rng, 1 << 18, zero_frac=0.05)
    f = rtf.build(to_dev(w), 1 << 16)
    nodes, cells, W = f.export_raw()
    g = rtf.forest_import(nodes, cells, W)
    u = to_dev(rng.integers(0, 2 ** 64, 1 << 20, dtype=np.uint64))
    i1, x1 = rtf.sample(f, u)
    i2, x2 = rtf.sample(g, u)
    torch.cuda.synchronize()
    assert torch.equal(i1, i2) and torch.equal(x1, x2)
    n2, c2, W2 = g.export_raw()
    assert np.array_equal(n2, nodes) and np.array_equal(c2, cells) and np.array_equal(W2, W)
