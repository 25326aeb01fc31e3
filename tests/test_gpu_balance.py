"""GPU parity of the depth fallback (Sec. 3): rtf_forest_balance against the
oracle's balanced forest, bit for bit (keys, children, guide entries, cell
records, collapsed records), with the sampled indices unchanged."""
import numpy as np
import pytest

from gpu_util import (assert_forest, assert_samples, assert_wide, critical_u, forest_depth, note,
                      to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1901_05423_amd as rtf
    rtf.lib()
    return rtf


def comb(c):
    return np.array([1 << (c - 1 - k) for k in range(c)], np.uint32)


def offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def check_balance(rtf, orc, ws, cells, seed, what):
    rng = np.random.default_rng(seed)
    w = np.concatenate(ws)
    eo, co = offsets([x.size for x in ws]), offsets(cells)
    if len(ws) == 1:
        f = rtf.build(to_dev(w), int(cells[0]))
    else:
        f = rtf.build_batched(to_dev(w), to_dev(eo), to_dev(co))
    ref0 = orc.forest(w, elem_off=eo, cell_off=co)
    depth0 = f.depth()
    assert depth0 == forest_depth(ref0), what
    ref, want = orc.balance(ref0)
    got = f.balance()
    f.check()
    assert got == want, (what, got, want)
    assert_forest(f, ref, what)
    assert f.depth() == forest_depth(ref), what
    f.widen()
    assert_wide(f, ref, what)
    for d, wd in enumerate(ws):
        u = critical_u(ref.key[eo[d]:eo[d + 1]], int(ref.W[d]), int(cells[d]), extra=20000, rng=rng)
        i_ref, x_ref = orc.search(wd, u)
        if len(ws) == 1:
            idx, x = rtf.sample(f, to_dev(u))
        else:
            so = np.zeros(len(ws) + 1, np.int64)
            so[d + 1:] = u.size
            idx, x = rtf.sample_batched(f, to_dev(so), to_dev(u))
        assert_samples(idx.cpu().numpy(), x.cpu().numpy(), i_ref, x_ref)
    return got


def test_balance_combs_batched(rtf, orc):
    """Combs of 24 and 31 leaves (24-leaf combs three to a distribution), a
    comb with zero weights inside, and random weights, batched."""
    note("balance: comb batch")
    rng = np.random.default_rng(81)
    z = comb(16).astype(np.uint64)
    z[3:6] = 0
    ws = [np.tile(comb(24), 3), comb(31), z.astype(np.uint32),
          rng.integers(1, 2 ** 32, 500, dtype=np.uint64).astype(np.uint32)]
    assert check_balance(rtf, orc, ws, [2, 1, 1, 125], 1, "combs") >= 4


def test_balance_edge_of_criterion(rtf, orc):
    """Combs of 7 to 10 leaves, one per distribution: only 8 and 10 rebuild."""
    note("balance: criterion edge")
    assert check_balance(rtf, orc, [comb(c) for c in (7, 8, 9, 10)], [1, 1, 1, 1], 2,
                         "edge") == 2


def test_balance_single_distribution_many_combs(rtf, orc):
    """One distribution of 2^16 weights made of 24-leaf combs with a guide
    table of one cell per 32 weights: tiles, halos and the fix-up of the
    build meet many degenerate cells."""
    note("balance: n=2^16 combs")
    w = np.tile(comb(24), (1 << 16) // 24 + 1)[: 1 << 16]
    assert check_balance(rtf, orc, [w], [(1 << 16) // 32], 3, "many combs") > 0


@pytest.mark.parametrize("family", ["pow20", "mod32_pow25", "mod64_pow35"])
def test_balance_table1(rtf, orc, family):
    """The paper's high-dynamic-range densities at n = m = 2^16: the
    fallback acts exactly as the oracle's does."""
    from paper_1901_05423_amd import workloads as wl
    note(f"balance: table-1 {family}")
    n = 1 << 16
    q, _ = orc.quantize(wl.table1_weights(family, n))
    check_balance(rtf, orc, [q], [n], 4, family)


def test_balance_leaves_ordinary_forests(rtf, orc):
    """Random weights at n = 2^20, m = n/4: nothing is degenerate."""
    note("balance: n=2^20 uniform")
    rng = np.random.default_rng(85)
    w = rng.integers(1, 2 ** 32, 1 << 20, dtype=np.uint64).astype(np.uint32)
    assert check_balance(rtf, orc, [w], [1 << 18], 5, "uniform") == 0
