"""The quantise -> build -> sample chain of a batch captured as a HIP graph:
every replay must equal the eager run and the oracle (Sec. 5, many
distributions at once)."""
import numpy as np
import pytest

from gpu_util import assert_samples, note, to_dev

pytestmark = pytest.mark.gpu


def offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def oracle_batch(orc, v, eo, so, u):
    q, _ = orc.quantize(v, eo)
    idx = np.empty(u.size, np.int32)
    x = np.empty(u.size)
    for d in range(eo.size - 1):
        a, b = so[d], so[d + 1]
        if a < b:
            idx[a:b], x[a:b] = orc.search(q[eo[d]:eo[d + 1]], u[a:b])
    return idx, x


def test_graph_replays_match_eager_and_oracle(orc):
    import torch
    from paper_1901_05423_amd.plan import BatchedPlan
    note("graph replay D=80")
    rng = np.random.default_rng(77)
    D = 80
    sizes = rng.integers(1, 5000, D)
    counts = rng.integers(0, 4000, D)
    eo, so = offsets(sizes), offsets(counts)
    co = eo.copy()  # m_d = n_d
    v1 = (1e-3 + rng.random(int(eo[-1]))).astype(np.float32)
    v1[rng.random(v1.size) < 0.05] = 0
    u1 = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    v = to_dev(v1)
    u = to_dev(u1)
    plan = BatchedPlan(to_dev(eo), to_dev(co), to_dev(so), eo[-1], co[-1], so[-1])
    idx, x = plan.run(v, u)
    plan.check()
    e_idx, e_x = idx.cpu().numpy().copy(), x.cpu().numpy().copy()
    r_idx, r_x = oracle_batch(orc, v1, eo, so, u1)
    assert_samples(e_idx, e_x, r_idx, r_x)

    g = plan.capture(v, u)
    for rep in range(4):
        plan.idx.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(plan.idx.cpu().numpy(), e_idx), rep
        assert np.array_equal(plan.x.cpu().numpy(), e_x), rep
        _ = (v * 2).sum().item()  # eager work between replays

    # new data in the same buffers, same graph
    v2 = (1e-3 + rng.random(v1.size)).astype(np.float32) ** 3
    u2 = rng.integers(0, 2 ** 64, u1.size, dtype=np.uint64)
    v.copy_(to_dev(v2))
    u.copy_(to_dev(u2))
    g.replay()
    torch.cuda.synchronize()
    r_idx, r_x = oracle_batch(orc, v2, eo, so, u2)
    assert_samples(plan.idx.cpu().numpy(), plan.x.cpu().numpy(), r_idx, r_x)


def test_tuned_cell_ratio_keeps_indices(orc, tmp_path, monkeypatch):
    """Whatever guide size the tuner picks, the indices are the oracle's."""
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd import tune
    note("tuner")
    monkeypatch.setenv("RTF_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.delenv("RTF_CELL_RATIO", raising=False)
    rng = np.random.default_rng(8)
    w = rng.integers(1, 2 ** 32, 50000, dtype=np.uint64).astype(np.uint32)
    u = rng.integers(0, 2 ** 64, 200000, dtype=np.uint64)
    wd, ud = to_dev(w), to_dev(u)
    r = tune.best_cell_ratio(wd, ud)
    assert r in tune.CANDIDATES
    assert tune.best_cell_ratio(wd, ud) == r  # from the cache
    f = rtf.build(wd, max(1, int(round(r * w.size))))
    idx, x = rtf.sample(f, ud)
    i_ref, x_ref = orc.search(w, u)
    assert_samples(idx.cpu().numpy(), x.cpu().numpy(), i_ref, x_ref)
