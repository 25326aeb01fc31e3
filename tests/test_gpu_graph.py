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


def test_graph_captured_autograd_forward_backward(orc):
    """RTFSample through a DiffPlan: the differentiable step (softplus, quantise,
    build, sample, the adjoint of L = sum sin(7x)) captured as one graph; every
    replay's dL/dz against the oracle's FP64 gradient (1e-4 of its norms)."""
    import torch
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd.plan import DiffPlan
    note("graph autograd D=8 n=4096")
    rng = np.random.default_rng(91)
    D, n, per = 8, 4096, 1 << 15
    z_h = rng.standard_normal((D, n)).astype(np.float32)
    u_h = rng.integers(0, 2 ** 64, D * per, dtype=np.uint64)
    eo = to_dev(np.arange(D + 1, dtype=np.int64) * n)
    so = to_dev(np.arange(D + 1, dtype=np.int64) * per)
    co = to_dev(np.arange(D + 1, dtype=np.int64) * (n // 4))
    plan = DiffPlan(eo, co, so, D * n, D * (n // 4), D * per)
    z = to_dev(z_h).requires_grad_(True)
    u = to_dev(u_h)

    def step():
        v = torch.nn.functional.softplus(z).reshape(-1)
        x = rtf.RTFSample.apply(v, u, plan)
        # dL/dx of L = sum sin(7x), passed directly: no reduction kernel in
        # the captured graph
        x.backward(7.0 * torch.cos(7.0 * x.detach()))
        return x

    # eager warm-up on a side stream, then the capture
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            z.grad = None
            step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    z.grad = None
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        x_c = step()
    sig = 1.0 / (1.0 + np.exp(-z_h.astype(np.float64)))
    for rep in range(3):
        z.grad.fill_(np.nan)
        g.replay()
        torch.cuda.synchronize()
        gz = z.grad.detach().double().cpu().numpy()
        x_h = x_c.detach().cpu().numpy()
        v32 = torch.nn.functional.softplus(z.detach()).reshape(-1).cpu().numpy()
        for d in (0, 3, 7):
            q, sc = orc.quantize(v32[d * n:(d + 1) * n])
            uu = u_h[d * per:(d + 1) * per]
            i_ref, x_ref = orc.search(q, uu)
            assert np.abs(x_h[d * per:(d + 1) * per] - x_ref).max() <= 1e-12, (rep, d)
            ref = orc.grad(q, sc[0], uu, 7.0 * np.cos(7.0 * x_ref)) * sig[d]
            err = gz[d] - ref
            assert np.abs(err).max() <= 1e-4 * np.abs(ref).max(), (rep, d)
            assert np.linalg.norm(err) <= 1e-4 * np.linalg.norm(ref), (rep, d)
        _ = (z * 2).sum().item()  # eager work between replays
