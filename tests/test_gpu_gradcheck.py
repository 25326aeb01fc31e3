"""The adjoint of x (Sec. 5, the sub-pixel position as a function of the
weights) checked by differencing the GPU forward path itself:

* torch.autograd.gradcheck in float64 on tiny batches, with every uniform in
  the middle of its interval so that no perturbation moves a sample across
  a kink of x (the index is held fixed, as the adjoint assumes);
* central differences with the indices recomputed at every evaluation (the
  full quantise-free build + sample path on integer weights, each perturbed
  by an exact integer step), on random uniforms: a sanity bar of 1e-3, since
  a few samples cross an interval boundary (where x has a kink) per
  coordinate.
"""
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


def mid_interval_uniforms(orc, q, per):
    """`per` uniforms inside each positive-weight interval of q, at fractions
    (k + 1) / (per + 1) of it (exact integers: u = U_i + (U_{i+1} - U_i) f)."""
    C = [int(c) for c in orc.prefix(q)]
    W = C[-1]
    out = []
    for i in range(q.size):
        if q[i] == 0:
            continue
        lo = -((-C[i] << 64) // W)
        hi = -((-C[i + 1] << 64) // W) if C[i + 1] < W else 1 << 64
        for k in range(per):
            out.append(lo + (hi - lo) * (k + 1) // (per + 1))
    return np.array(out, dtype=np.uint64)


def test_gradcheck_float64_tiny(rtf, orc):
    import torch
    note("gradcheck D=2 n=7,5")
    rng = np.random.default_rng(61)
    sizes = [7, 5]
    v_h = [(0.2 + rng.random(s)) for s in sizes]
    eo = np.array([0, 7, 12], np.int64)
    us = []
    for d in range(2):
        q, _ = orc.quantize(v_h[d].astype(np.float32))
        us.append(mid_interval_uniforms(orc, q, 3))
    so = np.array([0, us[0].size, us[0].size + us[1].size], np.int64)
    u = to_dev(np.concatenate(us))
    eod, sod = to_dev(eo), to_dev(so)
    v64 = torch.from_numpy(np.concatenate(v_h)).to("cuda:0").requires_grad_(True)

    def fn(v):
        return rtf.RTFSample.apply(v.float(), u, eod, sod, 1.0)

    # the forward rounds v to float32 (about 6e-8 relative): with eps = 1e-4
    # the numerical Jacobian carries about 6e-4 relative error; FP64 atomics
    # in the adjoint make repeated backward passes differ by rounding only
    assert torch.autograd.gradcheck(fn, (v64,), eps=1e-4, atol=2e-5, rtol=2e-3,
                                    nondet_tol=1e-9, fast_mode=False)


def test_fd_recomputed_indices(rtf, orc):
    """dL/dv of L = sum sin(7 x) for one distribution of 64 weights and 4096
    random uniforms, against central differences of L through rtf.build +
    rtf.sample with the weights moved by integer steps (h = 1e-6 relative)."""
    import torch
    note("FD with recomputed indices n=64 S=4096")
    rng = np.random.default_rng(62)
    n, S = 64, 4096
    # integer weights below 2^31, so that every step up stays a uint32; the
    # real weights are v = q / scale, in (0, 1]
    q = ((rng.integers(1, 2 ** 32, n, dtype=np.uint64) >> 1) + 1).astype(np.int64)
    scale = 2.0 ** 31
    s_d = torch.tensor([scale], dtype=torch.float64, device="cuda:0")
    u = to_dev(rng.integers(0, 2 ** 64, S, dtype=np.uint64))

    def loss(qq):
        f = rtf.build(to_dev(qq.astype(np.uint32)), n)
        idx, x = rtf.sample(f, u)
        return torch.sin(7.0 * x).sum().item(), idx, x

    L0, idx, x = loss(q)
    f0 = rtf.build(to_dev(q.astype(np.uint32)), n)
    g = rtf.backward(f0, u, idx, 7.0 * torch.cos(7.0 * x), s_d).cpu().numpy()
    fd = np.zeros(n)
    for k in range(n):
        step = max(1, int(round(q[k] * 1e-6)))
        qp, qm = q.copy(), q.copy()
        qp[k] += step
        qm[k] -= step
        assert qp[k] < 2 ** 32 and qm[k] >= 1
        # v = q / scale: a step of `step` in q is step / scale in v
        fd[k] = (loss(qp)[0] - loss(qm)[0]) / (2.0 * step / scale)
    torch.cuda.synchronize()
    err = np.abs(fd - g)
    assert err.max() <= 1e-3 * np.abs(g).max(), (err.max(), np.abs(g).max())
    assert np.linalg.norm(fd - g) <= 1e-3 * np.linalg.norm(g)


def test_rtfsample_rejects_bad_weights(rtf):
    """The differentiable forward raises on a NaN or negative weight and on a
    distribution whose weights are all zero, instead of sampling them."""
    import torch
    note("RTFSample data errors")
    dev = torch.device("cuda:0")
    eo = torch.tensor([0, 5, 10], dtype=torch.int64, device=dev)
    so = torch.tensor([0, 4, 8], dtype=torch.int64, device=dev)
    u = torch.arange(8, dtype=torch.int64, device=dev) * (1 << 60)
    good = torch.rand(10, device=dev) + 0.1
    x = rtf.RTFSample.apply(good, u, eo, so, 1.0)
    assert x.shape == (8,) and bool(torch.isfinite(x).all())
    for bad_value, code in ((float("nan"), rtf.RTF_ERR_VALUE), (-1.0, rtf.RTF_ERR_VALUE)):
        v = good.clone()
        v[3] = bad_value
        with pytest.raises(rtf.RtfError) as e:
            rtf.RTFSample.apply(v, u, eo, so, 1.0)
        assert e.value.code == code
    v = good.clone()
    v[5:] = 0.0
    with pytest.raises(rtf.RtfError) as e:
        rtf.RTFSample.apply(v, u, eo, so, 1.0)
    assert e.value.code == rtf.RTF_ERR_ZERO_TOTAL
