"""rtf_backward_static (the backward pass over the library's fixed device
scratch, for callers that cannot allocate) against rtf_backward and the FP64
oracle gradient: two calls in a row on one GPU, the second on a smaller
input, so that the second runs over what the first left in the array."""
import ctypes

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


def case(rtf, sizes, counts, seed):
    """Quantise, build and sample a batch; returns what both backward entry
    points take, plus the host copies the oracle needs."""
    rng = np.random.default_rng(seed)
    vs = [(0.01 + rng.random(s)).astype(np.float32) for s in sizes]
    vs[0][: min(5, sizes[0] - 1)] = 0  # a zero run at the start
    v = np.concatenate(vs)
    eo, so = offsets(sizes), offsets(counts)
    u = rng.integers(0, 2 ** 64, int(so[-1]), dtype=np.uint64)
    g = rng.standard_normal(int(so[-1]))
    eod, sod, ud = to_dev(eo), to_dev(so), to_dev(u)
    q, s = rtf.quantize(to_dev(v), eod)
    f = rtf.build_batched(q, eod, eod)
    idx, _ = rtf.sample_batched(f, sod, ud)
    return dict(f=f, sod=sod, ud=ud, idx=idx, gd=to_dev(g), s=s, q=q, eo=eo, so=so, u=u, g=g)


def static_call(rtf, c, out):
    """rtf_backward_static through the C ABI (ctypes), into a preallocated output."""
    import torch
    L = rtf.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    rc = L.rtf_backward_static(ctypes.byref(c["f"].desc), p(c["sod"]), p(c["ud"]), p(c["idx"]),
                               p(c["gd"]), c["ud"].numel(), p(c["s"]), p(out), st)
    assert rc == rtf.RTF_OK, L.rtf_status_string(rc).decode()
    return out


def check(rtf, orc, c, got):
    import torch
    ws_grad = rtf.backward(c["f"], c["ud"], c["idx"], c["gd"], c["s"], sample_off=c["sod"])
    torch.cuda.synchronize()
    got, ref_ws = got.cpu().numpy(), ws_grad.cpu().numpy()
    # both sum with FP64 atomics in whatever order the hardware takes them
    tol = 1e-9 * max(np.abs(ref_ws).max(), 1.0)
    assert np.abs(got - ref_ws).max() <= tol
    q_h, s_h = c["q"].cpu().numpy(), c["s"].cpu().numpy()
    eo, so = c["eo"], c["so"]
    for d in range(eo.size - 1):
        a, b = eo[d], eo[d + 1]
        ref = orc.grad(q_h[a:b], s_h[d], c["u"][so[d]:so[d + 1]], c["g"][so[d]:so[d + 1]])
        scale = max(np.abs(ref).max(), 1.0)
        assert np.abs(got[a:b] - ref).max() <= 1e-4 * scale, d


def test_static_backward_two_calls(rtf, orc):
    import torch
    note("backward_static: D=5 n=24597 then D=3 n=4401")
    big = case(rtf, [4096, 17, 12000, 8190, 294], [200000, 50, 70000, 131072, 900], 71)
    small = case(rtf, [4096, 300, 5], [30000, 2000, 7], 72)
    out_big = torch.empty(big["f"].n_total, dtype=torch.float64, device="cuda:0")
    out_small = torch.empty(small["f"].n_total, dtype=torch.float64, device="cuda:0")
    static_call(rtf, big, out_big)
    static_call(rtf, small, out_small)  # reuses the array the first call filled
    torch.cuda.synchronize()
    check(rtf, orc, big, out_big)
    check(rtf, orc, small, out_small)


def test_static_backward_limits(rtf):
    """Sizes past the array's limits are rejected before anything runs."""
    import torch
    note("backward_static: size limits")
    L = rtf.lib()
    n = (1 << 20) + 1
    q = torch.ones(n, dtype=torch.uint32, device="cuda:0")
    f = rtf.build(q, n // 4)
    s = torch.ones(1, dtype=torch.float64, device="cuda:0")
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.rtf_backward_static(ctypes.byref(f.desc), None, None, None, None, 0,
                               ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(out.data_ptr()), st)
    assert rc == rtf.RTF_ERR_SIZE
    torch.cuda.synchronize()
