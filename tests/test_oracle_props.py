"""Property tests of the oracle on adversarial weight vectors drawn by
hypothesis: extreme weights (1 and 2^32 - 1 side by side), long zero runs, a
single positive weight, n = 1, and guide tables from m = 1 to m = 3n.  The
properties hold by the mathematics of the method, whatever the input:

* Alg. 2 on the oracle's forest returns the binary search's index at every
  critical uniform (each lower bound, one below and one above it, each cell
  edge, 0 and 2^64 - 1), before and after the depth fallback (Sec. 3);
* binary search equals linear search, and never returns a zero-weight
  interval;
* the mapping is monotone (Sec. 1): sorted uniforms give non-decreasing
  indices and positions, and every x lies in [0, 1].
"""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

TWO64 = 1 << 64
EXTREMES = [0, 1, 2, 3, (1 << 31), (1 << 32) - 2, (1 << 32) - 1]


@st.composite
def weight_vectors(draw):
    n = draw(st.integers(1, 200))
    kind = draw(st.sampled_from(["extremes", "runs", "single", "random"]))
    if kind == "extremes":
        w = draw(st.lists(st.sampled_from(EXTREMES), min_size=n, max_size=n))
    elif kind == "runs":
        # blocks of zeros and of one repeated positive value
        w = []
        while len(w) < n:
            ln = draw(st.integers(1, 40))
            val = draw(st.sampled_from([0, 0, 1, 7, (1 << 32) - 1]))
            w += [val] * ln
        w = w[:n]
    elif kind == "single":
        w = [0] * n
        w[draw(st.integers(0, n - 1))] = draw(st.integers(1, (1 << 32) - 1))
    else:
        w = draw(st.lists(st.integers(0, (1 << 32) - 1), min_size=n, max_size=n))
    if not any(w):
        w[draw(st.integers(0, n - 1))] = 1
    ratio = draw(st.sampled_from([None, 0.1, 0.25, 1.0, 3.0]))
    m = 1 if ratio is None else max(1, int(round(ratio * n)))
    return np.array(w, np.uint64).astype(np.uint32), m


def critical(w, m):
    C = np.concatenate([[0], np.cumsum(w.astype(object))])
    W = int(C[-1])
    u = {0, TWO64 - 1}
    for c in C[:-1]:
        c = int(c)
        if c < W:
            k = -((-(c << 64)) // W)
            u.update([k, max(k - 1, 0), min(k + 1, TWO64 - 1)])
    for g in range(1, m):
        e = -((-(g << 64)) // m)
        u.update([e, e - 1])
    return np.array(sorted(u), np.uint64)


SETTINGS = settings(max_examples=300, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(weight_vectors())
def test_forest_descent_is_the_inverse_cdf(orc, case):
    w, m = case
    u = critical(w, m)
    i_ref, x_ref = orc.search(w, u)
    assert np.array_equal(orc.linear_search(w, u), i_ref)
    assert np.all(w[i_ref] > 0)  # a zero-weight interval is never sampled
    f = orc.forest(w, m=m)
    assert np.array_equal(orc.descend(f, u), i_ref)
    g, _ = orc.balance(f)
    assert np.array_equal(orc.descend(g, u), i_ref)
    # monotone: sorted uniforms give non-decreasing indices and positions
    assert np.all(np.diff(i_ref) >= 0)
    assert np.all(np.diff(x_ref) >= 0)
    assert np.all((x_ref >= 0.0) & (x_ref <= 1.0))

