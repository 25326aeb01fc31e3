"""The Hammersley point set generator against its definition, written out
digit by digit on small sizes."""
import numpy as np
import pytest


def radical_inverse_bits(i, k):
    """Base-2 radical inverse of i as a k-bit integer: digit b of i becomes
    digit k-1-b."""
    r = 0
    for b in range(k):
        if (i >> b) & 1:
            r |= 1 << (k - 1 - b)
    return r


@pytest.mark.parametrize("k", [1, 2, 5, 10, 13])
def test_hammersley_definition(k):
    from paper_1901_05423_amd import workloads as wl
    N = 1 << k
    h = wl.hammersley_u64(N)
    for i in range(N):
        assert int(h[i, 0]) == i << (64 - k)
        assert int(h[i, 1]) == radical_inverse_bits(i, k) << (64 - k)
    # a (0, m, 2)-net in base 2: every dyadic box of volume 1/N holds one point
    for a in range(k + 1):
        cols = (h[:, 0] >> np.uint64(64 - a)) if a else np.zeros(N, np.uint64)
        rows = (h[:, 1] >> np.uint64(64 - (k - a))) if k - a else np.zeros(N, np.uint64)
        boxes = cols.astype(np.int64) * (1 << (k - a)) + rows.astype(np.int64)
        assert np.array_equal(np.sort(boxes), np.arange(N))


def test_hammersley_rejects_other_sizes():
    from paper_1901_05423_amd import workloads as wl
    for N in (0, 1, 3, 1000):
        with pytest.raises(ValueError):
            wl.hammersley_u64(N)
