"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and arranges them into the shapes of the
workloads; it performs none of the sampling method's arithmetic (no prefix sums,
no quantisation, no searching).  Both the CPU oracle and the GPU path consume
what it returns.

Every generator takes a ``config_id`` and seeds ``numpy.random.default_rng``
with ``190105423 + config_id`` (PCG64).  Uniform variates are full 64-bit raw
PCG64 outputs, standing for xi = u * 2^-64 in [0, 1).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 190105423

# workload ids
C1_UNIFORM_1K = 1
C2_ZIPF_1M = 2
C3_MAP_2D = 3
C4_BATCHED = 4
C5_DIFF = 5
H24_UNIFORM = 24
H24_ZIPF = 25
TABLE1 = 30  # uniforms for the load-count families
MAX_SIZE = 40  # the largest single distribution the library accepts


def rng(config_id: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + int(config_id))


def uniforms(r: np.random.Generator, count: int) -> np.ndarray:
    """``count`` raw 64-bit uniforms."""
    return r.bit_generator.random_raw(int(count)).astype(np.uint64)


def weights_uniform(r: np.random.Generator, n: int) -> np.ndarray:
    """i.i.d. uniform(0, 1] weights as float32."""
    return (1.0 - r.random(int(n))).astype(np.float32)


def weights_zipf(r: np.random.Generator, n: int, a: float = 1.1) -> np.ndarray:
    """p_i proportional to (i+1)^-a, randomly permuted, as float32."""
    base = np.power(np.arange(1, n + 1, dtype=np.float64), -a)
    return base[r.permutation(int(n))].astype(np.float32)


def map_2d(r: np.random.Generator, rows: int = 4096, cols: int = 4096,
           spots: int = 8, amp: float = 1e4, sigma: float = 3.0):
    """Log-normal(0, 1.5) map plus Gaussian hot spots at pixel centres.

    Returns (image float32[rows, cols], marginal float32[rows]) where the
    marginal is the FP64 row sum of the float32 image, cast to float32.
    """
    img = r.lognormal(0.0, 1.5, size=(rows, cols))
    centres = r.uniform(0.0, float(max(rows, cols)), size=(spots, 2))
    yy = np.arange(rows, dtype=np.float64)[:, None] + 0.5
    xx = np.arange(cols, dtype=np.float64)[None, :] + 0.5
    for cy, cx in centres:
        img += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * sigma * sigma))
    img32 = img.astype(np.float32)
    marginal = img32.astype(np.float64).sum(axis=1).astype(np.float32)
    return img32, marginal


def batched_uneven(r: np.random.Generator, D: int = 10000, lo: int = 16,
                   hi: int = 65536, per_1k: int = 64):
    """Uneven batch: sizes log-uniform in [lo, hi]; per distribution a fair coin
    picks uniform(0,1] or Pareto(alpha=1.2) weights; ceil(per_1k*n_d/1000)
    samples per distribution.

    Returns (weights float32[sum n_d], elem_off int64[D+1], sample_off int64[D+1]).
    """
    sizes = np.floor(np.exp(r.uniform(np.log(lo), np.log(hi), size=D))).astype(np.int64)
    sizes = np.clip(sizes, lo, hi)
    coins = r.random(D) < 0.5
    parts = []
    for d in range(D):
        v = 1.0 - r.random(int(sizes[d]))
        if coins[d]:
            v = np.power(v, -1.0 / 1.2)
        parts.append(v.astype(np.float32))
    w = np.concatenate(parts)
    elem_off = np.zeros(D + 1, np.int64)
    elem_off[1:] = np.cumsum(sizes)
    counts = (per_1k * sizes + 999) // 1000
    sample_off = np.zeros(D + 1, np.int64)
    sample_off[1:] = np.cumsum(counts)
    return w, elem_off, sample_off


def logits(r: np.random.Generator, D: int = 256, n: int = 4096) -> np.ndarray:
    """N(0, 1) float32 logits, shape [D, n]."""
    return r.standard_normal((D, n)).astype(np.float32)


# The three densities of the paper's load-count table (Table 1, Sec. 4), with index
# i = 0 .. n-1; each is normalised to a maximum of 1 in FP64 before the cast
# to float32, so values below float32's range become zero weights.
TABLE1_FAMILIES = ("pow20", "mod32_pow25", "mod64_pow35")


def table1_weights(family: str, n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    if family == "pow20":  # p_i ~ i^20
        w = (i / max(n - 1, 1)) ** 20
    elif family == "mod32_pow25":  # p_i ~ (i mod 32 + 1)^25
        w = ((np.mod(i, 32) + 1) / 32.0) ** 25
    elif family == "mod64_pow35":  # p_i ~ (i mod 64 + 1)^35
        w = ((np.mod(i, 64) + 1) / 64.0) ** 35
    else:
        raise ValueError(family)
    return w.astype(np.float32)


def hammersley_u64(N: int) -> np.ndarray:
    """The two-dimensional Hammersley point set of N = 2^k points (k >= 1) as
    0.64 fixed-point pairs, shape [N, 2]: (i / N, the base-2 radical inverse
    of i), i = 0 .. N-1 -- the low-discrepancy input of the paper's quality
    study (Figs. 2d_zoom, convergence).  Both components are exact: i / N is
    i << (64 - k), and the radical inverse mirrors the k bits of i about the
    binary point."""
    N = int(N)
    k = N.bit_length() - 1
    if N < 2 or N != 1 << k or k > 32:
        raise ValueError("N must be a power of two in [2, 2^32]")
    i = np.arange(N, dtype=np.uint64)
    r = i.astype(np.uint32)
    # reverse the 32 bits of i (swap halves, bytes, nibbles, pairs, bits)
    r = (r >> np.uint32(16)) | (r << np.uint32(16))
    r = ((r >> np.uint32(8)) & np.uint32(0x00FF00FF)) | ((r & np.uint32(0x00FF00FF)) << np.uint32(8))
    r = ((r >> np.uint32(4)) & np.uint32(0x0F0F0F0F)) | ((r & np.uint32(0x0F0F0F0F)) << np.uint32(4))
    r = ((r >> np.uint32(2)) & np.uint32(0x33333333)) | ((r & np.uint32(0x33333333)) << np.uint32(2))
    r = ((r >> np.uint32(1)) & np.uint32(0x55555555)) | ((r & np.uint32(0x55555555)) << np.uint32(1))
    out = np.empty((N, 2), np.uint64)
    out[:, 0] = i << np.uint64(64 - k)
    out[:, 1] = r.astype(np.uint64) << np.uint64(32)
    return out
