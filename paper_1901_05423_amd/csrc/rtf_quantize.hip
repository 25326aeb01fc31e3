// rtf_quantize.hip -- real weights to uint32, per distribution.
//
// The method needs exact partial sums; weights are therefore quantised before
// the build: s_d = (2^32 - 1) / max_d v in FP64, q = rint(v * s_d) clamped to
// [1, 2^32 - 1] for v > 0 and q = 0 for v == 0.  One FP64 multiply and a
// round-half-even, so the result is the same on every IEEE machine.
//
// Kernels: k_qinit clears the per-distribution maxima (kept in the low word of
// scale[d] while the call runs), k_qmax takes the maxima with integer atomics
// on the float bits (order-preserving for non-negative floats), k_qapply
// writes q, k_qfinal writes the scales (for one distribution k_qapply does).
#include "rtf_internal.h"

namespace rtf {

namespace {

constexpr int QT = 256;
constexpr int QI = 16;
constexpr int QMAX_LDS_DISTS = 64;  // distributions a k_qmax block sums in LDS

// Index d with off[d] <= i < off[d+1] over off[0..D], found by the whole
// block (uniform i): each round probes QT evenly spaced offsets at once, so
// 10^4 distributions take two dependent loads instead of a binary search's
// fourteen.  Every thread of the block must call it.
__device__ inline int32_t block_find_segment(const int64_t *off, int32_t D, int64_t i) {
    int32_t lo = 0, hi = D;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int32_t step = (hi - lo + QT - 1) / QT;
        const int32_t p = lo + ((int32_t)threadIdx.x + 1) * step;
        const int below = (p < hi && off[p] <= i) ? 1 : 0;
        const int32_t nlo = lo + __syncthreads_count(below) * step;
        hi = nlo + step < hi ? nlo + step : hi;
        lo = nlo;
    }
    return lo;
}

// Both d0 with off[d0] <= i0 < off[d0+1] and d1 with off[d1] <= i1 <
// off[d1+1] (uniform i0 <= i1), found at once: waves 0-1 search for i0 and
// waves 2-3 for i1, 128 probes per round each, so 10^4 distributions take two
// rounds for both.  Every thread must call it; s_cnt holds 2 x 4 counts.
__device__ inline void block_find_two(const int64_t *off, int32_t D, int64_t i0, int64_t i1,
                                      int32_t *s_cnt, int32_t &d0, int32_t &d1) {
    static_assert(QT == 256, "four waves, two per search");
    const int w = threadIdx.x >> 6, t = threadIdx.x & 127;
    const bool second = w >= 2;
    const int64_t i = second ? i1 : i0;
    int32_t lo0 = 0, hi0 = D, lo1 = 0, hi1 = D;  // off[lo] <= i < off[hi]
    for (int round = 0; hi0 - lo0 > 1 || hi1 - lo1 > 1; ++round) {
        const int32_t lo = second ? lo1 : lo0, hi = second ? hi1 : hi0;
        const int32_t step = (hi - lo + 127) / 128;
        const int32_t p = lo + (t + 1) * step;
        const bool below = hi - lo > 1 && p < hi && off[p] <= i;
        const int32_t c = __popcll(__ballot(below));
        int32_t *cnt = s_cnt + 4 * (round & 1);  // alternate, so one barrier a round
        if ((threadIdx.x & 63) == 0) cnt[w] = c;
        __syncthreads();
        const int32_t step0 = (hi0 - lo0 + 127) / 128, step1 = (hi1 - lo1 + 127) / 128;
        if (hi0 - lo0 > 1) {
            const int32_t n0 = lo0 + (cnt[0] + cnt[1]) * step0;
            hi0 = n0 + step0 < hi0 ? n0 + step0 : hi0;
            lo0 = n0;
        }
        if (hi1 - lo1 > 1) {
            const int32_t n1 = lo1 + (cnt[2] + cnt[3]) * step1;
            hi1 = n1 + step1 < hi1 ? n1 + step1 : hi1;
            lo1 = n1;
        }
    }
    d0 = lo0;
    d1 = lo1;
}

__device__ inline uint32_t *max_word(double *scale, int32_t d) {
    return reinterpret_cast<uint32_t *>(scale + d);
}

__global__ void k_qinit(double *scale, int32_t D) {
    int32_t d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < D) scale[d] = 0.0;
}

// Element (t, k) of a block is b0 + t + QT*k, so every load and store of a
// wave covers 64 consecutive elements.  Blocks whose elements all lie in one
// distribution reduce in LDS and issue one atomic; blocks that straddle
// distributions flush per lane and segment.
__global__ __launch_bounds__(QT) void k_qmax(const float *__restrict__ v,
                                             const int64_t *__restrict__ off, int32_t D,
                                             int64_t n, double *scale, uint32_t *status) {
    __shared__ uint32_t s_max[QT / 64];
    __shared__ uint32_t s_dmax[QMAX_LDS_DISTS];
    __shared__ int32_t s_cnt[8];
    __shared__ int s_bad;
    const int64_t b0 = (int64_t)blockIdx.x * QT * QI;
    const int64_t b1 = b0 + (int64_t)QT * QI < n ? b0 + (int64_t)QT * QI : n;
    // all of the thread's loads first (clamped, in range), so that they and
    // the search for the block's first distribution are in flight together
    float xs[QI];
#pragma unroll
    for (int k = 0; k < QI; ++k) {
        const int64_t i = b0 + threadIdx.x + (int64_t)QT * k;
        xs[k] = v[i < n ? i : n - 1];
    }
    int32_t dfirst = 0, dlast = 0;
    if (off) block_find_two(off, D, b0, b1 - 1, s_cnt, dfirst, dlast);
    const bool one = dlast == dfirst;
    // a block over a few distributions collects their maxima in LDS and adds
    // each to global memory once; only one over very many uses global atomics
    const bool lds = !one && dlast - dfirst < QMAX_LDS_DISTS;
    if (threadIdx.x == 0) s_bad = 0;
    if (lds)
        for (int32_t q = threadIdx.x; q <= dlast - dfirst; q += QT) s_dmax[q] = 0u;
    __syncthreads();
    int32_t d = dfirst;
    int64_t dend = off ? off[d + 1] : n;
    uint32_t mx = 0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < QI; ++k) {
        const int64_t i = b0 + threadIdx.x + (int64_t)QT * k;
        if (i >= b1) break;
        if (!one) {
            // d stays within [dfirst, dlast] even for offsets that break the
            // rules, so the LDS slots and the maxima stay in bounds
            while (i >= dend && d < dlast) {
                if (mx) {
                    if (lds) atomicMax(s_dmax + (d - dfirst), mx);
                    else atomicMax(max_word(scale, d), mx);
                }
                mx = 0;
                ++d;
                dend = off[d + 1];
            }
        }
        const float x = xs[k];
        if (!(x >= 0.0f) || isinf(x)) {
            bad = true;
            continue;
        }
        // -0.0 passes the sign test; dropping the sign bit maps it to 0, so
        // it cannot win the unsigned maximum over the positive weights
        const uint32_t b = __float_as_uint(x) & 0x7fffffffu;
        mx = b > mx ? b : mx;
    }
    if (bad) s_bad = 1;
    if (one) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t y = __shfl_down(mx, o, 64);
            mx = y > mx ? y : mx;
        }
        if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t m = 0;
            for (int w = 0; w < QT / 64; ++w) m = s_max[w] > m ? s_max[w] : m;
            // the maximum only grows, so a block whose value does not exceed
            // what it reads skips the atomic (a stale read is low, which just
            // means one more atomic); this keeps thousands of blocks of one
            // large distribution from serialising on one address
            const uint32_t seen = __hip_atomic_load(max_word(scale, dfirst), __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
            if (m > seen) atomicMax(max_word(scale, dfirst), m);
            if (s_bad && status) atomicOr(status, status_bit(RTF_ERR_VALUE));
        }
    } else {
        if (mx) {
            if (lds) atomicMax(s_dmax + (d - dfirst), mx);
            else atomicMax(max_word(scale, d), mx);
        }
        __syncthreads();
        if (lds)
            for (int32_t q = threadIdx.x; q <= dlast - dfirst; q += QT)
                if (s_dmax[q]) atomicMax(max_word(scale, dfirst + q), s_dmax[q]);
        if (threadIdx.x == 0 && s_bad && status) atomicOr(status, status_bit(RTF_ERR_VALUE));
    }
}

// One distribution: a fixed grid strides over the weights with 16-byte
// loads, so only a few thousand blocks reach the atomic.
constexpr int QMAX_BLOCKS = 1024;  // fewer blocks, fewer atomics on the one maximum
__global__ __launch_bounds__(QT) void k_qmax_single(const float *__restrict__ v, int64_t n,
                                                    bool vec, double *scale, uint32_t *status) {
    __shared__ uint32_t s_max[QT / 64];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    uint32_t mx = 0;
    bool bad = false;
    auto take = [&](float x) {
        if (!(x >= 0.0f) || isinf(x)) {
            bad = true;
            return;
        }
        const uint32_t b = __float_as_uint(x) & 0x7fffffffu;  // -0.0 counts as 0
        mx = b > mx ? b : mx;
    };
    const int64_t stride = (int64_t)gridDim.x * QT;
    const int64_t n4 = vec ? n / 4 : 0;
    const float4 *v4 = reinterpret_cast<const float4 *>(v);
    // four 16-byte loads per thread in flight; an index past the end is
    // clamped to the last vector, which a maximum may read twice
    constexpr int QU = 4;
    for (int64_t i0 = (int64_t)blockIdx.x * QT + threadIdx.x; i0 < n4; i0 += stride * QU) {
        float4 xq[QU];
#pragma unroll
        for (int k = 0; k < QU; ++k) {
            const int64_t i = i0 + stride * k;
            xq[k] = v4[i < n4 ? i : n4 - 1];
        }
#pragma unroll
        for (int k = 0; k < QU; ++k) {
            take(xq[k].x);
            take(xq[k].y);
            take(xq[k].z);
            take(xq[k].w);
        }
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * QT + threadIdx.x; i < n; i += stride) take(v[i]);
    if (bad) s_bad = 1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_down(mx, o, 64);
        mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = 0;
        for (int w = 0; w < QT / 64; ++w) m = s_max[w] > m ? s_max[w] : m;
        const uint32_t seen = __hip_atomic_load(max_word(scale, 0), __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        if (m > seen) atomicMax(max_word(scale, 0), m);
        if (s_bad && status) atomicOr(status, status_bit(RTF_ERR_VALUE));
    }
}

__device__ inline double scale_of(const double *scale, int32_t d) {
    const float mx = __uint_as_float(*reinterpret_cast<const uint32_t *>(scale + d));
    return mx > 0.0f ? 4294967295.0 / (double)mx : 0.0;
}

// One distribution: scale[0] holds either the maximum's float bits in its low
// word (high word zero, as k_qinit and k_qmax_single leave it) or the final
// scale, which block 0 of k_qapply writes while other blocks may still read.
// The two are told apart by the high word: a scale of a positive maximum is
// at least (2^32 - 1) / FLT_MAX, about 1.3e-29, so its exponent bits are not
// zero, and a scale of 0 decodes as a maximum of 0.  Both forms give the same
// bits of s.
__device__ inline double scale_single(const double *scale) {
    const uint64_t word = __hip_atomic_load(reinterpret_cast<const uint64_t *>(scale),
                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (word >> 32) return __longlong_as_double((long long)word);
    const float mx = __uint_as_float((uint32_t)word);
    return mx > 0.0f ? 4294967295.0 / (double)mx : 0.0;
}

__global__ __launch_bounds__(QT) void k_qapply(const float *__restrict__ v,
                                               const int64_t *__restrict__ off, int32_t D,
                                               int64_t n, double *scale,
                                               uint32_t *__restrict__ out) {
    const int64_t b0 = (int64_t)blockIdx.x * QT * QI;
    const int64_t b1 = b0 + (int64_t)QT * QI < n ? b0 + (int64_t)QT * QI : n;
    float xs[QI];  // every load in flight before the distribution search
#pragma unroll
    for (int k = 0; k < QI; ++k) {
        const int64_t i = b0 + threadIdx.x + (int64_t)QT * k;
        xs[k] = v[i < n ? i : n - 1];
    }
    int32_t d = off ? block_find_segment(off, D, b0) : 0;
    int64_t dend = off ? off[d + 1] : n;
    double s = off ? scale_of(scale, d) : scale_single(scale);
    if (!off && blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_store(reinterpret_cast<uint64_t *>(scale), (uint64_t)__double_as_longlong(s),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int k = 0; k < QI; ++k) {
        const int64_t i = b0 + threadIdx.x + (int64_t)QT * k;
        if (i >= b1) break;
        if (i >= dend) {
            while (i >= dend && d + 1 < D) {  // d < D for any offsets
                ++d;
                dend = off[d + 1];
            }
            s = scale_of(scale, d);
        }
        const float x = xs[k];
        uint32_t q = 0;
        if (x > 0.0f && !isinf(x)) {
            double y = rint((double)x * s);
            y = y < 1.0 ? 1.0 : y;
            y = y > 4294967295.0 ? 4294967295.0 : y;
            q = (uint32_t)y;
        }
        out[i] = q;
    }
}

__global__ void k_qfinal(double *scale, int32_t D) {
    int32_t d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= D) return;
    const float mx = __uint_as_float(*reinterpret_cast<const uint32_t *>(scale + d));
    scale[d] = mx > 0.0f ? 4294967295.0 / (double)mx : 0.0;
}

}  // namespace

hipError_t launch_quantize(const float *v, const int64_t *elem_off, int32_t D, int64_t n_total,
                           uint32_t *out, double *scale, uint32_t *status, hipStream_t st) {
    const int db = (D + 255) / 256;
    const int64_t nb = (n_total + (int64_t)QT * QI - 1) / ((int64_t)QT * QI);
    hipLaunchKernelGGL(k_qinit, dim3(db), dim3(256), 0, st, scale, D);
    if (elem_off) {
        hipLaunchKernelGGL(k_qmax, dim3((unsigned)nb), dim3(QT), 0, st, v, elem_off, D, n_total,
                           scale, status);
    } else {
        const int64_t g = nb < QMAX_BLOCKS ? nb : QMAX_BLOCKS;
        const bool vec = (reinterpret_cast<uintptr_t>(v) & 15) == 0;
        hipLaunchKernelGGL(k_qmax_single, dim3((unsigned)g), dim3(QT), 0, st, v, n_total, vec,
                           scale, status);
    }
    hipLaunchKernelGGL(k_qapply, dim3((unsigned)nb), dim3(QT), 0, st, v, elem_off, D, n_total,
                       scale, out);
    // one distribution's scale is written by k_qapply itself
    if (elem_off) hipLaunchKernelGGL(k_qfinal, dim3(db), dim3(256), 0, st, scale, D);
    return hipGetLastError();
}

}  // namespace rtf
