// rtf_backward.hip -- adjoint of the continuous position x (Sec. 5) with
// respect to the real weights v = q / scale, the sampled index held fixed.
//
// For sample s of distribution d with index i, xi = u 2^-64 and
// frac = ((t - C_i) + lo 2^-64) / w_i, x = (i + frac) / n_d with
// frac = (xi W - C_i) / w_i, so
//   dx/dv_k = (xi - [k < i] - [k == i] frac) / (n_d w_i)      (w in real units)
// and with a_s = g_s / (n_d w_{i_s}):
//   dL/dv_k = A_d - sum_{j > k} B_j - D_k,
//   A_d = sum_s a_s xi_s,  B_j = sum_{i_s = j} a_s,  D_j = sum_{i_s = j} a_s frac_s.
// k_bscatter accumulates A, B, D; k_bcombine does the segmented suffix sum of
// B per distribution.  A block whose samples all belong to one distribution
// of at most LBINS elements sums B and D in LDS first and adds each bin to
// global memory once; otherwise every sample adds with FP64 global atomics.
#include "rtf_internal.h"

namespace rtf {

namespace {

constexpr int CB = 1024;          // threads of the combining kernel (fewer chunk steps)
constexpr int SB = 1024;          // threads of a scatter block
constexpr int ILP = 2;            // samples a scatter thread loads at once
constexpr int CHUNK = SB * 128;   // samples per scatter block
constexpr int LBINS = 4096;       // bins a block can sum in LDS (2 x 32 KB)

__device__ inline int32_t find_segment_in(const int64_t *off, int32_t lo, int32_t hi, int64_t i) {
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_bzero(double *B, double *Dv, int64_t n, double *A, int32_t D) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        B[i] = 0.0;
        Dv[i] = 0.0;
        if (i < D) A[i] = 0.0;
    }
}

template <int NT>
__device__ inline double block_sum(double x, double *s_red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) s_red[w] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) t += s_red[i];
    __syncthreads();
    return t;  // valid in thread 0
}

// The samples [c0, c1) of one scatter block, ILP per thread and step, SB
// apart: all their stream loads are issued, then all their key loads, before
// any arithmetic, since the kernel is bound by the latency of these two
// dependent rounds (64 KB of LDS bins leave room for two blocks per CU).
// UNI: the block's samples all belong to distribution d0, whose parameters
// then stay in scalar registers.  acc accumulates a xi for distribution acc_d
// and is flushed to A when the distribution changes.
template <bool UNI>
__device__ inline void scatter_samples(const Node *__restrict__ nodes, const Dist *__restrict__ dists,
                                       const int64_t *__restrict__ soff, const uint64_t *__restrict__ u,
                                       const int32_t *__restrict__ idx, const double *__restrict__ gx,
                                       const double *__restrict__ scale, int64_t c0, int64_t c1,
                                       int32_t d0, int32_t d_last, double *B, double *Dv, double *A,
                                       double &acc, int32_t &acc_d) {
    int32_t d = d0;  // distribution of the thread's latest sample
    int64_t dend = UNI ? c1 : soff[d + 1];
    // the parameters are copied into registers: read through a reference they
    // would be fetched again after every atomic, one round trip each
    const Dist P0 = dists[d0];
    const double sc0 = scale[d0];
    for (int64_t s0 = c0 + threadIdx.x; s0 < c1; s0 += (int64_t)ILP * SB) {
        int32_t li[ILP], dq[ILP];
        uint64_t us[ILP];
        double g[ILP];
        // every load is unconditional (indices clamped into range), so that
        // all of them are in flight before the first wait
#pragma unroll
        for (int q = 0; q < ILP; ++q) {
            const int64_t s = s0 + (int64_t)q * SB;
            const int64_t sc = s < c1 ? s : c1 - 1;
            li[q] = idx[sc];
            us[q] = u[sc];
            g[q] = gx[sc];
        }
#pragma unroll
        for (int q = 0; q < ILP; ++q) {
            const int64_t s = s0 + (int64_t)q * SB;
            if (s >= c1) li[q] = -1;
            if (!UNI && s < c1 && s >= dend) {
                d = find_segment_in(soff, d, d_last + 1, s);
                dend = soff[d + 1];
            }
            dq[q] = UNI ? d0 : d;
        }
        uint64_t k0[ILP], k1[ILP];
        Dist Pq[ILP];
        double sq[ILP];
#pragma unroll
        for (int q = 0; q < ILP; ++q) {
            Pq[q] = UNI ? P0 : dists[dq[q]];
            sq[q] = UNI ? sc0 : scale[dq[q]];
        }
#pragma unroll
        for (int q = 0; q < ILP; ++q) {
            const Dist &P = Pq[q];
            const bool valid = li[q] >= 0 && li[q] < P.n && !(P.flags & DIST_ZERO);
            const int64_t lc = valid ? li[q] : 0;
            const bool last = lc + 1 >= P.n;
            const int64_t i = P.eo + lc;
            k0[q] = nodes[i].key;
            const uint64_t kn = nodes[last ? i : i + 1].key;
            k1[q] = last ? ~0ull : kn;
            if (!valid) li[q] = -1;
        }
        // the arithmetic runs for every sample (a skipped one yields values
        // that are discarded), which keeps the compiler from sinking the
        // loads above into the branch and waiting on them there
#pragma unroll
        for (int q = 0; q < ILP; ++q) {
            const Dist &P = Pq[q];
            const uint64_t W = P.W;
            const uint64_t Ci = mulhi64(k0[q], W);
            const uint64_t Cn = k1[q] != ~0ull ? mulhi64(k1[q], W) : W;
            const uint64_t t = mulhi64(us[q], W), lo = us[q] * W;
            const double wi = (double)(Cn - Ci);
            const double frac = ((double)(t - Ci) + ldexp((double)lo, -64)) / wi;
            const double xi = ldexp((double)us[q], -64);
            const double a = g[q] / ((double)P.n * (wi / sq[q]));
            const bool ok = li[q] >= 0;
            if (!UNI && ok && dq[q] != acc_d) {
                if (acc != 0.0) unsafeAtomicAdd(A + acc_d, acc);
                acc = 0.0;
                acc_d = dq[q];
            }
            acc += ok ? a * xi : 0.0;
            if (!ok) continue;
            const int64_t i = P.eo + li[q];
            unsafeAtomicAdd(B + i, a);
            unsafeAtomicAdd(Dv + i, a * frac);
        }
    }
}

// A block whose samples all belong to distribution P with n <= LBINS
// elements.  The low 32 bits of its partial sums C_k are staged in LDS
// (C_k = floor(U_k W / 2^64), and W for the trailing zero weights whose key
// is all ones): for the sampled i, 0 <= t - C_i < w_i < 2^32, so 32-bit
// differences give t - C_i and w_i = C_{i+1} - C_i exactly, and no sample
// reads a key from L2.  B and D are summed in LDS bins and added to global
// memory once per bin.
__device__ inline void scatter_local(const Node *__restrict__ nodes, const Dist P, double sc,
                                     const uint64_t *__restrict__ u, const int32_t *__restrict__ idx,
                                     const double *__restrict__ gx, int64_t c0, int64_t c1, double *s_b,
                                     double *s_d, uint32_t *s_clo, double &acc) {
    const int64_t n = P.n;
    for (int64_t k = threadIdx.x; k < n; k += SB) {
        const uint64_t key = nodes[P.eo + k].key;
        s_clo[k] = (uint32_t)(key == ~0ull ? P.W : mulhi64(key, P.W));
        s_b[k] = s_d[k] = 0.0;
    }
    __syncthreads();
    if (P.flags & DIST_ZERO) return;  // no sample of it has an index
    const uint32_t w_lo = (uint32_t)P.W;
    for (int64_t s0 = c0 + threadIdx.x; s0 < c1; s0 += (int64_t)ILP * SB) {
        int32_t li[ILP];
        uint64_t us[ILP];
        double g[ILP];
#pragma unroll
        for (int q = 0; q < ILP; ++q) {
            const int64_t s = s0 + (int64_t)q * SB;
            const int64_t sc_ = s < c1 ? s : c1 - 1;
            li[q] = idx[sc_];
            us[q] = u[sc_];
            g[q] = gx[sc_];
        }
#pragma unroll
        for (int q = 0; q < ILP; ++q) {
            const int64_t s = s0 + (int64_t)q * SB;
            const bool ok = s < c1 && li[q] >= 0 && li[q] < n;
            const int32_t lc = ok ? li[q] : 0;
            const uint32_t ci = s_clo[lc];
            const uint32_t cn = lc + 1 < n ? s_clo[lc + 1] : w_lo;
            const uint64_t t = mulhi64(us[q], P.W), lo = us[q] * P.W;
            const double wi = (double)(uint32_t)(cn - ci);
            const double frac = ((double)(uint32_t)((uint32_t)t - ci) + ldexp((double)lo, -64)) / wi;
            const double xi = ldexp((double)us[q], -64);
            const double a = g[q] / ((double)n * (wi / sc));
            acc += ok ? a * xi : 0.0;
            if (!ok) continue;
            atomicAdd(s_b + lc, a);
            atomicAdd(s_d + lc, a * frac);
        }
    }
}

template <bool BATCHED>
__global__ __launch_bounds__(SB) __attribute__((amdgpu_waves_per_eu(8))) void k_bscatter(
    const Node *__restrict__ nodes, const Dist *__restrict__ dists, int32_t D,
    const int64_t *__restrict__ soff, const uint64_t *__restrict__ u, const int32_t *__restrict__ idx,
    const double *__restrict__ gx, int64_t S, const double *__restrict__ scale, double *B, double *Dv,
    double *A) {
    // 80 KB, so that two blocks fit in a CU's 160 KB; the block sum reuses
    // the staged partial sums' space
    __shared__ double s_b[LBINS], s_d[LBINS];
    __shared__ uint32_t s_clo[LBINS];
    double *s_red = reinterpret_cast<double *>(s_clo);
    // chunks numbered per XCD: the 8 or so blocks of one distribution share
    // one L2
    const int64_t c0 = xcd_block() * CHUNK;
    const int64_t c1 = c0 + CHUNK < S ? c0 + CHUNK : S;
    const int32_t d_first = BATCHED ? find_segment_in(soff, 0, D, c0) : 0;
    const int32_t d_last = BATCHED ? find_segment_in(soff, d_first, D, c1 - 1) : 0;
    const bool uniform = d_first == d_last;
    const Dist P0 = dists[d_first];
    const bool local = uniform && P0.n <= LBINS;  // uniform across the block
    int32_t acc_d = d_first;
    double acc = 0.0;
    if (local)
        scatter_local(nodes, P0, scale[d_first], u, idx, gx, c0, c1, s_b, s_d, s_clo, acc);
    else if (uniform)
        scatter_samples<true>(nodes, dists, soff, u, idx, gx, scale, c0, c1, d_first, d_last, B, Dv, A, acc,
                              acc_d);
    else
        scatter_samples<false>(nodes, dists, soff, u, idx, gx, scale, c0, c1, d_first, d_last, B, Dv, A, acc,
                               acc_d);
    __syncthreads();
    if (local) {
        for (int64_t k = threadIdx.x; k < P0.n; k += SB) {
            if (s_b[k] != 0.0) unsafeAtomicAdd(B + P0.eo + k, s_b[k]);
            if (s_d[k] != 0.0) unsafeAtomicAdd(Dv + P0.eo + k, s_d[k]);
        }
    }
    if (uniform) {
        const double t = block_sum<SB>(acc, s_red);
        if (threadIdx.x == 0 && t != 0.0) unsafeAtomicAdd(A + d_first, t);
    } else if (acc != 0.0) {
        unsafeAtomicAdd(A + acc_d, acc);
    }
}

// One block per distribution: grad[k] = A - sum_{j>k} B_j - D_k, scanning the
// distribution from its end in chunks of CB elements.
__global__ __launch_bounds__(CB) void k_bcombine(const Dist *__restrict__ dists,
                                                 const double *__restrict__ B,
                                                 const double *__restrict__ Dv,
                                                 const double *__restrict__ A,
                                                 double *__restrict__ grad) {
    __shared__ double s_w[CB / 64];
    const Dist P = dists[blockIdx.x];
    const double Ad = A[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double carry = 0.0;  // sum of B over elements after the current chunk
    for (int64_t end = P.eo + P.n; end > P.eo; end -= CB) {
        // element handled by this thread: end-1-threadIdx.x (reverse order)
        const int64_t k = end - 1 - threadIdx.x;
        const bool ok = k >= P.eo;
        const double b = ok ? B[k] : 0.0;
        // inclusive scan over threads in reverse element order
        double x = b;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            double y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        double off = 0.0, tot = 0.0;
#pragma unroll
        for (int i = 0; i < CB / 64; ++i) {
            off += (i < w) ? s_w[i] : 0.0;
            tot += s_w[i];
        }
        __syncthreads();
        // exclusive sum of B over elements right of k
        const double right = carry + off + x - b;
        if (ok) grad[k] = Ad - right - Dv[k];
        carry += tot;
    }
}

}  // namespace

hipError_t launch_backward(const Node *nodes, const Dist *dists, int32_t D, int64_t n_total,
                           const int64_t *sample_off, const uint64_t *u, const int32_t *idx,
                           const double *gx, int64_t S, const double *scale, double *grad_w,
                           double *wsB, double *wsDv, double *wsA, hipStream_t st) {
    int64_t zb = (n_total + 255) / 256;
    if (zb > 4096) zb = 4096;
    hipLaunchKernelGGL(k_bzero, dim3((unsigned)zb), dim3(256), 0, st, wsB, wsDv, n_total, wsA,
                       D);
    if (S > 0) {
        const int64_t nb = (S + CHUNK - 1) / CHUNK;
        if (sample_off)
            hipLaunchKernelGGL(k_bscatter<true>, dim3((unsigned)nb), dim3(SB), 0, st, nodes, dists,
                               D, sample_off, u, idx, gx, S, scale, wsB, wsDv, wsA);
        else
            hipLaunchKernelGGL(k_bscatter<false>, dim3((unsigned)nb), dim3(SB), 0, st, nodes, dists,
                               D, sample_off, u, idx, gx, S, scale, wsB, wsDv, wsA);
    }
    hipLaunchKernelGGL(k_bcombine, dim3((unsigned)D), dim3(CB), 0, st, dists, wsB, wsDv, wsA,
                       grad_w);
    return hipGetLastError();
}

}  // namespace rtf
