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
// k_bscatter accumulates A, B, D; k_bhead, k_bcarry and k_bfinal do the
// suffix sum of B segmented by distribution.  A block whose samples all belong to one distribution
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
            // w_i < 2^32 for a sampled i (a skipped sample's values are dropped)
            const double wi = (double)(uint32_t)(Cn - Ci);
            const double rw = recip_small(__builtin_fmax(wi, 1.0));
            const double frac = ((double)(uint32_t)(t - Ci) + ldexp((double)lo, -64)) * rw;
            const double xi = ldexp((double)us[q], -64);
            const double a = g[q] * (sq[q] / (double)P.n) * rw;
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
    const double sn = sc / (double)n;  // a = g sc / (n w_i): the block's factor
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
            const double rw = recip_small(__builtin_fmax(wi, 1.0));  // w_i >= 1 for a sampled i
            const double frac = ((double)(uint32_t)((uint32_t)t - ci) + ldexp((double)lo, -64)) * rw;
            const double xi = ldexp((double)us[q], -64);
            const double a = g[q] * sn * rw;
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

// ---------------------------------------------------------------------------
// The combining pass: grad[k] = A_d - sum_{j > k, j in d} B_j - D_k, a suffix
// sum of B segmented by distribution, over the whole element range so that
// one large distribution spreads over the whole GPU.  The elements are cut
// into chunks of CCH; a chunk's own part of the suffix sum is a block-wide
// segmented scan, and the part from later chunks is a carry per chunk:
//   k_bhead    per chunk: the sum of B over its elements that belong to the
//              distribution of its first element, and whether the
//              distribution of its last element continues past it;
//   k_bcarry   one block: carry[c] = sum of B over the elements after chunk c
//              of the distribution of its last element, a segmented suffix
//              scan over the chunks;
//   k_bfinal   per chunk: the in-chunk segmented suffix scan plus the carry.
// ---------------------------------------------------------------------------
constexpr int CE = 4;           // elements per thread of a chunk
constexpr int CCH = CB * CE;    // elements per chunk
static_assert(CCH == BACKWARD_CHUNK, "chunk of the combining pass");
constexpr int CARRY_PER = 4;    // chunks per thread and round of k_bcarry

// One term of a segmented sum: f marks that a segment starts at this term
// (so nothing before it is added).  join(a, b), a before b in scan order.
struct SegSum {
    double v;
    int f;
};
__device__ inline SegSum seg_join(SegSum a, SegSum b) {
    SegSum r;
    r.v = b.f ? b.v : a.v + b.v;
    r.f = a.f | b.f;
    return r;
}

// Block-wide segmented scan in thread order: returns the join of the terms
// of all threads before this one (the identity {0, 0} for thread 0) and, in
// total, the join of all threads' terms.
template <int NT>
__device__ inline SegSum block_seg_excl(SegSum x, double *s_v, int *s_f, SegSum &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        SegSum y;
        y.v = __shfl_up(x.v, o, 64);
        y.f = __shfl_up(x.f, o, 64);
        if (lane >= o) x = seg_join(y, x);
    }
    if (lane == 63) {
        s_v[w] = x.v;
        s_f[w] = x.f;
    }
    SegSum prev;
    prev.v = __shfl_up(x.v, 1, 64);
    prev.f = __shfl_up(x.f, 1, 64);
    if (lane == 0) prev = SegSum{0.0, 0};
    __syncthreads();
    SegSum pre{0.0, 0}, tot{0.0, 0};
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const SegSum t{s_v[i], s_f[i]};
        if (i < w) pre = seg_join(pre, t);
        tot = seg_join(tot, t);
    }
    __syncthreads();
    total = tot;
    return seg_join(pre, prev);
}

// The distribution of the first and the last element of chunk [c0, c1), by
// two wave-wide searches (waves 0 and 1); valid in every thread.
__device__ inline void chunk_dists(const int64_t *eoff, int32_t D, int64_t c0, int64_t c1,
                                   int32_t *s_d, int32_t &dfirst, int32_t &dlast) {
    if (D == 1) {
        dfirst = dlast = 0;
        return;
    }
    const int w = threadIdx.x >> 6;
    if (w < 2) {
        const int32_t d = wave_upper_bound(eoff, D, w == 0 ? c0 : c1 - 1) - 1;
        if ((threadIdx.x & 63) == 0) s_d[w] = d;
    }
    __syncthreads();
    dfirst = s_d[0];
    dlast = s_d[1];
}

// head[c]: sum of B over chunk c's elements in the distribution of its first
// element; link[c]: bit 0 the chunk lies inside that distribution, bit 1 the
// distribution of its last element continues into the next chunk.
__global__ __launch_bounds__(CB) void k_bhead(const int64_t *__restrict__ eoff, int32_t D,
                                              int64_t n, const double *__restrict__ B,
                                              double *__restrict__ head, int32_t *__restrict__ link) {
    __shared__ int32_t s_d[2];
    __shared__ double s_red[CB / 64];
    const int64_t c = blockIdx.x;
    const int64_t c0 = c * CCH, c1 = c0 + CCH < n ? c0 + CCH : n;
    int32_t dfirst, dlast;
    chunk_dists(eoff, D, c0, c1, s_d, dfirst, dlast);
    const int64_t e_first = eoff[dfirst + 1], e_last = eoff[dlast + 1];
    const int64_t hend = e_first < c1 ? e_first : c1;
    double x = 0.0;
    for (int64_t k = c0 + threadIdx.x; k < hend; k += CB) x += B[k];
    const double t = block_sum<CB>(x, s_red);
    if (threadIdx.x == 0) {
        head[c] = t;
        link[c] = (e_first >= c1 ? 1 : 0) | (e_last > c1 ? 2 : 0);
    }
}

// carry[c] = [chunk c's last distribution continues] * (head[c+1] +
// [chunk c+1 lies inside it] * carry[c+1]): a segmented scan from the last
// chunk down, CB * CARRY_PER chunks per round, one block.
__global__ __launch_bounds__(CB) void k_bcarry(const double *__restrict__ head,
                                               const int32_t *__restrict__ link, int64_t nch,
                                               double *__restrict__ carry) {
    __shared__ double s_v[CB / 64];
    __shared__ int s_f[CB / 64];
    double carry_in = 0.0;  // carry of the chunk after the round
    for (int64_t top = nch - 1; top >= 0; top -= (int64_t)CB * CARRY_PER) {
        // thread T takes chunks top - CARRY_PER T - e, e = 0 .. CARRY_PER-1
        SegSum term[CARRY_PER], agg{0.0, 0};
#pragma unroll
        for (int e = 0; e < CARRY_PER; ++e) {
            const int64_t c = top - (int64_t)CARRY_PER * threadIdx.x - e;
            term[e] = SegSum{0.0, 1};
            if (c >= 0 && c + 1 < nch) {
                const int32_t lc = link[c];
                const bool cont = lc & 2;
                const bool through = cont && (link[c + 1] & 1);
                term[e] = SegSum{cont ? head[c + 1] : 0.0, through ? 0 : 1};
            }
            agg = seg_join(agg, term[e]);
        }
        SegSum total;
        SegSum run = block_seg_excl<CB>(agg, s_v, s_f, total);
#pragma unroll
        for (int e = 0; e < CARRY_PER; ++e) {
            const int64_t c = top - (int64_t)CARRY_PER * threadIdx.x - e;
            run = seg_join(run, term[e]);
            if (c >= 0) carry[c] = run.v + (run.f ? 0.0 : carry_in);
        }
        carry_in = total.v + (total.f ? 0.0 : carry_in);
    }
}

// grad[k] = A_d - (the in-chunk suffix sum of B after k within d) - (carry of
// the chunk when d continues past it) - D_k.  Thread T takes the elements
// c1 - 1 - (CE T + e), e = 0 .. CE-1 (scan order is descending k); a term
// starts a segment at the last element of its distribution.
__global__ __launch_bounds__(CB) void k_bfinal(const int64_t *__restrict__ eoff, int32_t D,
                                               int64_t n, const double *__restrict__ B,
                                               const double *__restrict__ Dv,
                                               const double *__restrict__ A,
                                               const double *__restrict__ carry,
                                               double *__restrict__ grad) {
    __shared__ int64_t s_off[CCH + 1];
    __shared__ int32_t s_d[2];
    __shared__ double s_v[CB / 64];
    __shared__ int s_f[CB / 64];
    const int64_t c = blockIdx.x;
    const int64_t c0 = c * CCH, c1 = c0 + CCH < n ? c0 + CCH : n;
    int32_t dfirst, dlast;
    chunk_dists(eoff, D, c0, c1, s_d, dfirst, dlast);
    // the ends of the chunk's distributions: s_off[q] = eoff[dfirst + 1 + q]
    const int32_t nd = dlast - dfirst + 1;  // <= CCH: every distribution holds an element
    for (int32_t q = threadIdx.x; q < nd; q += CB) s_off[q] = eoff[dfirst + 1 + q];
    __syncthreads();
    const double cin = carry[c];
    int64_t kk[CE];
    int32_t dq[CE];
    double b[CE];
    SegSum term[CE], agg{0.0, 0};
    // distribution of the thread's first (highest) element, then downwards
    const int64_t ktop = c1 - 1 - (int64_t)CE * threadIdx.x;
    int32_t lo = 0, hi = nd;  // first q with s_off[q] > ktop
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (s_off[mid] <= ktop) lo = mid + 1;
        else hi = mid;
    }
    int32_t q = lo < nd ? lo : nd - 1;
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        const int64_t k = ktop - e;
        kk[e] = k;
        const bool ok = k >= c0;
        while (ok && q > 0 && s_off[q - 1] > k) --q;
        dq[e] = q;
        b[e] = ok ? B[k] : 0.0;
        term[e] = SegSum{b[e], ok && s_off[q] == k + 1 ? 1 : 0};
        agg = seg_join(agg, term[e]);
    }
    SegSum total;
    SegSum run = block_seg_excl<CB>(agg, s_v, s_f, total);
#pragma unroll
    for (int e = 0; e < CE; ++e) {
        run = seg_join(run, term[e]);
        const int64_t k = kk[e];
        if (k < c0) continue;
        const int32_t d = dfirst + dq[e];
        const double right = run.v - b[e] + (d == dlast ? cin : 0.0);
        grad[k] = A[d] - right - Dv[k];
    }
}

}  // namespace

hipError_t launch_backward(const Node *nodes, const Dist *dists, const int64_t *elem_off,
                           int32_t D, int64_t n_total, const int64_t *sample_off,
                           const uint64_t *u, const int32_t *idx, const double *gx, int64_t S,
                           const double *scale, double *grad_w, const BackwardScratch &w,
                           hipStream_t st) {
    int64_t zb = (n_total + 255) / 256;
    if (zb > 4096) zb = 4096;
    hipLaunchKernelGGL(k_bzero, dim3((unsigned)zb), dim3(256), 0, st, w.B, w.Dv, n_total, w.A,
                       D);
    if (S > 0) {
        const int64_t nb = (S + CHUNK - 1) / CHUNK;
        if (sample_off)
            hipLaunchKernelGGL(k_bscatter<true>, dim3((unsigned)nb), dim3(SB), 0, st, nodes, dists,
                               D, sample_off, u, idx, gx, S, scale, w.B, w.Dv, w.A);
        else
            hipLaunchKernelGGL(k_bscatter<false>, dim3((unsigned)nb), dim3(SB), 0, st, nodes, dists,
                               D, sample_off, u, idx, gx, S, scale, w.B, w.Dv, w.A);
    }
    const int64_t nch = backward_chunks(n_total);
    hipLaunchKernelGGL(k_bhead, dim3((unsigned)nch), dim3(CB), 0, st, elem_off, D, n_total, w.B,
                       w.head, w.link);
    hipLaunchKernelGGL(k_bcarry, dim3(1), dim3(CB), 0, st, w.head, w.link, nch, w.carry);
    hipLaunchKernelGGL(k_bfinal, dim3((unsigned)nch), dim3(CB), 0, st, elem_off, D, n_total, w.B,
                       w.Dv, w.A, w.carry, grad_w);
    return hipGetLastError();
}

}  // namespace rtf
