// rtf_alias.hip -- the Alias Method (Sec. 2.6; Walker's table of cells that
// hold at most two intervals, Fig. alias_map), the non-monotone comparison
// mapping of the paper's quality study (Figs. results_sine64, 2d_zoom,
// convergence).  It is not on the inversion path; it exists so that the
// same uniforms can be pushed through both mappings on the GPU.
//
// Table (exact integers): item i of a distribution of n weights carries the
// mass w_i n, a cell holds W = sum w.  Record j = { thr_j, alias_j }: the part
// thr_j in [0, W] of cell j kept by item j, the rest going to alias_j.
// Construction: Vose's two-worklist method ("A linear algorithm for
// generating random numbers with a given distribution", IEEE TSE 1991) in a
// fixed order -- items of mass below W ("small") and at least W ("large") on
// two stacks in increasing index order; each step pops one of each, gives the
// small item's cell remainder to the large item, and pushes the large item
// back on the stack its remaining mass belongs to; large items left at the
// end keep their whole cell.  The setup is serial per distribution (the
// paper's remark in Sec. 2.6): one thread per distribution, the stacks in
// the workspace.
//
// Sampling: xi = u 2^-64 lies in cell j = floor(u n / 2^64) at offset
// r = (u n) mod 2^64; the item is j when floor(r W / 2^64) < thr_j, else
// alias_j (exact: f < thr/W  <=>  r W < thr 2^64).
#include "rtf_internal.h"

namespace rtf {

namespace {

struct alignas(16) AliasRec {
    uint64_t thr;
    int32_t alias;
    int32_t pad;
};

// One thread per distribution: the total, the masses, the two stacks, the
// pairing.  recs, small and large cover the distribution's own range.
__global__ __launch_bounds__(64) void k_alias_build(const uint32_t *__restrict__ w,
                                                    const int64_t *__restrict__ eoff, int32_t D,
                                                    AliasRec *__restrict__ recs,
                                                    int32_t *__restrict__ small_st,
                                                    int32_t *__restrict__ large_st,
                                                    uint64_t *__restrict__ Wd,
                                                    uint32_t *__restrict__ status) {
    const int32_t d = (int32_t)(blockIdx.x * 64 + threadIdx.x);
    if (d >= D) return;
    const int64_t e0 = eoff[d], e1 = eoff[d + 1];
    const int64_t n = e1 - e0;
    uint64_t W = 0;
    for (int64_t i = e0; i < e1; ++i) W += w[i];
    Wd[d] = W;
    if (W == 0) {
        atomicOr(status, status_bit(RTF_ERR_ZERO_TOTAL));
        return;
    }
    int32_t *sm = small_st + e0, *lg = large_st + e0;
    int64_t ns = 0, nl = 0;
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t mass = (uint64_t)w[e0 + i] * (uint64_t)n;
        recs[e0 + i].thr = mass;
        recs[e0 + i].alias = (int32_t)i;
        recs[e0 + i].pad = 0;
        if (mass < W) sm[ns++] = (int32_t)i;
        else lg[nl++] = (int32_t)i;
    }
    while (ns > 0 && nl > 0) {
        const int32_t s = sm[--ns], l = lg[--nl];
        recs[e0 + s].alias = l;
        const uint64_t rest = recs[e0 + l].thr - (W - recs[e0 + s].thr);
        recs[e0 + l].thr = rest;
        if (rest < W) sm[ns++] = l;
        else lg[nl++] = l;
    }
    while (nl > 0) {  // mass exactly W: the cell is the item's own
        const int32_t l = lg[--nl];
        recs[e0 + l].thr = W;
        recs[e0 + l].alias = l;
    }
    if (ns > 0) atomicOr(status, status_bit(RTF_ERR_VALUE));  // cannot happen with exact sums
}

__device__ inline int32_t alias_pick(const AliasRec *__restrict__ recs, int64_t e0, int64_t n,
                                     uint64_t W, uint64_t u) {
    const uint64_t j = mulhi64(u, (uint64_t)n);
    const uint64_t r = u * (uint64_t)n;
    const uint64_t t = mulhi64(r, W);
    const uint4 v = *reinterpret_cast<const uint4 *>(recs + e0 + (int64_t)j);
    const uint64_t thr = ((uint64_t)v.y << 32) | v.x;
    return t < thr ? (int32_t)j : (int32_t)v.z;
}

constexpr int AT = 256;

// Samples of one distribution each: sample s belongs to distribution d with
// sample_off[d] <= s < sample_off[d+1] (one distribution: sample_off null).
__global__ __launch_bounds__(AT) void k_alias_sample(const AliasRec *__restrict__ recs,
                                                     const int64_t *__restrict__ eoff,
                                                     const uint64_t *__restrict__ Wd, int32_t D,
                                                     const int64_t *__restrict__ soff,
                                                     const uint64_t *__restrict__ u, int64_t S,
                                                     int32_t *__restrict__ idx) {
    const int64_t s = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (s >= S) return;
    int32_t d = 0;
    if (soff) {
        int32_t lo = 0, hi = D;  // last d with soff[d] <= s
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (soff[mid] <= s) lo = mid;
            else hi = mid;
        }
        d = lo;
    }
    const int64_t e0 = eoff[d], n = eoff[d + 1] - e0;
    const uint64_t W = Wd[d];
    idx[s] = W == 0 ? -1 : alias_pick(recs, e0, n, W, u[s]);
}

// Pairs: distribution 0 is the marginal over the R = D - 1 rows, row r is
// distribution r + 1; u2[2s] picks the row, u2[2s+1] the column.
__global__ __launch_bounds__(AT) void k_alias_sample_2d(const AliasRec *__restrict__ recs,
                                                        const int64_t *__restrict__ eoff,
                                                        const uint64_t *__restrict__ Wd, int32_t D,
                                                        const uint64_t *__restrict__ u2, int64_t S,
                                                        int32_t *__restrict__ rc) {
    const int64_t s = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (s >= S) return;
    const uint4 uv = *reinterpret_cast<const uint4 *>(u2 + 2 * s);
    const uint64_t ua = ((uint64_t)uv.y << 32) | uv.x, ub = ((uint64_t)uv.w << 32) | uv.z;
    const uint64_t Wm = Wd[0];
    int32_t r = -1, c = -1;
    if (Wm != 0) {
        r = alias_pick(recs, 0, eoff[1], Wm, ua);
        if (r + 1 < D) {  // the marginal must have one item per row table 1..D-1
            const int64_t e0 = eoff[r + 1], n = eoff[r + 2] - e0;
            const uint64_t W = Wd[r + 1];
            c = W == 0 ? -1 : alias_pick(recs, e0, n, W, ub);
        } else {
            r = -1;
        }
    }
    *reinterpret_cast<int2 *>(rc + 2 * s) = make_int2(r, c);
}

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct AliasLayout {
    size_t status, recs, W, eoff, small_st, large_st, total;
};

AliasLayout alias_layout(int32_t D, int64_t n) {
    AliasLayout L;
    size_t o = 0;
    L.status = o;
    o = a256(o + 256);
    L.recs = o;
    o = a256(o + sizeof(AliasRec) * (size_t)n);
    L.W = o;
    o = a256(o + sizeof(uint64_t) * (size_t)D);
    L.eoff = o;
    o = a256(o + sizeof(int64_t) * (size_t)(D + 1));
    L.small_st = o;
    o = a256(o + sizeof(int32_t) * (size_t)n);
    L.large_st = o;
    o = a256(o + sizeof(int32_t) * (size_t)n);
    L.total = o;
    return L;
}

__global__ void k_alias_offsets(const int64_t *src, int32_t D, int64_t n, int64_t *dst,
                                uint32_t *status) {
    for (int64_t q = threadIdx.x; q <= D; q += blockDim.x) dst[q] = src ? src[q] : (q ? n : 0);
    if (threadIdx.x == 0) *status = 0u;
}

constexpr int64_t MAX_ALIAS_N = 2147483647;

bool alias_ok(const rtf_alias_table *t) {
    return t && t->recs && t->W && t->elem_off && t->status && t->D >= 1 && t->n_total >= t->D;
}

}  // namespace

}  // namespace rtf

using namespace rtf;

extern "C" {

size_t rtf_alias_workspace_bytes(int32_t D, int64_t n_total) {
    if (D < 1 || n_total < D || n_total > MAX_ALIAS_N) return 0;
    return alias_layout(D, n_total).total;
}

rtf_status rtf_alias_build(const uint32_t *w, const int64_t *elem_off, int32_t D, int64_t n_total,
                           void *ws, size_t ws_bytes, hipStream_t stream, rtf_alias_table *out) {
    if (!w || !ws || !out || (D > 1 && !elem_off)) return RTF_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) || (reinterpret_cast<uintptr_t>(w) & 3))
        return RTF_ERR_INVALID_ARG;
    if (D < 1 || n_total < D) return RTF_ERR_INVALID_ARG;
    if (n_total > MAX_ALIAS_N) return RTF_ERR_SIZE;
    const AliasLayout L = alias_layout(D, n_total);
    if (ws_bytes < L.total) return RTF_ERR_WORKSPACE;
    char *b = static_cast<char *>(ws);
    rtf_alias_table t;
    t.D = D;
    t.n_total = n_total;
    t.recs = b + L.recs;
    t.W = reinterpret_cast<uint64_t *>(b + L.W);
    t.elem_off = reinterpret_cast<int64_t *>(b + L.eoff);
    t.status = reinterpret_cast<uint32_t *>(b + L.status);
    hipLaunchKernelGGL(k_alias_offsets, dim3(1), dim3(256), 0, stream, D > 1 ? elem_off : nullptr,
                       D, n_total, t.elem_off, t.status);
    hipLaunchKernelGGL(k_alias_build, dim3((unsigned)((D + 63) / 64)), dim3(64), 0, stream, w,
                       t.elem_off, D, static_cast<AliasRec *>(t.recs),
                       reinterpret_cast<int32_t *>(b + L.small_st),
                       reinterpret_cast<int32_t *>(b + L.large_st), t.W, t.status);
    if (hipGetLastError() != hipSuccess) return RTF_ERR_HIP;
    *out = t;
    return RTF_OK;
}

rtf_status rtf_alias_sample(const rtf_alias_table *t, const int64_t *sample_off, const uint64_t *u,
                            int64_t S, int32_t *out_idx, hipStream_t stream) {
    if (!alias_ok(t) || S < 0 || (t->D > 1 && !sample_off)) return RTF_ERR_INVALID_ARG;
    if (S == 0) return RTF_OK;
    if (!u || !out_idx || (reinterpret_cast<uintptr_t>(u) & 7) || (reinterpret_cast<uintptr_t>(out_idx) & 3))
        return RTF_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_alias_sample, dim3((unsigned)((S + AT - 1) / AT)), dim3(AT), 0, stream,
                       static_cast<const AliasRec *>(t->recs), t->elem_off, t->W, t->D,
                       t->D > 1 ? sample_off : nullptr, u, S, out_idx);
    return hipGetLastError() == hipSuccess ? RTF_OK : RTF_ERR_HIP;
}

rtf_status rtf_alias_sample_2d(const rtf_alias_table *t, const uint64_t *u2, int64_t S,
                               int32_t *out_rc, hipStream_t stream) {
    if (!alias_ok(t) || t->D < 2 || S < 0) return RTF_ERR_INVALID_ARG;
    if (S == 0) return RTF_OK;
    if (!u2 || !out_rc || (reinterpret_cast<uintptr_t>(u2) & 15) ||
        (reinterpret_cast<uintptr_t>(out_rc) & 7))
        return RTF_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_alias_sample_2d, dim3((unsigned)((S + AT - 1) / AT)), dim3(AT), 0, stream,
                       static_cast<const AliasRec *>(t->recs), t->elem_off, t->W, t->D, u2, S,
                       out_rc);
    return hipGetLastError() == hipSuccess ? RTF_OK : RTF_ERR_HIP;
}

rtf_status rtf_alias_export(const rtf_alias_table *t, uint64_t *h_thr, int32_t *h_alias,
                            uint64_t *h_W, hipStream_t stream) {
    if (!alias_ok(t)) return RTF_ERR_INVALID_ARG;
    if (hipStreamSynchronize(stream) != hipSuccess) return RTF_ERR_HIP;
    uint32_t st = 0;
    if (hipMemcpy(&st, t->status, sizeof st, hipMemcpyDeviceToHost) != hipSuccess) return RTF_ERR_HIP;
    if (h_thr || h_alias) {
        AliasRec *tmp = static_cast<AliasRec *>(malloc(sizeof(AliasRec) * (size_t)t->n_total));
        if (!tmp) return RTF_ERR_INVALID_ARG;
        const hipError_t e = hipMemcpy(tmp, t->recs, sizeof(AliasRec) * (size_t)t->n_total,
                                       hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            for (int64_t i = 0; i < t->n_total; ++i) {
                if (h_thr) h_thr[i] = tmp[i].thr;
                if (h_alias) h_alias[i] = tmp[i].alias;
            }
        free(tmp);
        if (e != hipSuccess) return RTF_ERR_HIP;
    }
    if (h_W && hipMemcpy(h_W, t->W, sizeof(uint64_t) * (size_t)t->D, hipMemcpyDeviceToHost) !=
                   hipSuccess)
        return RTF_ERR_HIP;
    for (int c = 1; c < 32; ++c)
        if (st & (1u << c)) return static_cast<rtf_status>(c);
    return RTF_OK;
}

}  // extern "C"
