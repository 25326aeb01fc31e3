// rtf_sample.hip -- Alg. 2 (guide-table lookup plus tree descent), the
// continuous position of Sec. 5, the 2D component-by-component inversion of
// Sec. 5, and two baselines with the identical mapping (Sec. 4): binary search
// over all keys (Sec. 2.2) and the Cutpoint Method with bisection (Sec. 2.5).
#include "rtf_internal.h"

namespace rtf {

namespace {

// Index d with off[d] <= i < off[d+1] over off[0..D], found by a whole block
// of NT threads (uniform i): each round probes NT evenly spaced offsets, so
// 10^4 distributions take two dependent loads.  Every thread must call it.
template <int NT = 256>
__device__ inline int32_t block_find_segment(const int64_t *off, int32_t D, int64_t i) {
    int32_t lo = 0, hi = D;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int32_t step = (hi - lo + NT - 1) / NT;
        const int32_t p = lo + ((int32_t)threadIdx.x + 1) * step;
        const int below = (p < hi && off[p] <= i) ? 1 : 0;
        const int32_t nlo = lo + __syncthreads_count(below) * step;
        hi = nlo + step < hi ? nlo + step : hi;
        lo = nlo;
    }
    return lo;
}

constexpr int SCHUNK = 256 * 8;  // samples per block step of the batched kernel
constexpr int CHUNK_DISTS = 256;  // distributions a chunk can stage in LDS

static_assert(sizeof(Dist) == 64, "a staged record is four 16-byte words");
__device__ inline Dist lds_dist(const uint4 *s_dist, int32_t k) {
    Dist P;
    uint4 *q = reinterpret_cast<uint4 *>(&P);
#pragma unroll
    for (int w = 0; w < 4; ++w) q[w] = s_dist[4 * k + w];
    return P;
}

// index k in [lo, hi) with off[k] <= i < off[k+1], given off[lo] <= i < off[hi]
// (off may hold equal neighbours; the last k with off[k] <= i is taken)
__device__ inline int32_t find_segment_in(const int64_t *off, int32_t lo, int32_t hi, int64_t i) {
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ inline Node load_node(const Node *nodes, int64_t j) {
    uint4 v = *reinterpret_cast<const uint4 *>(nodes + j);
    Node r;
    r.key = ((uint64_t)v.y << 32) | v.x;
    r.c0 = (int32_t)v.z;
    r.c1 = (int32_t)v.w;
    return r;
}

__device__ inline Cell load_cell(const Cell *cells, int64_t g) {
    const uint4 *p = reinterpret_cast<const uint4 *>(cells + g);
    uint4 v[CELL_WORDS];
#pragma unroll
    for (int w = 0; w < CELL_WORDS; ++w) v[w] = p[w];  // all in flight together
    Cell r;
#pragma unroll
    for (int w = 0; w < CELL_WORDS; ++w) {
        r.k[2 * w] = ((uint64_t)v[w].y << 32) | v[w].x;
        if (w + 1 < CELL_WORDS) r.k[2 * w + 1] = ((uint64_t)v[w].w << 32) | v[w].z;
    }
    r.ref = (int32_t)v[CELL_WORDS - 1].z;
    r.aux = (int32_t)v[CELL_WORDS - 1].w;
    return r;
}

// Marks every word of a record as used here, so that the record's loads,
// issued before, complete together (one wait).  Without it, when x is not
// wanted, the compiler splits the record load along the branches that use
// each word: up to three round trips to the same line, one after another.
__device__ inline void pin_cell(Cell &c) {
#pragma unroll
    for (int t = 0; t < CELL_KEYS; ++t) asm volatile("" : "+v"(c.k[t]));
    asm volatile("" : "+v"(c.ref), "+v"(c.aux));
}

// A sampled leaf with the keys of its interval's two ends (KEY_END for the
// distribution's end); leaf -1 flags a damaged workspace.
struct Hit {
    int64_t i;
    uint64_t lo, hi;
};

// Alg. 2: g = floor(xi * m); follow the reference until it names a leaf.
// The cell record resolves the guide step and, for a cell that holds at most
// CELL_BOUNDS lower bounds (or for u below the record's last key), the whole
// sample: the leaf is a - 1 plus the number of the cell's lower bounds at or
// below u.  Otherwise the descent continues from the cell's tree root.  A
// reference outside the forest, or a path longer than the forest has nodes,
// can only come from a damaged workspace.
__device__ inline Hit resolve(const Node *nodes, const Wide *wide, const Cell &c, const Dist &P,
                              uint64_t u, int64_t n_total);

// floor(u m / 2^64) for distribution P's m cells, P the same for the whole
// wave: a shift when m is a power of two (the shift is in the distribution's
// flags), else the high word of the product
__device__ inline int64_t cell_in(const Dist &P, uint64_t u) {
    const uint32_t sh = P.flags >> DIST_SHIFT_BIT;
    return sh ? (int64_t)(u >> sh) : (int64_t)mulhi64(u, (uint64_t)P.m);
}

__device__ inline int64_t cell_index(const Dist &P, uint64_t u) {
    return P.co + (int64_t)mulhi64(u, (uint64_t)P.m);
}

__device__ inline Hit descend(const Node *nodes, const Wide *wide, const Cell *cells, const Dist &P,
                              uint64_t u, int64_t n_total) {
    Cell c = load_cell(cells, cell_index(P, u));
    pin_cell(c);
    return resolve(nodes, wide, c, P, u, n_total);
}

__device__ inline Wide load_wide(const Wide *wide, int64_t j) {
    const uint4 *p = reinterpret_cast<const uint4 *>(wide + j);
    const uint4 a = p[0], b = p[1], c = p[2];  // 48 bytes of one line, in flight together
    Wide r;
    r.k = ((uint64_t)a.y << 32) | a.x;
    r.kc[0] = ((uint64_t)a.w << 32) | a.z;
    r.kc[1] = ((uint64_t)b.y << 32) | b.x;
    r.r[0] = (int32_t)b.z;
    r.r[1] = (int32_t)b.w;
    r.r[2] = (int32_t)c.x;
    r.r[3] = (int32_t)c.y;
    return r;
}

// The sample's leaf from its cell record c (and, past the record, the tree).
// The record's own answer is computed for every kind of cell with selects
// only (a covered cell is a record holding no bounds); only a descent
// branches.
__device__ inline Hit resolve(const Node *nodes, const Wide *wide, const Cell &c, const Dist &P,
                              uint64_t u, int64_t n_total) {
    const bool covered = c.ref < 0;  // one interval covers the cell
    const int lim = covered ? 0 : (c.aux < 0 ? ~c.aux : CELL_BOUNDS);  // lower bounds held
    int j = 0;
    uint64_t lo = c.k[0], hi = c.k[1];
#pragma unroll
    for (int t = 1; t <= CELL_BOUNDS; ++t) {
        const bool le = t <= lim && c.k[t] <= u;
        j = le ? t : j;
        lo = le ? c.k[t] : lo;
        hi = le ? c.k[t + 1] : hi;
    }
    Hit h;
    h.i = covered ? ~(int64_t)c.ref : (int64_t)c.ref - 1 + j;
    h.lo = lo;
    h.hi = hi;
    if (!covered && c.aux >= 0 && u >= c.k[CELL_KEYS - 1]) {  // past the record: the tree
        // Both bounds adjacent to the sampled leaf i are its ancestors when
        // they lie inside the cell, so the descent meets U_i as the last key
        // at or below u and U_{i+1} as the last key above it; only when i is
        // the cell's last leaf is U_{i+1} read after the descent.
        uint64_t klo = c.k[CELL_KEYS - 1], khi = 0;
        bool hi_seen = false;
        int32_t jn = c.aux;
        if (wide) {
            // collapsed nodes: two binary levels per record (Sec. 5)
            for (int64_t steps = 0; jn >= 0; steps += 2) {
                if (jn >= n_total || steps > n_total) {
                    h.i = -1;
                    return h;
                }
                const Wide wn = load_wide(wide, jn);
                const bool right = u >= wn.k;
                klo = right ? wn.k : klo;
                khi = right ? khi : wn.k;
                hi_seen = hi_seen || !right;
                const int32_t g0 = right ? wn.r[2] : wn.r[0];
                const int32_t g1 = right ? wn.r[3] : wn.r[1];
                const uint64_t kc = right ? wn.kc[1] : wn.kc[0];
                if (g0 == g1) {  // the child is a leaf
                    jn = g0;
                } else {
                    const bool r2 = u >= kc;
                    klo = r2 ? kc : klo;
                    khi = r2 ? khi : kc;
                    hi_seen = hi_seen || !r2;
                    jn = r2 ? g1 : g0;
                }
            }
        } else {
            for (int64_t steps = 0; jn >= 0; ++steps) {
                if (jn >= n_total || steps > n_total) {
                    h.i = -1;
                    return h;
                }
                const Node nd = load_node(nodes, jn);
                const bool right = u >= nd.key;
                klo = right ? nd.key : klo;
                khi = right ? khi : nd.key;
                hi_seen = hi_seen || !right;
                jn = right ? nd.c1 : nd.c0;
            }
        }
        h.i = ~(int64_t)jn;
        if (h.i < P.eo || h.i >= P.eo + P.n) {
            h.i = -1;
            return h;
        }
        h.lo = klo;
        h.hi = hi_seen ? khi : ((h.i + 1 < P.eo + P.n) ? nodes[h.i + 1].key : KEY_END);
    }
    if (h.i < P.eo || h.i >= P.eo + P.n) h.i = -1;
    return h;
}

// x = (i + ((t - C_i) + lo * 2^-64) / w_i) / n with t:lo = u * W, where
// C_i = floor(U_i * W / 2^64) recovers the exact partial sum from a key.
// For the sampled i, 0 <= t - C_i < w_i = C_{i+1} - C_i < 2^32 and
// i - eo < 2^31, so those three convert to FP64 from 32 bits (one
// instruction each, and the same values).  The division by n is a product
// with 1/n, computed once where the distribution is the same for a whole
// loop; the result is kept at most 1 (it could round one ulp above 1 when
// the offset in the interval rounds up to w_i in the last leaf).
__device__ inline double position(const Dist &P, const Hit &h, uint64_t u) {
    const uint64_t W = P.W;
    const uint64_t Ci = mulhi64(h.lo, W);
    const uint64_t Cn = (h.hi == KEY_END) ? W : mulhi64(h.hi, W);
    const uint64_t t = mulhi64(u, W);
    const uint64_t lo = u * W;
    const double frac = div_small((double)(uint32_t)(t - Ci) + ldexp((double)lo, -64), (double)(uint32_t)(Cn - Ci));
    const double x = ((double)(int32_t)(h.i - P.eo) + frac) * (1.0 / (double)P.n);
    return __builtin_fmin(x, 1.0);
}

// The same, for a leaf found without its keys (the baselines).
__device__ inline double position_of(const Node *nodes, const Dist &P, int64_t i, uint64_t u) {
    Hit h;
    h.i = i;
    h.lo = nodes[i].key;
    h.hi = (i + 1 < P.eo + P.n) ? nodes[i + 1].key : KEY_END;
    return position(P, h, u);
}

template <bool BATCHED, bool WANT_X>
__global__ __launch_bounds__(256) void k_sample(const Node *__restrict__ nodes,
                                                const Wide *__restrict__ wide,
                                                const Cell *__restrict__ cells,
                                                const Dist *__restrict__ dists,
                                                const int64_t *__restrict__ sample_off,
                                                int32_t D, int64_t n_total,
                                                const uint64_t *__restrict__ u, int64_t S,
                                                int32_t *__restrict__ idx,
                                                double *__restrict__ x) {
    auto one = [&](int64_t s, const Dist &P) {
        const uint64_t us = __builtin_nontemporal_load(u + s);
        Hit h;
        h.i = -1;
        if (!(P.flags & DIST_ZERO)) h = descend(nodes, wide, cells, P, us, n_total);
        if (h.i < 0) {
            idx[s] = -1;
            if (WANT_X) x[s] = __builtin_nan("");
            return;
        }
        __builtin_nontemporal_store((int32_t)(h.i - P.eo), idx + s);
        if (WANT_X) __builtin_nontemporal_store(position(P, h, us), x + s);
    };
    if (!BATCHED) {
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += stride)
            one(s, dists[0]);
        return;
    }
    __shared__ int64_t s_soff[256];
    __shared__ uint4 s_dist[4 * CHUNK_DISTS];
    // batched: a block takes chunks of SCHUNK consecutive samples (numbered
    // per XCD, so that one XCD's L2 serves a few neighbouring distributions),
    // finds the chunk's first distribution once (block-wide), and each lane
    // steps on through the few distributions the chunk spans, two samples
    // 256 apart at a time with both samples' loads issued together.  A chunk
    // inside one distribution keeps its parameters in scalar registers.
    auto store = [&](int64_t s, const Dist &P, const Hit &h, uint64_t us) {
        if (h.i < 0) {
            idx[s] = -1;
            if (WANT_X) x[s] = __builtin_nan("");
            return;
        }
        __builtin_nontemporal_store((int32_t)(h.i - P.eo), idx + s);
        if (WANT_X) __builtin_nontemporal_store(position(P, h, us), x + s);
    };
    // two samples whose parameters are Pa and Pb, taken by value: through a
    // reference the fields would be fetched again after the stores
    auto two = [&](int64_t sa, int64_t sb, bool has_b, const Dist Pa, const Dist Pb) {
        const uint64_t ua = __builtin_nontemporal_load(u + sa);
        const uint64_t ub = __builtin_nontemporal_load(u + (has_b ? sb : sa));  // no branch
        const bool za = Pa.flags & DIST_ZERO, zb = Pb.flags & DIST_ZERO;
        Cell ca = load_cell(cells, za ? 0 : cell_index(Pa, ua));
        Cell cb = load_cell(cells, zb ? 0 : cell_index(Pb, ub));
        pin_cell(ca);
        pin_cell(cb);
        Hit ha, hb;
        ha.i = hb.i = -1;
        if (!za) ha = resolve(nodes, wide, ca, Pa, ua, n_total);
        if (!zb) hb = resolve(nodes, wide, cb, Pb, ub, n_total);
        store(sa, Pa, ha, ua);
        if (has_b) store(sb, Pb, hb, ub);
    };
    for (int64_t c0 = xcd_block() * SCHUNK; c0 < S; c0 += (int64_t)gridDim.x * SCHUNK) {
        int32_t d = __builtin_amdgcn_readfirstlane(block_find_segment(sample_off, D, c0));
        int64_t dend = sample_off[d + 1];
        const int64_t cend = c0 + SCHUNK < S ? c0 + SCHUNK : S;
        if (dend >= cend) {
            // the chunk lies in one distribution: its parameters are uniform
            const Dist P = dists[d];
#pragma unroll
            for (int k = 0; k < SCHUNK / 256; k += 2) {
                const int64_t sa = c0 + threadIdx.x + 256 * k, sb = sa + 256;
                if (sa >= cend) break;
                two(sa, sb, sb < cend, P, P);
            }
            continue;
        }
        // Several distributions: thread k reads offset d + k, and those below
        // the chunk's end count the distributions starting inside it.  With
        // fewer than CHUNK_DISTS of them their offsets and parameters are
        // staged in LDS, and each sample finds its own by a search there;
        // otherwise each lane walks the offsets in global memory.
        const int64_t ok = sample_off[d + (int32_t)threadIdx.x <= D ? d + (int32_t)threadIdx.x : D];
        s_soff[threadIdx.x] = ok;
        const int nb = __syncthreads_count(threadIdx.x > 0 && d + (int32_t)threadIdx.x < D && ok < cend);
        if (nb < CHUNK_DISTS - 1) {  // offsets d .. d + nb + 1 held, the last at or past cend
            const uint4 *src = reinterpret_cast<const uint4 *>(dists + d);
            for (int q = threadIdx.x; q < 4 * (nb + 1); q += 256) s_dist[q] = src[q];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < SCHUNK / 256; k += 2) {
                const int64_t sa = c0 + threadIdx.x + 256 * k, sb = sa + 256;
                if (sa >= cend) break;
                const bool has_b = sb < cend;
                const int32_t ka = find_segment_in(s_soff, 0, nb + 1, sa);
                const int32_t kb = has_b ? find_segment_in(s_soff, ka, nb + 1, sb) : ka;
                two(sa, sb, has_b, lds_dist(s_dist, ka), lds_dist(s_dist, kb));
            }
            __syncthreads();  // before the next chunk restages
            continue;
        }
#pragma unroll
        for (int k = 0; k < SCHUNK / 256; k += 2) {
            const int64_t sa = c0 + threadIdx.x + 256 * k, sb = sa + 256;
            if (sa >= S) break;
            // (d stays below D even for offsets that break the rules)
            while (sa >= dend && d + 1 < D) dend = sample_off[++d + 1];
            const int32_t da = d;
            const bool has_b = sb < S;
            if (has_b)
                while (sb >= dend && d + 1 < D) dend = sample_off[++d + 1];
            two(sa, sb, has_b, dists[da], dists[d]);
        }
        __syncthreads();  // s_soff is rewritten by the next chunk
    }
}

// Batched sampling with the guide cells staged in LDS, for batches with
// several samples per cell and distributions of at most LCELLS cells: a block
// of SB_T threads takes a contiguous share of the samples, walks it one
// distribution segment at a time, and copies a segment's cells into LDS when
// the segment has at least STAGE_MIN samples per cell, so that a sample reads
// its cell record from LDS and only the rare descents reach L2.  Copying a
// record streams 64 bytes, at most 32 per sample of the segment; a random L2
// read per sample costs more.
constexpr int SB_T = 1024;
constexpr int LCELLS = 1024;    // 64 KB of records: two blocks per CU
constexpr int STAGE_MIN = 2;
template <bool WANT_X>
__global__ __launch_bounds__(SB_T) __attribute__((amdgpu_waves_per_eu(8))) void k_sample_staged(
    const Node *__restrict__ nodes, const Wide *__restrict__ wide, const Cell *__restrict__ cells,
    const Dist *__restrict__ dists, const int64_t *__restrict__ sample_off, int32_t D, int64_t n_total,
    const uint64_t *__restrict__ u, int64_t S, int32_t *__restrict__ idx, double *__restrict__ x) {
    __shared__ uint4 s_cell[LCELLS * CELL_WORDS];
    const int64_t per = (S + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = xcd_block() * per;
    const int64_t r1 = r0 + per < S ? r0 + per : S;
    auto store = [&](int64_t s, const Dist &P, const Hit &h, uint64_t us) {
        if (h.i < 0) {
            idx[s] = -1;
            if (WANT_X) x[s] = __builtin_nan("");
            return;
        }
        __builtin_nontemporal_store((int32_t)(h.i - P.eo), idx + s);
        if (WANT_X) __builtin_nontemporal_store(position(P, h, us), x + s);
    };
    for (int64_t s0 = r0; s0 < r1;) {  // uniform loop over the share's segments
        const int32_t d = __builtin_amdgcn_readfirstlane(block_find_segment<SB_T>(sample_off, D, s0));
        const int64_t de = sample_off[d + 1];
        // the segment ends past s0 (offsets that break the rules still make
        // progress, one sample at a time)
        const int64_t e = de > s0 ? (de < r1 ? de : r1) : s0 + 1;
        const Dist P = dists[d];
        const bool zero = P.flags & DIST_ZERO;
        const bool staged = !zero && P.m <= LCELLS && e - s0 >= STAGE_MIN * P.m;
        if (staged) {
            const uint4 *src = reinterpret_cast<const uint4 *>(cells + P.co);
            for (int64_t k = threadIdx.x; k < CELL_WORDS * P.m; k += SB_T) s_cell[k] = src[k];
            __syncthreads();
        }
        if (staged) {
            // cells from LDS: two samples per step, both uniforms loaded
            // together (the second index clamped: no branch)
            const Cell *sc = reinterpret_cast<const Cell *>(s_cell);
            for (int64_t sa = s0 + threadIdx.x; sa < e; sa += 2 * SB_T) {
                const int64_t sb = sa + SB_T;
                const uint64_t ua = __builtin_nontemporal_load(u + sa);
                const uint64_t ub = __builtin_nontemporal_load(u + (sb < e ? sb : sa));
                Cell ca = load_cell(sc, cell_in(P, ua));
                Cell cb = load_cell(sc, cell_in(P, ub));
                pin_cell(ca);
                pin_cell(cb);
                const Hit ha = resolve(nodes, wide, ca, P, ua, n_total);
                const Hit hb = resolve(nodes, wide, cb, P, ub, n_total);
                store(sa, P, ha, ua);
                if (sb < e) store(sb, P, hb, ub);
            }
        } else {
            // cells from global memory (segments too short to stage, or
            // distributions with more than LCELLS cells)
            for (int64_t sa = s0 + threadIdx.x; sa < e; sa += SB_T) {
                const uint64_t us = __builtin_nontemporal_load(u + sa);
                Hit h;
                h.i = -1;
                if (!zero) h = descend(nodes, wide, cells, P, us, n_total);
                store(sa, P, h, us);
            }
        }
        if (staged) __syncthreads();  // before the next segment overwrites the cells
        s0 = e;
    }
}

// The 2D inversion of Sec. 5, component by component: the row from the
// marginal (distribution 0), then the column from that row's distribution.
// The marginal's guide cells are staged in LDS when it has at most LCELLS
// cells, so a pair resolves its row without a global record read.  A pair is
// read with one 16-byte load and written with one 8-byte and one 16-byte
// store, so every wave access covers whole consecutive lines.  Blocks of SB_T
// threads, two per CU, one pair per lane and step.
template <bool WANT_X>
__global__ __launch_bounds__(SB_T) __attribute__((amdgpu_waves_per_eu(8))) void k_sample_2d_staged(
    const Node *__restrict__ nodes, const Wide *__restrict__ wide, const Cell *__restrict__ cells,
    const Dist *__restrict__ dists, int32_t D, int64_t n_total, const uint64_t *__restrict__ u2, int64_t S,
    int32_t *__restrict__ rc,
    double *__restrict__ xy) {
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
    typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    __shared__ uint4 s_cell[LCELLS * CELL_WORDS];
    const u64x2 *up = reinterpret_cast<const u64x2 *>(u2);
    i32x2 *rcp = reinterpret_cast<i32x2 *>(rc);
    f64x2 *xyp = reinterpret_cast<f64x2 *>(xy);
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    const Dist M = dists[0];
    const bool mzero = (M.flags & DIST_ZERO) != 0;
    const bool staged = !mzero && M.m <= LCELLS;
    if (staged) {
        const uint4 *src = reinterpret_cast<const uint4 *>(cells + M.co);
        for (int64_t k = threadIdx.x; k < CELL_WORDS * M.m; k += SB_T) s_cell[k] = src[k];
        __syncthreads();
    }
    auto pair = [&](int64_t s, const u64x2 uu, const Cell &cr) {
        i32x2 out = {-1, -1};
        f64x2 pos = {__builtin_nan(""), __builtin_nan("")};
        Hit hr;
        hr.i = -1;
        if (!mzero) hr = resolve(nodes, wide, cr, M, uu.x, n_total);
        const int64_t r = hr.i - M.eo;
        // the marginal must have one weight per row distribution 1..D-1
        if (hr.i >= 0 && 1 + r < D) {
            out.x = (int32_t)r;
            if (WANT_X) pos.x = position(M, hr, uu.x);
            const Dist R = dists[1 + r];
            Hit hc;
            hc.i = -1;
            if (!(R.flags & DIST_ZERO)) hc = descend(nodes, wide, cells, R, uu.y, n_total);
            if (hc.i >= 0) {
                out.y = (int32_t)(hc.i - R.eo);
                if (WANT_X) pos.y = position(R, hc, uu.y);
            }
        }
        __builtin_nontemporal_store(out, rcp + s);
        if (WANT_X) __builtin_nontemporal_store(pos, xyp + s);
    };
    const int64_t s_first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (staged) {
        const Cell *sc = reinterpret_cast<const Cell *>(s_cell);
        for (int64_t s = s_first; s < S; s += T) {
            const u64x2 uu = __builtin_nontemporal_load(up + s);
            Cell cr = load_cell(sc, cell_in(M, uu.x));
            pin_cell(cr);
            pair(s, uu, cr);
        }
    } else {
        for (int64_t s = s_first; s < S; s += T) {
            const u64x2 uu = __builtin_nontemporal_load(up + s);
            Cell cr = load_cell(cells, mzero ? 0 : cell_index(M, uu.x));
            pin_cell(cr);
            pair(s, uu, cr);
        }
    }
}

// last leaf x in [lo, hi] of the distribution with key_x <= u; keys of leaves
// past the last positive weight are all-ones and never qualify
__device__ inline int64_t bisect(const Node *nodes, int64_t lo, int64_t hi, uint64_t u) {
    // invariant: key[lo] <= u (lo qualifies), hi + 1 does not
    int64_t a = lo, b = hi + 1;
    while (b - a > 1) {
        int64_t mid = a + (b - a) / 2;
        uint64_t k = nodes[mid].key;
        if (k != ~0ull && k <= u) a = mid;
        else b = mid;
    }
    return a;
}

template <bool CUTPOINT, bool WANT_X>
__global__ __launch_bounds__(256) void k_sample_bsearch(const Node *__restrict__ nodes,
                                                        const Cell *__restrict__ cells,
                                                        const Dist *__restrict__ dists,
                                                        const uint64_t *__restrict__ u,
                                                        int64_t S, int32_t *__restrict__ idx,
                                                        double *__restrict__ x) {
    const Dist &P = dists[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += stride) {
        const uint64_t us = u[s];
        if (P.flags & DIST_ZERO) {
            idx[s] = -1;
            if (WANT_X) x[s] = __builtin_nan("");
            continue;
        }
        const int64_t first = P.eo, last = P.eo + P.n - 1;
        int64_t lo = first, hi = last;
        if (CUTPOINT) {
            // the cell's first overlapping interval bounds the search from
            // below, the next cell's first overlapping interval from above
            const int64_t g = (int64_t)mulhi64(us, (uint64_t)P.m);
            const int32_t r0 = cells[P.co + g].ref;
            if (r0 < 0) {
                lo = hi = ~r0;
            } else {
                lo = (r0 > P.eo) ? r0 - 1 : r0;
                if (g + 1 < P.m) {
                    const int32_t r1 = cells[P.co + g + 1].ref;
                    hi = (r1 < 0) ? ~r1 : r1;
                }
            }
        }
        lo = lo < first ? first : (lo > last ? last : lo);
        hi = hi < lo ? lo : (hi > last ? last : hi);
        const int64_t i = (lo == hi) ? lo : bisect(nodes, lo, hi, us);
        idx[s] = (int32_t)(i - P.eo);
        if (WANT_X) x[s] = position_of(nodes, P, i, us);
    }
}

inline int grid_for(int64_t S) {
    int64_t b = (S + 255) / 256;
    const int64_t cap = 256 * 64;  // 256 CUs x 64 blocks in flight at most
    return (int)(b < cap ? b : cap);
}

}  // namespace

hipError_t launch_sample(const Node *nodes, const Wide *wide, const Cell *cells, const Dist *dists,
                         const int64_t *sample_off, int32_t D, int64_t n_total, int64_t m_total,
                         const uint64_t *u, int64_t S, int32_t *idx, double *x,
                         hipStream_t st) {
    const bool batched = sample_off != nullptr;
    // many samples per cell and small distributions: stage the cells in LDS
    // (two blocks of SB_T threads per CU)
    if (batched && S >= (int64_t)STAGE_MIN * m_total && m_total <= (int64_t)LCELLS * D) {
        int64_t nb = (S + 4 * SB_T - 1) / (4 * SB_T);
        nb = nb < 512 ? nb : 512;
        if (x)
            hipLaunchKernelGGL((k_sample_staged<true>), dim3((unsigned)nb), dim3(SB_T), 0, st, nodes, wide, cells, dists,
                               sample_off, D, n_total, u, S, idx, x);
        else
            hipLaunchKernelGGL((k_sample_staged<false>), dim3((unsigned)nb), dim3(SB_T), 0, st, nodes, wide, cells,
                               dists, sample_off, D, n_total, u, S, idx, x);
        return hipGetLastError();
    }
    const dim3 g(batched ? grid_for((S + SCHUNK / 256 - 1) / (SCHUNK / 256)) : grid_for(S)), b(256);
    if (batched && x)
        hipLaunchKernelGGL((k_sample<true, true>), g, b, 0, st, nodes, wide, cells, dists, sample_off,
                           D, n_total, u, S, idx, x);
    else if (batched)
        hipLaunchKernelGGL((k_sample<true, false>), g, b, 0, st, nodes, wide, cells, dists,
                           sample_off, D, n_total, u, S, idx, x);
    else if (x)
        hipLaunchKernelGGL((k_sample<false, true>), g, b, 0, st, nodes, wide, cells, dists,
                           sample_off, D, n_total, u, S, idx, x);
    else
        hipLaunchKernelGGL((k_sample<false, false>), g, b, 0, st, nodes, wide, cells, dists,
                           sample_off, D, n_total, u, S, idx, x);
    return hipGetLastError();
}

hipError_t launch_sample_2d(const Node *nodes, const Wide *wide, const Cell *cells, const Dist *dists,
                            int32_t D, int64_t n_total, const uint64_t *u2, int64_t S,
                            int32_t *rc, double *xy, hipStream_t st) {
    // two blocks per CU, each copying the marginal's records once
    int64_t nb = (S + SB_T - 1) / SB_T;
    nb = nb < 512 ? nb : 512;
    const dim3 g((unsigned)nb), b(SB_T);
    if (xy)
        hipLaunchKernelGGL((k_sample_2d_staged<true>), g, b, 0, st, nodes, wide, cells, dists, D, n_total, u2,
                           S, rc, xy);
    else
        hipLaunchKernelGGL((k_sample_2d_staged<false>), g, b, 0, st, nodes, wide, cells, dists, D, n_total,
                           u2, S, rc, xy);
    return hipGetLastError();
}

hipError_t launch_sample_bsearch(const Node *nodes, const Cell *cells, const Dist *dists,
                                 bool cutpoint, const uint64_t *u, int64_t S, int32_t *idx,
                                 double *x, hipStream_t st) {
    const dim3 g(grid_for(S)), b(256);
    if (cutpoint && x)
        hipLaunchKernelGGL((k_sample_bsearch<true, true>), g, b, 0, st, nodes, cells, dists, u,
                           S, idx, x);
    else if (cutpoint)
        hipLaunchKernelGGL((k_sample_bsearch<true, false>), g, b, 0, st, nodes, cells, dists, u,
                           S, idx, x);
    else if (x)
        hipLaunchKernelGGL((k_sample_bsearch<false, true>), g, b, 0, st, nodes, cells, dists, u,
                           S, idx, x);
    else
        hipLaunchKernelGGL((k_sample_bsearch<false, false>), g, b, 0, st, nodes, cells, dists,
                           u, S, idx, x);
    return hipGetLastError();
}

}  // namespace rtf
