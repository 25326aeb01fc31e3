// rtf_build.hip -- parallel construction of the guide table and radix tree
// forest (Binder & Keller, Sec. 3.1-3.2, Alg. 1; many distributions: Sec. 5).
//
// The forest is the unique tree Alg. 1 builds from the per-boundary levels
// (position of the highest differing bit of neighbouring fixed-point lower
// bounds, or SENT where merges may not cross): within a cell, the root of a
// leaf range is its boundary of highest level (the rightmost one on a tie),
// which is what Alg. 1's bottom-up merges produce under every schedule.  Alg.
// 1 finds it with an atomic exchange per merge; here each node instead finds
// the two boundaries of higher level that enclose it (its subtree) by a short
// scan over the levels held in LDS, and writes its own 16-byte record once.
// With m proportional to n the cells hold a few leaves, so the scans are a few
// LDS reads; scans that leave a tile's LDS window or exceed SCAN_CAP steps are
// finished by a fix-up kernel that searches the global keys.
//
// Kernels (stream order):
//   k_tile_sums    per-tile weight sums (+ in-tile prefix at distribution
//                  starts); block 0 copies the offsets into the workspace and
//                  clears the status word and the run list
//   k_dist_params  scan of tile sums; per distribution W, reciprocal, G0
//   k_dist_finish  the latter for more than PT distributions
//   k_build_tile   keys, levels, node records, guide-table entries per tile
//   k_fixup        deferred node records and long guide-table runs
#include "rtf_internal.h"

namespace rtf {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// Lane i receives lane i - k's value under the DPP row control CTRL (0 where
// the source lies outside the row or the row is masked off), for both halves.
template <int CTRL, int ROW_MASK>
__device__ inline uint64_t dpp_move(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)x, CTRL, ROW_MASK, 0xf, false);
    const uint32_t hi =
        __builtin_amdgcn_update_dpp(0u, (uint32_t)(x >> 32), CTRL, ROW_MASK, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan over the 64 lanes with DPP moves (no LDS round trips):
// row_shr 1, 2, 4, 8 scan each row of 16 lanes, then row_bcast 15 adds row 0's
// total to row 1 (and row 2's to row 3) and row_bcast 31 adds lanes 0..31's
// total to rows 2 and 3.
__device__ inline uint64_t wave_incl_scan(uint64_t x) {
    x += dpp_move<0x111, 0xf>(x);  // row_shr:1
    x += dpp_move<0x112, 0xf>(x);  // row_shr:2
    x += dpp_move<0x114, 0xf>(x);  // row_shr:4
    x += dpp_move<0x118, 0xf>(x);  // row_shr:8
    x += dpp_move<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_move<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// Inclusive suffix sum over the 64 lanes: the wave total (lane 63's prefix)
// minus the prefix before the lane.
__device__ inline uint64_t wave_incl_suffix(uint64_t x) {
    const uint64_t incl = wave_incl_scan(x);
    const uint64_t total = __shfl(incl, 63, 64);
    return total - incl + x;
}

// Exclusive scan over the block (NW waves); returns the thread's exclusive
// prefix and the block total.
template <int NW>
__device__ inline uint64_t block_excl_scan(uint64_t x, uint64_t *s_wave, uint64_t &total) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint64_t inc = wave_incl_scan(x);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        uint64_t v = s_wave[i];
        off += (i < w) ? v : 0;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

// index d in [lo, hi) with off[d] <= i < off[d+1], given off[lo] <= i < off[hi]
__device__ inline int32_t find_segment_in(const int64_t *off, int32_t lo, int32_t hi, int64_t i) {
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// first d in [0, D] with off[d] > i (off[0..D] non-decreasing)
__device__ inline int32_t upper_bound(const int64_t *off, int32_t D, int64_t i) {
    int32_t lo = 0, hi = D + 1;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first d in [0, D] with off[d] >= i
__device__ inline int32_t lower_bound(const int64_t *off, int32_t D, int64_t i) {
    int32_t lo = 0, hi = D + 1;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (off[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Load the ITEMS weights starting at i0.  FULL: every one is in range and w
// is 16-byte aligned, so the loads are unconditional vector loads.  Else each
// load reads a clamped, in-range index and the value is masked; neither form
// branches, so the compiler need not wait for a load at a branch join and
// several loads stay in flight.
template <int ITEMS, bool FULL>
__device__ inline void load_items(const uint32_t *w, int64_t i0, int64_t n, uint32_t *r) {
    static_assert(ITEMS == 2 || ITEMS % 4 == 0, "vector loads of 8 or 16 bytes");
    if constexpr (FULL) {
        if constexpr (ITEMS == 2) {
            const uint2 v = *reinterpret_cast<const uint2 *>(w + i0);
            r[0] = v.x;
            r[1] = v.y;
        } else {
            const uint4 *p = reinterpret_cast<const uint4 *>(w + i0);
#pragma unroll
            for (int q = 0; q < ITEMS / 4; ++q) {
                uint4 v = p[q];
                r[4 * q + 0] = v.x;
                r[4 * q + 1] = v.y;
                r[4 * q + 2] = v.z;
                r[4 * q + 3] = v.w;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < ITEMS; ++e) {
            const int64_t i = i0 + e;
            const uint32_t v = w[i < n ? (i >= 0 ? i : 0) : n - 1];
            r[e] = (i >= 0 && i < n) ? v : 0u;
        }
    }
}

// Leaf description used for levels: key and global cell; cell -1 marks a leaf
// past its distribution's last positive weight, -2 a position outside [0, n).
struct Leaf {
    uint64_t key;
    int32_t cell;
};

__device__ inline int level_between(const Leaf &a, const Leaf &b) {
    if (a.cell < 0 || b.cell < 0 || a.cell != b.cell) return SENT;
    return level_of(a.key, b.key);
}

// cell of a key: floor(key * m / 2^64), a shift when m is a power of two
__device__ inline int32_t cell_of_key(uint64_t key, const Dist &P) {
    const uint32_t sh = P.flags >> DIST_SHIFT_BIT;
    const uint64_t c = sh ? (key >> sh) : mulhi64(key, (uint64_t)P.m);
    return (int32_t)(P.co + (int64_t)c);
}

__device__ inline Leaf make_leaf(uint64_t C, const Dist &P) {
    Leaf L;
    if (C < P.W) {
        L.key = fixed_point_key(C, P.W << P.s, P.v, P.s);
        L.cell = cell_of_key(L.key, P);
    } else {
        L.key = ~0ull;
        L.cell = -1;
    }
    return L;
}

// A cell record with CELL_WORDS 16-byte stores.
__device__ inline void store_cell(Cell *cells, int64_t g, const uint64_t *k, int32_t ref,
                                  int32_t aux) {
    uint4 *p = reinterpret_cast<uint4 *>(cells + g);
#pragma unroll
    for (int w = 0; w + 1 < CELL_WORDS; ++w)
        p[w] = make_uint4((uint32_t)k[2 * w], (uint32_t)(k[2 * w] >> 32), (uint32_t)k[2 * w + 1],
                          (uint32_t)(k[2 * w + 1] >> 32));
    p[CELL_WORDS - 1] = make_uint4((uint32_t)k[CELL_KEYS - 1], (uint32_t)(k[CELL_KEYS - 1] >> 32), (uint32_t)ref,
                                   (uint32_t)aux);
}

// The record of a cell covered by interval i alone, whose keys are lo and hi.
__device__ inline void store_covered(Cell *cells, int64_t g, uint64_t lo, uint64_t hi, int32_t i) {
    uint64_t k[CELL_KEYS];
#pragma unroll
    for (int t = 0; t < CELL_KEYS; ++t) k[t] = t == 0 ? lo : (t == 1 ? hi : 0);
    store_cell(cells, g, k, ~i, ~i);
}

// The record of the cell whose first node is a, given the key and cell of a
// and of leaves a+1 .. a+CELL_BOUNDS (cell < 0: no mass, or outside [0, n)),
// the key of leaf a-1 and the cell tree's root c1 (used when the cell holds
// more than CELL_BOUNDS lower bounds).
__device__ inline void root_record(Cell *cells, int64_t g, int32_t a, uint64_t kprev,
                                   const uint64_t *key, const int32_t *cell, int32_t c1) {
    uint64_t k[CELL_KEYS];
    k[0] = key[0] == 0 ? 0 : kprev;  // 0 at a distribution start
    k[1] = key[0];
    int cnt = 1;  // lower bounds of the cell among a .. a+t-1
    bool open = true;
#pragma unroll
    for (int t = 1; t <= CELL_BOUNDS; ++t) {
        uint64_t v = 0;
        if (open && cell[t] == cell[0]) {
            v = key[t];
            ++cnt;
        } else if (open) {
            // leaf a+t starts the next cell: the upper end of the cell's last
            // interval, or the distribution's end
            const bool same_dist = cell[t] >= 0 && key[t] != 0;
            v = same_dist ? key[t] : KEY_END;
            open = false;
        }
        k[t + 1] = v;
    }
    store_cell(cells, g, k, a, open ? c1 : ~cnt);
}

// List the guide-table run [lo, hi), covered by interval i with keys k0 and
// k1, for the fix-up kernel.  One 64-bit atomic takes both the list slot and
// the run's offset in the sequence of listed cells, so offsets grow with the
// slot.
__device__ inline void push_run(const BuildArgs &a, int64_t lo, int64_t hi, int32_t i, uint64_t k0,
                                uint64_t k1) {
    const uint64_t len = (uint64_t)(hi - lo);
    const uint64_t old = atomicAdd((unsigned long long *)a.run_count, (1ull << 32) | len);
    const int64_t slot = (int64_t)(old >> 32);
    if (slot >= run_cap(a.m_total)) {  // impossible by the bound of run_cap
        atomicOr(a.status, status_bit(RTF_ERR_WORKSPACE));
        return;
    }
    Run r;
    r.k0 = k0;
    r.k1 = k1;
    r.lo = (int32_t)lo;
    r.len = (int32_t)len;
    r.i = i;
    r.off = (uint32_t)old;
    a.runs[slot] = r;
}

// A node record, stored non-temporally: the tile kernel's waves write 1 KiB
// of consecutive records per store, and the sampler reads nodes back only for
// the few samples whose cell record does not settle them (H24 build 183 ->
// 171 us, C3 294 -> 278 us, C4 1203 -> 1192 us, build + sample 1612 -> 1603
// us; the cell records, stored at a 64-byte stride per lane, took 2.3 times
// as long that way and stay ordinary stores).
__device__ inline void store_node(Node *nodes, int64_t j, uint64_t key, int32_t c0, int32_t c1) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = {(uint32_t)key, (uint32_t)(key >> 32), (uint32_t)c0, (uint32_t)c1};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(nodes + j));
}

// ---------------------------------------------------------------------------
// k_tile_sums: the prefix-sum pass over the weights (Sec. 2.6 notes that the
// prefix sum of an inversion method computes efficiently in parallel)
// ---------------------------------------------------------------------------
// Each block sums TS_TILES (one distribution: TS_SINGLE) tiles whose loads are
// all issued before the first reduction, so that enough bytes are in flight
// to stream at HBM rate.

// A distribution index from a search over the caller's offsets, kept in
// [0, D) also for offsets that break the rules.
__device__ inline int32_t clamp_dist(int32_t d, int32_t D) { return d < 0 ? 0 : (d < D ? d : D - 1); }

__device__ inline uint64_t wave_sum(uint64_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <class T, bool BATCHED, bool FULL>
__device__ inline void tile_sums_body(const BuildArgs &a, int64_t t0, uint64_t *s_wave,
                                      uint64_t *s_thr, int32_t *s_first) {
    constexpr int BT = T::BT, ITEMS = T::ITEMS, TILE = T::TILE;
    constexpr int TS_TILES = BATCHED ? T::TS_TILES : T::TS_SINGLE;
    constexpr int NW = BT / 64;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    uint32_t r[TS_TILES][ITEMS];
#pragma unroll
    for (int k = 0; k < TS_TILES; ++k)
        load_items<ITEMS, FULL>(a.w, (t0 + k) * TILE + (int64_t)tid * ITEMS, a.n_total, r[k]);
    uint64_t sum[TS_TILES];
#pragma unroll
    for (int k = 0; k < TS_TILES; ++k) {
        sum[k] = 0;
#pragma unroll
        for (int e = 0; e < ITEMS; ++e) sum[k] += r[k][e];
    }
    if (!BATCHED) {
        // one distribution: only the tile totals are needed
#pragma unroll
        for (int k = 0; k < TS_TILES; ++k) {
            const uint64_t ws = wave_sum(sum[k]);
            if (lane == 0) s_wave[k * NW + w] = ws;
        }
        __syncthreads();
        if (tid < TS_TILES && t0 + tid < a.ntiles) {
            uint64_t tot = 0;
#pragma unroll
            for (int i = 0; i < NW; ++i) tot += s_wave[tid * NW + i];
            a.tile_sum[t0 + tid] = tot;
        }
        return;
    }
    // per tile, two searches over the caller's offsets, one whole wave each
    // and all eight at once (64 probes per step: three steps for 10^4
    // distributions): the first distribution starting at or after the tile's
    // first element (waves 0..TS_TILES-1), and the distribution holding that
    // element (waves TS_TILES..2 TS_TILES-1, into tile_dist); the block of the
    // last tile also fills tile_dist[ntiles] and tile_dist[ntiles + 1]
    static_assert(!BATCHED || 2 * TS_TILES == BT / 64, "one wave per search");
    {
        const int k = w % TS_TILES;
        const int64_t t = t0 + k;
        if (t < a.ntiles) {
            if (w < TS_TILES) {
                const int32_t d = wave_upper_bound(a.src_elem_off, a.D, t * TILE - 1);  // first off >= t*TILE
                if (lane == 0) s_first[k] = d;
            } else {
                const int32_t d = clamp_dist(wave_upper_bound(a.src_elem_off, a.D, t * TILE) - 1, a.D);
                if (lane == 0) a.tile_dist[t] = d;
            }
        }
        if (w == 0 && t0 + TS_TILES >= a.ntiles) {
            const int32_t d = clamp_dist(wave_upper_bound(a.src_elem_off, a.D, a.n_total - 1) - 1, a.D);
            if (lane == 0) {
                a.tile_dist[a.ntiles] = d;
                a.tile_dist[a.ntiles + 1] = d;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < TS_TILES; ++k) {
        const int64_t t = t0 + k;
        if (t >= a.ntiles) break;  // uniform across the block
        uint64_t total;
        const uint64_t ex = block_excl_scan<NW>(sum[k], s_wave, total);  // has barriers
        if (tid == 0) a.tile_sum[t] = total;
        s_thr[tid] = ex;
        __syncthreads();
        // distributions that start inside this tile: record the in-tile prefix
        const int64_t base = t * TILE, end = base + TILE;
        const int32_t dlo = s_first[k];
        for (int32_t d = dlo + tid; d < a.D; d += BT) {
            int64_t e = a.src_elem_off[d];
            if (e >= end) break;
            if (e < base || e >= a.n_total) continue;  // only offsets that break the rules
            int64_t off = e - base;
            int64_t tq = off / ITEMS;
            uint64_t L = s_thr[tq];
            for (int64_t q = base + tq * ITEMS; q < e; ++q) L += a.w[q];
            a.dist_local[d] = L;
        }
        __syncthreads();  // s_thr and s_wave are reused by the next tile
    }
}

template <class T, bool BATCHED>
__global__ __launch_bounds__(T::BT) void k_tile_sums(BuildArgs a, bool vec) {
    constexpr int BT = T::BT, TILE = T::TILE;
    constexpr int TS_TILES = BATCHED ? T::TS_TILES : T::TS_SINGLE;
    __shared__ uint64_t s_wave[TS_TILES * (BT / 64)];
    __shared__ uint64_t s_thr[BT];
    __shared__ int32_t s_first[TS_TILES];
    const int tid = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * TS_TILES;
    if (blockIdx.x == 0) {
        // this build's status word, run list and the offsets later kernels
        // read.  The caller's offsets are checked first: offsets that break
        // the rules (0 first, strictly increasing, n_total and m_total last)
        // are reported as RTF_ERR_INVALID_ARG and replaced in the workspace by
        // a valid partition (one weight and one cell for each distribution
        // but the last), so that every later kernel stays in bounds.
        bool bad = false;
        if (BATCHED) {
            for (int64_t q = tid; q <= a.D; q += BT) {
                const int64_t e = a.src_elem_off[q], c = a.src_cell_off[q];
                if (q == 0) bad = bad || e != 0 || c != 0;
                else bad = bad || e <= a.src_elem_off[q - 1] || c <= a.src_cell_off[q - 1];
                if (q == a.D) bad = bad || e != a.n_total || c != a.m_total;
            }
        }
        bad = __syncthreads_or(bad);
        if (tid == 0) {
            *a.status = bad ? status_bit(RTF_ERR_INVALID_ARG) : 0u;
            *a.run_count = 0;
            *a.item_count = 0u;
        }
        for (int64_t q = tid; q <= a.D; q += BT) {
            const bool own = BATCHED && !bad;
            a.elem_off[q] = own ? a.src_elem_off[q] : (q == a.D ? a.n_total : (BATCHED ? q : 0));
            a.cell_off[q] = own ? a.src_cell_off[q] : (q == a.D ? a.m_total : (BATCHED ? q : 0));
        }
    }
    if (vec && (t0 + TS_TILES) * TILE <= a.n_total)
        tile_sums_body<T, BATCHED, true>(a, t0, s_wave, s_thr, s_first);
    else tile_sums_body<T, BATCHED, false>(a, t0, s_wave, s_thr, s_first);
}

// ---------------------------------------------------------------------------
// k_dist_params: one block.  Exclusive scan of the tile sums, then per
// distribution the total W, the divisor normalisation and reciprocal, and the
// global prefix at its first element; more than PT distributions are left to
// k_dist_finish, one thread each over many blocks.
// ---------------------------------------------------------------------------
constexpr int PT = 1024;

// Distribution d's parameters: the total W, the divisor normalisation and
// reciprocal, and the global prefix at its first element.
template <class T, bool BATCHED>
__device__ inline void dist_params_of(const BuildArgs &a, int32_t d, uint64_t total) {
    constexpr int TILE = T::TILE;
    // one distribution: the whole forest, known without a read
    const int64_t eo = BATCHED ? a.elem_off[d] : 0, e1 = BATCHED ? a.elem_off[d + 1] : a.n_total;
    uint64_t G0 = 0, G1 = total;
    if (BATCHED) {
        G0 = a.tile_prefix[eo / TILE] + a.dist_local[d];
        if (d + 1 < a.D) G1 = a.tile_prefix[e1 / TILE] + a.dist_local[d + 1];
    }
    Dist P;
    P.W = G1 - G0;
    P.G0 = G0;
    P.eo = eo;
    P.n = e1 - eo;
    P.co = BATCHED ? a.cell_off[d] : 0;
    P.m = BATCHED ? a.cell_off[d + 1] - P.co : a.m_total;
    P.flags = 0;
    if (P.W == 0) {
        P.s = 0;
        P.v = 0;
        P.flags = DIST_ZERO;
        atomicOr(a.status, status_bit(RTF_ERR_ZERO_TOTAL));
    } else {
        P.s = (uint32_t)clz64(P.W);
        P.v = reciprocal_2by1(P.W << P.s);
    }
    if (P.m > 1 && (P.m & (P.m - 1)) == 0)
        P.flags |= (uint32_t)(64 - __builtin_ctzll((uint64_t)P.m)) << DIST_SHIFT_BIT;
    a.dists[d] = P;
}

template <class T, bool BATCHED>
__global__ __launch_bounds__(PT) void k_dist_params(BuildArgs a) {
    __shared__ uint64_t s_wave[PT / 64];
    const int64_t nt = a.ntiles;
    // rounds of PT x 8 tile sums; thread t scans 8 consecutive ones
    constexpr int CH = 8;
    uint64_t carry = 0;
    for (int64_t r0 = 0; r0 < nt; r0 += (int64_t)PT * CH) {
        const int64_t lo = r0 + (int64_t)threadIdx.x * CH;
        uint64_t v[CH];
        if (lo + CH <= nt) {
            const uint4 *p = reinterpret_cast<const uint4 *>(a.tile_sum + lo);
#pragma unroll
            for (int q = 0; q < CH / 2; ++q) {
                const uint4 x = p[q];
                v[2 * q] = ((uint64_t)x.y << 32) | x.x;
                v[2 * q + 1] = ((uint64_t)x.w << 32) | x.z;
            }
        } else {
#pragma unroll
            for (int q = 0; q < CH; ++q) v[q] = (lo + q < nt) ? a.tile_sum[lo + q] : 0;
        }
        uint64_t sum = 0;
#pragma unroll
        for (int q = 0; q < CH; ++q) sum += v[q];
        uint64_t round_total;
        uint64_t run = carry + block_excl_scan<PT / 64>(sum, s_wave, round_total);
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            if (lo + q < nt) a.tile_prefix[lo + q] = run;
            run += v[q];
        }
        carry += round_total;
    }
    const uint64_t total = carry;
    if (a.D > PT) {  // k_dist_finish takes the distributions, one thread each
        if (threadIdx.x == 0) a.tile_prefix[nt] = total;
        return;
    }
    if (BATCHED) {  // the parameters read back this block's tile prefixes
        __threadfence_block();
        __syncthreads();
    }
    if ((int32_t)threadIdx.x < a.D) dist_params_of<T, BATCHED>(a, (int32_t)threadIdx.x, total);
}

template <class T, bool BATCHED>
__global__ __launch_bounds__(256) void k_dist_finish(BuildArgs a) {
    const int32_t d = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (d < a.D) dist_params_of<T, BATCHED>(a, d, a.tile_prefix[a.ntiles]);
}

// ---------------------------------------------------------------------------
// k_build_tile
//
// Phase 1 (thread t owns ITEMS consecutive leaves): prefix sums, keys and
// cells into LDS, plus HALO leaves on either side of the tile.  Phase 2: the
// levels of all boundaries held.  Phase 3: parent links.  Alg. 1 merges a
// subtree across whichever of its two outside boundaries has the lower level
// (the left one on a tie); so the subtree rooted at boundary b, which spans
// the leaves between L = the nearest boundary left of b with a higher level
// and R = the nearest boundary right of b with a level at least as high, is
// child 0 of node R+1 when lvl(L) > lvl(R) and child 1 of node L+1
// otherwise; a leaf is the same with L, R its two adjacent boundaries.  Every
// boundary and leaf of the window writes itself into its parent's child slot
// in LDS; the nearest-higher searches read eight levels per LDS access.
// Phase 4: node records, 64 consecutive 16-byte records per wave store, and
// the guide cells into an LDS window.  Phase 5: the guide cell records, 64
// consecutive 32-byte records per wave.  A node with an empty child slot (its
// child lies outside the window) is finished by the fix-up kernel.  Indices
// inside the tile are 32-bit: local leaf li is global leaf lb0 + li, local
// boundary bi lies between local leaves bi and bi + 1 (it is node bi + 1).
// ---------------------------------------------------------------------------
static_assert(2 * HALO == 64, "wave 0 loads both halos, one leaf per lane");
// Child slots hold local node indices (16 bits) and window entries 16-bit
// owner codes, so that the tile's LDS (about 38 KB) lets four blocks share a
// CU.
// An empty child slot holds -1 in LDS and reads as SLOT_EMPTY, never a node
// or leaf reference.
constexpr int32_t SLOT_EMPTY = INT32_MIN;

// Owner codes of the guide cells staged in the window: which local leaf a
// cell record comes from (low 14 bits) and how (top 2 bits).
constexpr uint16_t WIN_EMPTY = 0xFFFF;
constexpr uint16_t WIN_ROOT = 0 << 14;  // the cell's first node
constexpr uint16_t WIN_HEAD = 1 << 14;  // covered by the leaf before that node
constexpr uint16_t WIN_TAIL = 2 << 14;  // covered by a distribution's last leaf
constexpr uint16_t WIN_KIND = 0xC000, WIN_LEAF = 0x3FFF;
template <class T>
struct alignas(16) TileSmem {
    static constexpr int LEAF_N = T::TILE + 2 * HALO;
    static constexpr int LVL_N = LEAF_N - 1;  // real boundaries; lvl[LVL_N] is padding
    static_assert(LEAF_N % 8 == 0, "levels are read 8 at a time");
    static_assert(T::WIN % 8 == 0 && (2 * T::TILE) % 8 == 0, "16-byte clears of slot and window");
    static_assert(LEAF_N <= WIN_LEAF, "local leaf indices fit an owner code");
    static_assert(2 * T::TILE <= 32767, "local node indices fit a 16-bit slot");
    uint64_t key[LEAF_N];
    int32_t cell[LEAF_N];
    int16_t slot[2 * T::TILE];  // child slots of the tile's own nodes (local node index)
    uint16_t win[T::WIN];       // owner codes of cells c_begin .. c_begin + WIN - 1
    uint64_t lvl8[LEAF_N / 8];
    uint64_t wave[T::BT / 64];
    int64_t c_begin;
    int32_t win_hi;  // highest window position phase 4 wrote
    int32_t ndefer;
    int32_t item_base;  // this tile's place in the grid-wide deferral list
    int32_t items[T::DEFER_CAP];
};

template <class T>
__device__ inline void push_item(TileSmem<T> &sm, int32_t item) {
    int32_t k = atomicAdd(&sm.ndefer, 1);
    if (k < T::DEFER_CAP) sm.items[k] = item;
}

// the level of local boundary bi: byte bi of the level array (one LDS byte
// read, no shift)
template <class T>
__device__ inline int lvl_at(const TileSmem<T> &sm, int bi) {
    return reinterpret_cast<const uint8_t *>(sm.lvl8)[bi];
}

// bit 7 of every byte of w (eight levels, each < 128) that is >= t, for
// 0 <= t <= 128: a byte plus 128 - t reaches 128 exactly when it is >= t and
// never carries into the next byte, so each 32-bit half is done on its own
__device__ inline uint64_t ge_mask(uint64_t w, int t) {
    const uint32_t rep = __builtin_amdgcn_perm(0u, (uint32_t)(128 - t), 0u);  // byte 0 x4
    const uint32_t lo = ((uint32_t)w + rep) & 0x80808080u;
    const uint32_t hi = ((uint32_t)(w >> 32) + rep) & 0x80808080u;
    return ((uint64_t)hi << 32) | lo;
}

constexpr int SCAN_WORDS = SCAN_CAP / 8;

// nearest boundary at or left of bi with a level >= t, or -1
template <class T>
__device__ inline int nearest_ge_left(const TileSmem<T> &sm, int bi, int t) {
    if (bi < 0) return -1;
    int wi = bi >> 3;
    const int pos = bi & 7;
    uint64_t m = ge_mask(sm.lvl8[wi], t);
    if (pos < 7) m &= (1ull << (8 * pos + 8)) - 1;
    for (int steps = 0; m == 0; ++steps) {
        if (--wi < 0 || steps >= SCAN_WORDS) return -1;
        m = ge_mask(sm.lvl8[wi], t);
    }
    return wi * 8 + (63 - clz64(m)) / 8;
}

// nearest boundary at or right of bi with a level >= t, or -1
template <class T>
__device__ inline int nearest_ge_right(const TileSmem<T> &sm, int bi, int t) {
    constexpr int LEAF_N = TileSmem<T>::LEAF_N, LVL_N = TileSmem<T>::LVL_N;
    if (bi >= LVL_N) return -1;
    int wi = bi >> 3;
    uint64_t m = ge_mask(sm.lvl8[wi], t) & (~0ull << (8 * (bi & 7)));
    for (int steps = 0; m == 0; ++steps) {
        if (++wi >= LEAF_N / 8 || steps >= SCAN_WORDS) return -1;
        m = ge_mask(sm.lvl8[wi], t);
    }
    const int r = wi * 8 + __builtin_ctzll(m) / 8;
    return r < LVL_N ? r : -1;
}

// write local node `child` into child slot `side` of local node pn if the
// tile owns it
template <class T>
__device__ inline void link(TileSmem<T> &sm, int pn, int side, int child) {
    const int s = pn - HALO;
    if (s >= 0 && s < T::TILE) sm.slot[2 * s + side] = (int16_t)child;
}

// child slot k as a global reference (SLOT_EMPTY when nothing was linked)
template <class T>
__device__ inline int32_t slot_ref(const TileSmem<T> &sm, int k, int32_t lb0) {
    const int16_t v = sm.slot[k];
    return v < 0 ? SLOT_EMPTY : lb0 + v;
}

// stage the record of cell c (owner code w) in the window, or store it
// directly when the cell lies past the window
// (returns the window position written, or -1)
template <class T>
__device__ inline int put_cell(TileSmem<T> &sm, Cell *cells, int64_t c, uint16_t w, int32_t lb0) {
    const int64_t x = c - sm.c_begin;
    if (x >= 0 && x < T::WIN) {
        sm.win[x] = w;
        return (int)x;
    }
    const int li = w & WIN_LEAF;
    const int32_t g = lb0 + li;
    if ((w & WIN_KIND) == WIN_HEAD) store_covered(cells, c, sm.key[li - 1], sm.key[li], g - 1);
    else store_covered(cells, c, sm.key[li], KEY_END, g);  // WIN_TAIL
    return -1;
}

template <class T>
__device__ inline void root_cell_record(const TileSmem<T> &sm, Cell *cells, int64_t c, int li,
                                        int32_t lb0) {
    uint64_t key[CELL_BOUNDS + 1];
    int32_t cell[CELL_BOUNDS + 1];
#pragma unroll
    for (int t = 0; t <= CELL_BOUNDS; ++t) {
        key[t] = sm.key[li + t];
        cell[t] = sm.cell[li + t];
    }
    // child 1 of a cell's first node: the cell tree's root (read only when
    // the cell holds more than CELL_BOUNDS leaves, so it is an internal node)
    root_record(cells, c, lb0 + li, sm.key[li - 1], key, cell, slot_ref(sm, 2 * (li - HALO) + 1, lb0));
}

// Phase 1 of k_build_tile (thread t owns ITEMS consecutive leaves): prefix
// sums, keys and cells into LDS, plus HALO leaves on either side of the tile.
// Every global load of the phase (weights, halo weights, tile prefix,
// distribution parameters) is issued before the block scan and none sits
// under a branch, so a block waits for one round trip.  FULL: the tile lies
// inside [0, n) and the weights are 16-byte aligned.
template <class T, bool BATCHED, bool FULL, bool UNI>
__device__ inline void build_keys(const BuildArgs &a, TileSmem<T> &sm, int64_t t) {
    constexpr int BT = T::BT, ITEMS = T::ITEMS, TILE = T::TILE;
    const int tid = threadIdx.x;
    const int64_t base = t * TILE;
    const int64_t n = a.n_total;
    // halo leaves: lanes 0..HALO-1 of wave 0 the HALO leaves left of the
    // tile, lanes HALO..63 the HALO leaves right of it; every lane loads a
    // clamped index so that the load needs no branch
    const bool left = tid < HALO;
    const int64_t hi_ = base - HALO + tid + (left ? 0 : TILE);
    const bool hexists = tid < 64 && hi_ >= 0 && hi_ < n;
    const uint32_t hraw = a.w[hi_ < 0 ? 0 : (hi_ < n ? hi_ : n - 1)];
    __builtin_amdgcn_sched_barrier(0);  // issue the halo load first
    const int64_t i0 = base + (int64_t)tid * ITEMS;
    const int li0 = HALO + tid * ITEMS;
    uint32_t wv[ITEMS];
    load_items<T::ITEMS, FULL>(a.w, i0, n, wv);
    const uint64_t tp = a.tile_prefix[t];
    // the distributions of the tile's elements lie in [d_lo, d_hi]; UNI: in
    // one distribution, whose parameters are then uniform (scalar registers)
    int32_t dcur = 0, d_lo = 0, d_hi = 0;
    if (BATCHED) {
        d_lo = a.tile_dist[t];
        d_hi = a.tile_dist[t + 1];
        dcur = UNI ? d_lo : find_segment_in(a.elem_off, d_lo, d_hi + 1, i0 < n ? i0 : n - 1);
    }
    Dist P = a.dists[dcur];
    const uint64_t hw = hexists ? hraw : 0u;
    Dist HP = P;
    if (BATCHED && tid < 64 && hexists) {
        // left halo: between the previous tile's first distribution and d_lo;
        // right halo: between d_hi and the next tile's last
        const int32_t lo = left ? a.tile_dist[t > 0 ? t - 1 : 0] : d_hi;
        const int32_t hi = left ? d_lo : a.tile_dist[t + 2];
        HP = a.dists[find_segment_in(a.elem_off, lo, hi + 1, hi_)];
    }

    uint64_t sum = 0;
#pragma unroll
    for (int e = 0; e < ITEMS; ++e) sum += wv[e];
    uint64_t tile_total;
    uint64_t G = tp + block_excl_scan<BT / 64>(sum, sm.wave, tile_total);
    int64_t dend = P.eo + P.n;
    const int live = FULL ? ITEMS : (int)(n - i0 < ITEMS ? (n - i0 > 0 ? n - i0 : 0) : ITEMS);
#pragma unroll
    for (int e = 0; e < ITEMS; ++e) {
        Leaf L;
        L.key = 0;
        L.cell = -2;
        if (e < live) {
            if (BATCHED && !UNI) {
                while (i0 + e >= dend) {
                    ++dcur;
                    P = a.dists[dcur];
                    dend = P.eo + P.n;
                }
            }
            L = make_leaf(G - P.G0, P);
        }
        sm.key[li0 + e] = L.key;
        sm.cell[li0 + e] = L.cell;
        G += wv[e];
    }
    if (tid < 64) {
        const uint64_t suf = wave_incl_suffix(left ? hw : 0);
        const uint64_t pre = wave_incl_scan(left ? 0 : hw);
        Leaf L;
        L.key = 0;
        L.cell = -2;
        if (hexists) {
            const uint64_t Gi = left ? tp - suf : tp + tile_total + pre - hw;
            L = make_leaf(Gi - HP.G0, HP);
        }
        const int slot = left ? tid : TILE + tid;
        sm.key[slot] = L.key;
        sm.cell[slot] = L.cell;
    }
}

// With 2048-element tiles the LDS allows four blocks per CU.  The
// single-distribution instance fits 64 registers and runs four (eight waves
// per SIMD); the batched instance, which needs more, is held to 80 registers
// for three blocks, at the price of a few spilled ones.  With 1024-element
// tiles of 256 threads the LDS allows seven blocks, and the batched instance
// fits its 80 registers without spills.
template <class T, bool BATCHED>
__global__ __launch_bounds__(T::BT) __attribute__((amdgpu_waves_per_eu(BATCHED ? T::WAVES_BATCHED : T::WAVES_ONE))) void k_build_tile(BuildArgs a, bool vec) {
    constexpr int BT = T::BT, TILE = T::TILE, WIN = T::WIN, DEFER_CAP = T::DEFER_CAP;
    constexpr int LEAF_N = TileSmem<T>::LEAF_N, LVL_N = TileSmem<T>::LVL_N;
    __shared__ TileSmem<T> sm;
    const int tid = threadIdx.x;
    const int64_t t = blockIdx.x;
    const int64_t base = t * TILE;
    const int64_t n = a.n_total;
    const int32_t lb0 = (int32_t)(base - HALO);  // global index of local leaf 0
    // distributions of the tile's own elements: [d_lo, d_hi]
    const int32_t d_lo = BATCHED ? a.tile_dist[t] : 0, d_hi = BATCHED ? a.tile_dist[t + 1] : 0;
    if (tid == 0) sm.ndefer = 0;

    // ---- phase 1: keys and cells of the tile's leaves -----------------------
    // a tile inside one distribution (the common case) takes the phase with
    // uniform parameters
    const bool full = vec && base + TILE <= n;
    if (!BATCHED || d_lo == d_hi) {
        if (full) build_keys<T, BATCHED, true, true>(a, sm, t);
        else build_keys<T, BATCHED, false, true>(a, sm, t);
    } else {
        if (full) build_keys<T, BATCHED, true, false>(a, sm, t);
        else build_keys<T, BATCHED, false, false>(a, sm, t);
    }
    __syncthreads();

    // ---- phase 2: levels of all boundaries held; empty slots and window ----
    {
        // one level per thread and byte (consecutive lanes, no bank conflicts);
        // byte bi of the array is byte bi & 7 of word bi >> 3
        uint8_t *lv = reinterpret_cast<uint8_t *>(sm.lvl8);
        for (int bi = tid; bi < LEAF_N; bi += BT) {
            int l = SENT;  // the padding byte past the last boundary
            if (bi < LVL_N)
                l = level_between(Leaf{sm.key[bi], sm.cell[bi]}, Leaf{sm.key[bi + 1], sm.cell[bi + 1]});
            lv[bi] = (uint8_t)l;
        }
    }
    {
        // 16-bit entries, eight per 16-byte store; both empty codes are all ones
        const int4 ones = make_int4(-1, -1, -1, -1);
        for (int x = tid; x < 2 * TILE / 8; x += BT) reinterpret_cast<int4 *>(sm.slot)[x] = ones;
        for (int x = tid; x < WIN / 8; x += BT) reinterpret_cast<int4 *>(sm.win)[x] = ones;
    }
    if (tid == 0) {
        // first guide cell whose record comes from a leaf of this tile
        const int32_t c = sm.cell[HALO], cp = sm.cell[HALO - 1];
        int64_t cb;
        if (c >= 0) {
            const bool dist_start = cp < 0 || (sm.key[HALO] == 0 && cp != c);
            cb = dist_start ? c : (int64_t)cp + 1;
        } else {  // the tile starts past its distribution's last positive weight
            const Dist &P = a.dists[d_lo];
            cb = P.co + P.m;
        }
        sm.c_begin = cb;
        sm.win_hi = -1;
    }
    __syncthreads();

    // ---- phase 3: parent links of the internal nodes ------------------------
    // Only a boundary inside a cell (level below SENT) is a node under
    // another node; the leaf children follow from three neighbouring levels
    // (phase 4).  Thread g takes the four boundaries 4g..4g+3 and holds the
    // twenty levels around them as five 32-bit words.  Each boundary's
    // nearest higher boundary on either side comes from byte-parallel
    // compares and selects, without branches; only a subtree wider than the
    // window scans on in LDS.
    {
        const uint32_t *lv32 = reinterpret_cast<const uint32_t *>(sm.lvl8);
        constexpr int NW32 = LEAF_N / 4;  // 32-bit level words
        for (int g = tid; g < NW32; g += BT) {
            uint32_t W[5];
            bool V[5];  // word inside the tile's level array
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int gi = g - 2 + k;
                V[k] = gi >= 0 && gi < NW32;
                W[k] = V[k] ? lv32[gi] : 0u;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int bi = 4 * g + q;
                const int l = (int)((W[2] >> (8 * q)) & 0xff);
                const bool active = bi < LVL_N && l < SENT;
                // L: nearest boundary left of bi with a level above l
                const uint32_t tl = __builtin_amdgcn_perm(0u, (uint32_t)(127 - l), 0u);
                const uint32_t m2 = ((W[2] + tl) & 0x80808080u) & ((1u << (8 * q)) - 1u);
                const uint32_t m1 = V[1] ? (W[1] + tl) & 0x80808080u : 0u;
                const uint32_t m0 = V[0] ? (W[0] + tl) & 0x80808080u : 0u;
                const uint32_t mL = m2 ? m2 : (m1 ? m1 : m0);
                const uint32_t wL = m2 ? W[2] : (m1 ? W[1] : W[0]);
                const int kL = m2 ? 2 : (m1 ? 1 : 0);
                const int pL = (31 - __builtin_clz(mL | 0x80u)) >> 3;
                int L = 4 * (g - 2 + kL) + pL;
                int lL = (int)((wL >> (8 * pL)) & 0xff);
                // R: nearest boundary right of bi with a level at least l
                const uint32_t tr = __builtin_amdgcn_perm(0u, (uint32_t)(128 - l), 0u);
                const uint32_t r2 = q < 3 ? ((W[2] + tr) & 0x80808080u) & (~0u << (8 * q + 8)) : 0u;
                const uint32_t r3 = V[3] ? (W[3] + tr) & 0x80808080u : 0u;
                const uint32_t r4 = V[4] ? (W[4] + tr) & 0x80808080u : 0u;
                const uint32_t mR = r2 ? r2 : (r3 ? r3 : r4);
                const uint32_t wR = r2 ? W[2] : (r3 ? W[3] : W[4]);
                const int kR = r2 ? 2 : (r3 ? 3 : 4);
                const int pR = __builtin_ctz(mR | 0x80000000u) >> 3;
                int R = 4 * (g - 2 + kR) + pR;
                int lR = (int)((wR >> (8 * pR)) & 0xff);
                if (active && mL == 0) {  // wider subtree: scan on left of the window
                    L = nearest_ge_left(sm, 4 * (g - 2) - 1, l + 1);
                    lL = L >= 0 ? lvl_at(sm, L) : 0;
                }
                if (active && mR == 0) {  // and right of it
                    R = nearest_ge_right(sm, 4 * (g + 3), l);
                    lR = R >= 0 ? lvl_at(sm, R) : 0;
                }
                if (R >= LVL_N) R = -1;  // the padding byte: beyond the window
                if (active && L >= 0 && R >= 0) {  // else the fix-up finds the parent
                    if (lL > lR) link(sm, R + 1, 0, bi + 1);
                    else link(sm, L + 1, 1, bi + 1);
                }
            }
        }
    }
    __syncthreads();

    // ---- phase 4: node records; guide cells into the window ----------------
    const int live_nodes = (int)(n - base < TILE ? n - base : TILE);
    int xmax = -1;  // highest window position this thread wrote
    for (int jl = tid; jl < live_nodes; jl += BT) {
        const int li = HALO + jl;
        const int32_t gj = lb0 + li;  // global node / leaf index
        const uint64_t kj = sm.key[li];
        const int32_t cj = sm.cell[li];
        int32_t c0 = ~gj, c1 = ~gj;
        if (cj >= 0) {
            // boundary li - 1 is node gj's own; a leaf child follows from the
            // levels of its two boundaries, an internal child was linked into
            // the slot in phase 3
            const int l2 = lvl_at(sm, li - 2), l1 = lvl_at(sm, li - 1), l0 = lvl_at(sm, li);
            const bool root = l1 == SENT;
            c0 = root ? ((kj == 0) ? ~gj : ~(gj - 1)) : (l2 > l1 ? ~(gj - 1) : slot_ref(sm, 2 * jl, lb0));
            c1 = l1 <= l0 ? ~gj : slot_ref(sm, 2 * jl + 1, lb0);
            if (c0 == SLOT_EMPTY || c1 == SLOT_EMPTY) push_item(sm, gj);
            // leaf gj+1 carries mass and belongs to gj's distribution
            const int32_t nc = sm.cell[li + 1];
            const bool next_same = nc >= 0 && !(sm.key[li + 1] == 0 && nc != cj);
            if (root) {
                const int64_t x = cj - sm.c_begin;
                if (x >= 0 && x < WIN) {
                    sm.win[x] = (uint16_t)(WIN_ROOT | li);
                    xmax = max(xmax, (int)x);
                } else {
                    root_cell_record(sm, a.cells, cj, li, lb0);
                }
                const int32_t pc = sm.cell[li - 1];
                if (kj != 0 && cj - pc > 1) {
                    if (cj - pc - 1 > RUN_CAP) push_run(a, pc + 1, cj, gj - 1, sm.key[li - 1], kj);
                    else
                        for (int64_t c = pc + 1; c < cj; ++c)
                            xmax = max(xmax, put_cell(sm, a.cells, c, (uint16_t)(WIN_HEAD | li), lb0));
                }
            }
            // the distribution's last leaf with mass covers the remaining cells
            if (!next_same) {
                const Dist &P = a.dists[BATCHED ? find_segment_in(a.elem_off, d_lo, d_hi + 1, gj) : 0];
                const int64_t cend = P.co + P.m;
                if (cend - cj > 1) {
                    if (cend - cj - 1 > RUN_CAP) push_run(a, cj + 1, cend, gj, kj, KEY_END);
                    else
                        for (int64_t c = cj + 1; c < cend; ++c)
                            xmax = max(xmax, put_cell(sm, a.cells, c, (uint16_t)(WIN_TAIL | li), lb0));
                }
            }
        }
        // a deferred node's children are rewritten by the fix-up kernel
        store_node(a.nodes, gj, kj, c0, c1);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) xmax = max(xmax, __shfl_xor(xmax, o, 64));
    if ((tid & 63) == 0) atomicMax(&sm.win_hi, xmax);
    __syncthreads();

    // ---- phase 5: the staged guide cells, 64 consecutive records per wave ---
    const int span = sm.win_hi + 1;
    for (int x = tid; x < span; x += BT) {
        const uint16_t w = sm.win[x];
        if (w == WIN_EMPTY) continue;
        const int64_t c = sm.c_begin + x;
        const int li = w & WIN_LEAF;
        const int32_t g = lb0 + li;
        const int kind = w & WIN_KIND;
        if (kind == WIN_ROOT) root_cell_record(sm, a.cells, c, li, lb0);
        else if (kind == WIN_HEAD) store_covered(a.cells, c, sm.key[li - 1], sm.key[li], g - 1);
        else store_covered(a.cells, c, sm.key[li], KEY_END, g);
    }
    // the deferred nodes join one grid-wide list (a tile with more than
    // DEFER_CAP of them is redone whole by the fix-up instead)
    const int32_t nd = sm.ndefer;
    if (tid == 0) a.defer_count[t] = nd;
    if (nd > 0 && nd <= DEFER_CAP) {  // uniform across the block
        if (tid == 0) sm.item_base = (int32_t)atomicAdd(a.item_count, (uint32_t)nd);
        __syncthreads();
        for (int32_t q = tid; q < nd; q += BT) a.defer_items[sm.item_base + q] = sm.items[q];
    }
}

// ---------------------------------------------------------------------------
// k_fixup: the deferred work, from the keys in global memory
// ---------------------------------------------------------------------------
// Wave-wide search for the end of a run: pred(d) holds for 0 <= d <= D and
// fails for d > D; d past `lim` counts as failing without being evaluated.
// pred(0) must hold.  The lanes probe 64 distances per step, first galloping
// (strides 1, 64, 4096, ...) and then cutting the bracket 64-fold per step.
// Every lane returns D.
template <class Pred>
__device__ inline int64_t wave_run(Pred pred, int64_t lim) {
    const int64_t lane = threadIdx.x & 63;
    int64_t good = 0, bad = 0, s = 1;
    for (;;) {
        const int64_t d = good + s * (lane + 1);
        const uint64_t fail = __ballot(!(d <= lim && pred(d)));
        if (fail == 0) {
            good += 64 * s;
            s *= 64;
            continue;
        }
        const int64_t f = __builtin_ctzll(fail);
        bad = good + s * (f + 1);
        bad = bad < lim + 1 ? bad : lim + 1;  // the refinement probes only d < bad
        good += s * f;
        break;
    }
    while (bad - good > 1) {
        const int64_t step = (bad - good + 63) / 64;
        const int64_t d = good + step * (lane + 1);  // lane 63 reaches bad
        const uint64_t fail = __ballot(!(d < bad && pred(d)));
        const int64_t f = __builtin_ctzll(fail);
        const int64_t nb = good + step * (f + 1);
        good += step * f;
        bad = nb < bad ? nb : bad;
    }
    return good;
}

// The view is confined to one distribution: a subtree, a cell and a run never
// leave it, and a leaf outside it reads as a position outside [0, n) (it can
// be neither in the same cell nor in the same distribution).
template <bool BATCHED>
struct GlobalView {
    const BuildArgs &a;
    const Dist &P;
    const int64_t e0, e1;  // the distribution's elements [e0, e1)
    __device__ GlobalView(const BuildArgs &args, const Dist &dist)
        : a(args), P(dist), e0(dist.eo), e1(dist.eo + dist.n) {}
    __device__ Leaf leaf(int64_t i) const {
        Leaf L;
        L.key = 0;
        L.cell = -2;
        if (i < e0 || i >= e1) return L;
        L.key = a.nodes[i].key;
        if (L.key == ~0ull) {
            L.cell = -1;
            return L;
        }
        L.cell = cell_of_key(L.key, P);
        return L;
    }
    __device__ int level(int64_t b) const { return level_between(leaf(b), leaf(b + 1)); }
    // leaf x lies in the subtree range of a leaf with key kk in cell c at level l
    __device__ bool in_range(int64_t x, uint64_t kk, int32_t c, int l) const {
        Leaf L = leaf(x);
        if (L.cell != c) return false;
        if (l >= 64) return true;
        return ((L.key ^ kk) >> l) == 0;
    }
    // smallest a <= k with in_range on [a, k] (in_range(k) holds)
    __device__ int64_t extend_left(int64_t k, uint64_t kk, int32_t c, int l) const {
        int64_t good = k, bad = e0 - 1;
        for (int64_t dd = 1;; dd <<= 1) {
            int64_t x = k - dd;
            if (x < e0 || !in_range(x, kk, c, l)) {
                bad = x < e0 - 1 ? e0 - 1 : x;
                break;
            }
            good = x;
        }
        while (good - bad > 1) {
            int64_t mid = bad + (good - bad) / 2;
            if (in_range(mid, kk, c, l)) good = mid;
            else bad = mid;
        }
        return good;
    }
    // largest b >= k with in_range on [k, b] (in_range(k) holds)
    __device__ int64_t extend_right(int64_t k, uint64_t kk, int32_t c, int l) const {
        int64_t good = k, bad = e1;
        for (int64_t dd = 1;; dd <<= 1) {
            int64_t x = k + dd;
            if (x >= e1 || !in_range(x, kk, c, l)) {
                bad = x > e1 ? e1 : x;
                break;
            }
            good = x;
        }
        while (bad - good > 1) {
            int64_t mid = good + (bad - good) / 2;
            if (in_range(mid, kk, c, l)) good = mid;
            else bad = mid;
        }
        return good;
    }
    // root of the subtree over leaves [lo, hi] of one cell: the boundary of
    // highest level, where the highest bit in which key_lo and key_hi differ
    // turns from 0 to 1 (the rightmost boundary if all keys are equal)
    __device__ int32_t root(int64_t lo, int64_t hi) const {
        if (lo == hi) return ~(int32_t)lo;
        uint64_t klo = a.nodes[lo].key, khi = a.nodes[hi].key;
        int lam = level_of(klo, khi);
        if (lam == 0) return (int32_t)hi;
        const int bit = lam - 1;
        int64_t g = lo, b = hi;  // bit clear at g, set at b
        while (b - g > 1) {
            int64_t mid = g + (b - g) / 2;
            if ((a.nodes[mid].key >> bit) & 1) b = mid;
            else g = mid;
        }
        return (int32_t)(g + 1);
    }
    // the record of node j, and whether j is the first node of its cell
    __device__ bool node(int64_t j, uint64_t &kj, int32_t &c0, int32_t &c1) const {
        Leaf Lj = leaf(j);
        kj = Lj.key;
        c0 = c1 = ~(int32_t)j;
        if (Lj.cell < 0) return false;
        Leaf Lp = leaf(j - 1);
        int l = level_between(Lp, Lj);
        if (l == SENT) {
            c0 = (Lj.key == 0) ? ~(int32_t)j : ~(int32_t)(j - 1);
            int64_t b = extend_right(j, Lj.key, Lj.cell, 64);
            c1 = root(j, b);
            return true;
        }
        const int64_t k = j - 1;
        int64_t lo = extend_left(k, Lp.key, Lp.cell, l);
        int64_t hi = (l == 0) ? j : extend_right(j, Lp.key, Lp.cell, l);
        c0 = root(lo, k);
        c1 = root(j, hi);
        return false;
    }
    // The same record computed by one whole wave for one node j (j uniform
    // across the wave): each search probes 64 positions per step, so a
    // subtree range of D leaves costs about 2 log64 D dependent loads in
    // place of 2 log2 D.
    __device__ bool node_wave(int64_t j, uint64_t &kj, int32_t &c0, int32_t &c1) const {
        Leaf Lj = leaf(j);
        kj = Lj.key;
        c0 = c1 = ~(int32_t)j;
        if (Lj.cell < 0) return false;
        Leaf Lp = leaf(j - 1);
        int l = level_between(Lp, Lj);
        if (l == SENT) {
            c0 = (Lj.key == 0) ? ~(int32_t)j : ~(int32_t)(j - 1);
            const int64_t b = j + wave_run([&](int64_t d) { return in_range(j + d, Lj.key, Lj.cell, 64); }, e1 - 1 - j);
            c1 = root_wave(j, b);
            return true;
        }
        const int64_t k = j - 1;
        const int64_t lo = k - wave_run([&](int64_t d) { return in_range(k - d, Lp.key, Lp.cell, l); }, k - e0);
        const int64_t hi =
            (l == 0) ? j : j + wave_run([&](int64_t d) { return in_range(j + d, Lp.key, Lp.cell, l); }, e1 - 1 - j);
        c0 = root_wave(lo, k);
        c1 = root_wave(j, hi);
        return false;
    }
    __device__ int32_t root_wave(int64_t lo, int64_t hi) const {
        if (lo == hi) return ~(int32_t)lo;
        const uint64_t klo = a.nodes[lo].key, khi = a.nodes[hi].key;
        const int lam = level_of(klo, khi);
        if (lam == 0) return (int32_t)hi;
        const int bit = lam - 1;
        // keys of [lo, hi] share the bits above `bit`, so the bit is clear on
        // a prefix of the range and set on the rest
        const int64_t D = wave_run([&](int64_t d) { return ((a.nodes[lo + d].key >> bit) & 1) == 0; }, hi - lo - 1);
        return (int32_t)(lo + D + 1);
    }
    // the guide cell record of the cell whose first node is j
    __device__ void root_cell(int64_t j, int32_t c1) const {
        uint64_t key[CELL_BOUNDS + 1];
        int32_t cell[CELL_BOUNDS + 1];
#pragma unroll
        for (int t = 0; t <= CELL_BOUNDS; ++t) {
            const Leaf L = leaf(j + t);
            key[t] = L.key;
            cell[t] = L.cell;
        }
        const uint64_t kprev = key[0] == 0 ? 0 : a.nodes[j - 1].key;
        root_record(a.cells, cell[0], (int32_t)j, kprev, key, cell, c1);
    }
};

template <class T, bool BATCHED>
__device__ void fixup_tile(const BuildArgs &a, int64_t t);

// The deferred nodes of all tiles are one list: while it is short, each
// wave of the grid takes one node at a time (its searches then take 64
// probes per step), else each thread does.  Each block also reads the
// deferral counts of a contiguous range of tiles in parallel and redoes, one
// thread per node, a tile that deferred more than it could list.  Then every
// wave fills an equal share of the cells of the listed guide-table runs.
template <class T, bool BATCHED>
__global__ __launch_bounds__(T::BT) void k_fixup(BuildArgs a) {
    constexpr int BT = T::BT, TILE = T::TILE, DEFER_CAP = T::DEFER_CAP;
    constexpr int NW = BT / 64;
    __shared__ int32_t s_list[BT];
    __shared__ int32_t s_nt;
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int64_t nwaves = (int64_t)gridDim.x * NW, gw = (int64_t)blockIdx.x * NW + wid;
    auto dist_of = [&](int64_t j) -> const Dist & {
        const int64_t tq = j / TILE;  // a listed node belongs to the tile that deferred it
        return a.dists[BATCHED ? find_segment_in(a.elem_off, a.tile_dist[tq], a.tile_dist[tq + 1] + 1, j) : 0];
    };
    const int64_t ni = *a.item_count;
    if (ni <= 2 * nwaves) {
        for (int64_t q = gw; q < ni; q += nwaves) {
            const int64_t j = a.defer_items[q];
            GlobalView<BATCHED> gv(a, dist_of(j));
            uint64_t kj;
            int32_t c0, c1;
            const bool first = gv.node_wave(j, kj, c0, c1);
            if (lane == 0) {
                if (first) gv.root_cell(j, c1);
                store_node(a.nodes, j, kj, c0, c1);
            }
        }
    } else {
        for (int64_t q = (int64_t)blockIdx.x * BT + tid; q < ni; q += (int64_t)gridDim.x * BT) {
            const int64_t j = a.defer_items[q];
            GlobalView<BATCHED> gv(a, dist_of(j));
            uint64_t kj;
            int32_t c0, c1;
            if (gv.node(j, kj, c0, c1)) gv.root_cell(j, c1);
            store_node(a.nodes, j, kj, c0, c1);
        }
    }
    const int64_t per = (a.ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t t_lo = (int64_t)blockIdx.x * per;
    const int64_t t_hi = t_lo + per < a.ntiles ? t_lo + per : a.ntiles;
    for (int64_t t0 = t_lo; t0 < t_hi; t0 += BT) {
        if (tid == 0) s_nt = 0;
        __syncthreads();
        const int64_t t = t0 + tid;
        if (t < t_hi && a.defer_count[t] > DEFER_CAP) s_list[atomicAdd(&s_nt, 1)] = tid;
        __syncthreads();
        const int32_t nt = s_nt;
        for (int32_t q = 0; q < nt; ++q) fixup_tile<T, BATCHED>(a, t0 + s_list[q]);
        __syncthreads();
    }
    // the listed cells [0, total) in equal contiguous shares, one per wave
    const uint64_t rc = *a.run_count;
    const int64_t cap = run_cap(a.m_total);
    const int64_t nrun = (int64_t)(rc >> 32);
    const int64_t total = nrun > 0 && nrun <= cap ? (int64_t)(uint32_t)rc : 0;  // else flagged
    int64_t p = total * gw / nwaves;
    const int64_t p_end = total * (gw + 1) / nwaves;
    if (p >= p_end) return;
    // the last run whose offset is at most p (runs[0].off = 0)
    int64_t r = wave_run([&](int64_t d) { return (int64_t)a.runs[d].off <= p; }, nrun - 1);
    // the records as a flat array of 16-byte words, so that one store of the
    // wave writes 1 KiB in a row: lane l always writes word l % CELL_WORDS of
    // a record (keys k0 and k1, zeros, then zero, ref and aux in the last)
    static_assert(64 % CELL_WORDS == 0, "a wave store covers whole records");
    uint4 *words = reinterpret_cast<uint4 *>(a.cells);
    const int wq = lane % CELL_WORDS;
    while (p < p_end) {
        const Run R = a.runs[r];
        const int64_t e = (int64_t)R.off + R.len < p_end ? (int64_t)R.off + R.len : p_end;
        const uint32_t ni = ~(uint32_t)R.i;
        const uint4 v = wq == 0                ? make_uint4((uint32_t)R.k0, (uint32_t)(R.k0 >> 32), (uint32_t)R.k1,
                                                            (uint32_t)(R.k1 >> 32))
                        : wq == CELL_WORDS - 1 ? make_uint4(0u, 0u, ni, ni)
                                               : make_uint4(0u, 0u, 0u, 0u);
        const int64_t w1 = CELL_WORDS * ((int64_t)R.lo + (e - (int64_t)R.off));
        for (int64_t w = CELL_WORDS * ((int64_t)R.lo + (p - (int64_t)R.off)) + lane; w < w1; w += 64) words[w] = v;
        p = e;
        ++r;
    }
}

template <class T, bool BATCHED>
__device__ void fixup_tile(const BuildArgs &a, int64_t t) {
    constexpr int BT = T::BT, TILE = T::TILE;
    // more deferrals than a tile lists: redo every node record of the tile
    const int64_t base = t * TILE;
    const int32_t d_lo = BATCHED ? a.tile_dist[t] : 0, d_hi = BATCHED ? a.tile_dist[t + 1] : 0;
    const int64_t count = a.n_total - base < TILE ? a.n_total - base : TILE;
    for (int64_t k = threadIdx.x; k < count; k += BT) {
        const int64_t j = base + k;
        const Dist &P = a.dists[BATCHED ? find_segment_in(a.elem_off, d_lo, d_hi + 1, j) : 0];
        GlobalView<BATCHED> gv(a, P);
        uint64_t kj;
        int32_t c0, c1;
        if (gv.node(j, kj, c0, c1)) gv.root_cell(j, c1);
        store_node(a.nodes, j, kj, c0, c1);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// k_widen: collapsed (4-ary) nodes for the cells whose trees samples descend
// (Sec. 5: a wider tree results from collapsing two binary levels; on this
// GPU every random read moves a whole line, so a 64-byte record holding two
// levels costs the same read as a 16-byte one).  One thread per node j; the
// record is written for the internal nodes of cells with more than
// CELL_BOUNDS lower bounds (all but the cell's first node a, whose child 1
// is where those samples' descent starts).
// ---------------------------------------------------------------------------
constexpr int WT = 256;

template <bool BATCHED>
__global__ __launch_bounds__(WT) void k_widen(const Node *__restrict__ nodes,
                                              const Cell *__restrict__ cells,
                                              const Dist *__restrict__ dists,
                                              const int64_t *__restrict__ eoff, int32_t D,
                                              int64_t n, Wide *__restrict__ wide) {
    __shared__ int32_t s_d[2];
    const int64_t j0 = (int64_t)blockIdx.x * WT;
    const int64_t j = j0 + threadIdx.x;
    int32_t dlo = 0, dhi = 0;
    if (BATCHED) {
        // distributions of the block's first and last node, one wave each
        const int w = threadIdx.x >> 6;
        if (w < 2) {
            const int64_t jl = j0 + WT - 1 < n ? j0 + WT - 1 : n - 1;
            const int32_t d = wave_upper_bound(eoff, D, w == 0 ? j0 : jl) - 1;
            if ((threadIdx.x & 63) == 0) s_d[w] = d;
        }
        __syncthreads();
        dlo = s_d[0];
        dhi = s_d[1];
    }
    if (j >= n) return;
    const Node nd = nodes[j];
    if (nd.key == KEY_END) return;  // past the last positive weight: never descended
    const int32_t d = (!BATCHED || dlo == dhi) ? dlo : find_segment_in(eoff, dlo, dhi + 1, j);
    const Dist P = dists[d];
    if (P.flags & DIST_ZERO) return;
    const int64_t g = cell_of_key(nd.key, P);
    const int2 ra = *reinterpret_cast<const int2 *>(&cells[g].ref);
    if (ra.x < 0 || ra.y < 0 || ra.x == (int32_t)j) return;  // covered, resolved by its record, or node a
    uint64_t kc[2];
    int32_t r[4];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int32_t c = side ? nd.c1 : nd.c0;
        if (c >= 0) {
            const Node cn = nodes[c];
            kc[side] = cn.key;
            r[2 * side] = cn.c0;
            r[2 * side + 1] = cn.c1;
        } else {
            kc[side] = 0;
            r[2 * side] = r[2 * side + 1] = c;
        }
    }
    uint4 *q = reinterpret_cast<uint4 *>(wide + j);
    q[0] = make_uint4((uint32_t)nd.key, (uint32_t)(nd.key >> 32), (uint32_t)kc[0],
                      (uint32_t)(kc[0] >> 32));
    q[1] = make_uint4((uint32_t)kc[1], (uint32_t)(kc[1] >> 32), (uint32_t)r[0], (uint32_t)r[1]);
    q[2] = make_uint4((uint32_t)r[2], (uint32_t)r[3], 0u, 0u);
    q[3] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_widen(const Node *nodes, const Cell *cells, const Dist *dists,
                        const int64_t *elem_off, int32_t D, int64_t n_total, Wide *wide,
                        hipStream_t st) {
    const dim3 g((unsigned)((n_total + WT - 1) / WT)), b(WT);
    if (D > 1)
        hipLaunchKernelGGL(k_widen<true>, g, b, 0, st, nodes, cells, dists, elem_off, D, n_total,
                           wide);
    else
        hipLaunchKernelGGL(k_widen<false>, g, b, 0, st, nodes, cells, dists, elem_off, D, n_total,
                           wide);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_depth: the deepest search of the forest, counted as Alg. 2 counts it (the
// guide entry, then one node per step).  Every u in leaf i's interval takes
// the path that u = U_i takes from the cell holding U_i (the keys compared
// lie outside the interval), and from a later cell the interval covers the
// search ends at once (a covered cell) or after node a, whose child 0 is i.
// So the maximum over the leaves with positive weight of the path for U_i
// is the deepest search any uniform makes.  One thread per leaf; the result
// goes to the forest's status block with an atomic maximum.
// ---------------------------------------------------------------------------
template <bool BATCHED>
__global__ __launch_bounds__(WT) void k_depth(const Node *__restrict__ nodes,
                                              const Cell *__restrict__ cells,
                                              const Dist *__restrict__ dists,
                                              const int64_t *__restrict__ eoff, int32_t D,
                                              int64_t n, uint32_t *depth) {
    __shared__ int32_t s_d[2];
    const int64_t i0 = (int64_t)blockIdx.x * WT;
    const int64_t i = i0 + threadIdx.x;
    int32_t dlo = 0, dhi = 0;
    if (BATCHED) {
        const int w = threadIdx.x >> 6;
        if (w < 2) {
            const int64_t il = i0 + WT - 1 < n ? i0 + WT - 1 : n - 1;
            const int32_t d = wave_upper_bound(eoff, D, w == 0 ? i0 : il) - 1;
            if ((threadIdx.x & 63) == 0) s_d[w] = d;
        }
        __syncthreads();
        dlo = s_d[0];
        dhi = s_d[1];
    }
    uint32_t steps = 0;
    if (i < n) {
        const int32_t d = (!BATCHED || dlo == dhi) ? dlo : find_segment_in(eoff, dlo, dhi + 1, i);
        const Dist P = dists[d];
        const uint64_t key = nodes[i].key;
        const uint64_t next = i + 1 < P.eo + P.n ? nodes[i + 1].key : KEY_END;
        // leaf i carries mass: its key is real and the next bound lies above it
        const bool live = !(P.flags & DIST_ZERO) && key != KEY_END && (next != key || next == KEY_END);
        if (live) {
            int32_t j = cells[cell_of_key(key, P)].ref;
            steps = 1;  // the guide entry
            for (int64_t guard = 0; j >= 0 && guard <= n; ++guard) {
                const Node nd = nodes[j];
                j = key < nd.key ? nd.c0 : nd.c1;
                ++steps;
            }
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t y = __shfl_xor(steps, o, 64);
        steps = y > steps ? y : steps;
    }
    if ((threadIdx.x & 63) == 0 && steps) atomicMax(depth, steps);
}

__global__ void k_clear_word(uint32_t *w) { *w = 0u; }

hipError_t launch_depth(const Node *nodes, const Cell *cells, const Dist *dists,
                        const int64_t *elem_off, int32_t D, int64_t n_total, uint32_t *depth,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, st, depth);
    const dim3 g((unsigned)((n_total + WT - 1) / WT)), b(WT);
    if (D > 1)
        hipLaunchKernelGGL(k_depth<true>, g, b, 0, st, nodes, cells, dists, elem_off, D, n_total,
                           depth);
    else
        hipLaunchKernelGGL(k_depth<false>, g, b, 0, st, nodes, cells, dists, elem_off, D, n_total,
                           depth);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Depth fallback (Sec. 3: a degenerate tree is replaced by a structure of
// logarithmic depth).  The tree of a cell holding c lower bounds (leaves
// a..b, hung as child 1 of node a) is replaced when a leaf with positive
// weight lies more than 2 ceil(log2 c) internal nodes deep in it, by the
// balanced tree that splits [lo, hi] at mid = ceil((lo + hi) / 2).  Keys and
// guide entries stay, so every search still returns the binary-search index.
//   k_bal_clear    per cell: deepest search 0, last leaf -1
//   k_bal_measure  per leaf: the cell's last leaf (atomic max of the index);
//                  for a leaf with positive weight, the nodes Alg. 2 visits
//                  from node a down to it (atomic max)
//   k_bal_rebuild  per node of a degenerate cell: its children in the
//                  balanced tree, found by descending the implicit splits
//                  from [a, b] (log2 c steps); node a takes the new root as
//                  child 1, and so does the cell record when c > CELL_BOUNDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WT) void k_bal_clear(int32_t *deep, int32_t *last, int64_t m,
                                                 uint32_t *count) {
    const int64_t g = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (g < m) {
        deep[g] = 0;
        last[g] = -1;
    }
    if (g == 0) *count = 0u;
}

// The distribution of element i of a block that spans distributions
// [dlo, dhi] (found once per block by two wave-wide searches).
template <bool BATCHED>
__device__ inline void block_dists(const int64_t *eoff, int32_t D, int64_t n, int64_t i0,
                                   int32_t *s_d, int32_t &dlo, int32_t &dhi) {
    dlo = dhi = 0;
    if (!BATCHED) return;
    const int w = threadIdx.x >> 6;
    if (w < 2) {
        const int64_t il = i0 + WT - 1 < n ? i0 + WT - 1 : n - 1;
        const int32_t d = wave_upper_bound(eoff, D, w == 0 ? i0 : il) - 1;
        if ((threadIdx.x & 63) == 0) s_d[w] = d;
    }
    __syncthreads();
    dlo = s_d[0];
    dhi = s_d[1];
}

template <bool BATCHED>
__global__ __launch_bounds__(WT) void k_bal_measure(const Node *__restrict__ nodes,
                                                   const Cell *__restrict__ cells,
                                                   const Dist *__restrict__ dists,
                                                   const int64_t *__restrict__ eoff, int32_t D,
                                                   int64_t n, int32_t *deep, int32_t *last) {
    __shared__ int32_t s_d[2];
    const int64_t i0 = (int64_t)blockIdx.x * WT;
    const int64_t i = i0 + threadIdx.x;
    int32_t dlo, dhi;
    block_dists<BATCHED>(eoff, D, n, i0, s_d, dlo, dhi);
    if (i >= n) return;
    const int32_t d = (!BATCHED || dlo == dhi) ? dlo : find_segment_in(eoff, dlo, dhi + 1, i);
    const Dist P = dists[d];
    const uint64_t key = nodes[i].key;
    if ((P.flags & DIST_ZERO) || key == KEY_END) return;  // no tree holds this leaf
    const int64_t g = cell_of_key(key, P);
    atomicMax(last + g, (int32_t)i);
    const uint64_t next = i + 1 < P.eo + P.n ? nodes[i + 1].key : KEY_END;
    if (next == key && next != KEY_END) return;  // zero weight: no uniform reaches it
    int32_t j = cells[g].ref;  // node a: the leaf's lower bound lies in g
    int32_t visits = 0;
    for (int64_t guard = 0; j >= 0 && guard <= n; ++guard) {
        const Node nd = nodes[j];
        j = key < nd.key ? nd.c0 : nd.c1;
        ++visits;
    }
    atomicMax(deep + g, visits);
}

__device__ inline int ceil_log2_i64(int64_t c) { return c <= 1 ? 0 : 64 - __builtin_clzll((uint64_t)(c - 1)); }

// reference to the balanced subtree over leaves [lo, hi]
__device__ inline int32_t split_ref(int64_t lo, int64_t hi) {
    return lo == hi ? ~(int32_t)lo : (int32_t)((lo + hi + 1) / 2);
}

template <bool BATCHED>
__global__ __launch_bounds__(WT) void k_bal_rebuild(Node *__restrict__ nodes, Cell *__restrict__ cells,
                                                   const Dist *__restrict__ dists,
                                                   const int64_t *__restrict__ eoff, int32_t D,
                                                   int64_t n, const int32_t *__restrict__ deep,
                                                   const int32_t *__restrict__ last,
                                                   uint32_t *count) {
    __shared__ int32_t s_d[2];
    const int64_t j0 = (int64_t)blockIdx.x * WT;
    const int64_t j = j0 + threadIdx.x;
    int32_t dlo, dhi;
    block_dists<BATCHED>(eoff, D, n, j0, s_d, dlo, dhi);
    if (j >= n) return;
    const int32_t d = (!BATCHED || dlo == dhi) ? dlo : find_segment_in(eoff, dlo, dhi + 1, j);
    const Dist P = dists[d];
    const uint64_t key = nodes[j].key;
    if ((P.flags & DIST_ZERO) || key == KEY_END) return;
    const int64_t g = cell_of_key(key, P);
    const int64_t a = cells[g].ref, b = last[g], c = b - a + 1;
    if (deep[g] - 1 <= 2 * ceil_log2_i64(c)) return;  // not degenerate
    if (j == a) {
        const int32_t root = split_ref(a, b);
        nodes[j].c1 = root;
        if (c > CELL_BOUNDS) cells[g].aux = root;
        atomicAdd(count, 1u);
        return;
    }
    int64_t lo = a, hi = b, mid = (lo + hi + 1) / 2;
    while (mid != j) {  // j in (a, b]: every range on the way holds it
        if (j < mid) hi = mid - 1;
        else lo = mid;
        mid = (lo + hi + 1) / 2;
    }
    nodes[j].c0 = split_ref(lo, mid - 1);
    nodes[j].c1 = split_ref(mid, hi);
}

hipError_t launch_balance(Node *nodes, Cell *cells, const Dist *dists, const int64_t *elem_off,
                          int32_t D, int64_t n_total, int64_t m_total, int32_t *deep,
                          int32_t *last, uint32_t *count, hipStream_t st) {
    hipLaunchKernelGGL(k_bal_clear, dim3((unsigned)((m_total + WT - 1) / WT)), dim3(WT), 0, st,
                       deep, last, m_total, count);
    const dim3 g((unsigned)((n_total + WT - 1) / WT)), b(WT);
    if (D > 1) {
        hipLaunchKernelGGL(k_bal_measure<true>, g, b, 0, st, nodes, cells, dists, elem_off, D,
                           n_total, deep, last);
        hipLaunchKernelGGL(k_bal_rebuild<true>, g, b, 0, st, nodes, cells, dists, elem_off, D,
                           n_total, deep, last, count);
    } else {
        hipLaunchKernelGGL(k_bal_measure<false>, g, b, 0, st, nodes, cells, dists, elem_off, D,
                           n_total, deep, last);
        hipLaunchKernelGGL(k_bal_rebuild<false>, g, b, 0, st, nodes, cells, dists, elem_off, D,
                           n_total, deep, last, count);
    }
    return hipGetLastError();
}

template <class T>
void enqueue_build(const BuildArgs &a, hipStream_t st) {
    constexpr int BT = T::BT;
    const bool vec = (reinterpret_cast<uintptr_t>(a.w) & 15) == 0;
    const dim3 grid((unsigned)a.ntiles);
    const int ts = a.D > 1 ? T::TS_TILES : T::TS_SINGLE;
    const dim3 sumgrid((unsigned)((a.ntiles + ts - 1) / ts));
    const dim3 fixgrid((unsigned)(a.ntiles < 1024 ? a.ntiles : 1024));
    if (a.D > 1) {
        hipLaunchKernelGGL((k_tile_sums<T, true>), sumgrid, dim3(BT), 0, st, a, vec);
        hipLaunchKernelGGL((k_dist_params<T, true>), dim3(1), dim3(PT), 0, st, a);
        if (a.D > PT)
            hipLaunchKernelGGL((k_dist_finish<T, true>), dim3((unsigned)((a.D + 255) / 256)), dim3(256), 0, st, a);
        hipLaunchKernelGGL((k_build_tile<T, true>), grid, dim3(BT), 0, st, a, vec);
        hipLaunchKernelGGL((k_fixup<T, true>), fixgrid, dim3(BT), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_tile_sums<T, false>), sumgrid, dim3(BT), 0, st, a, vec);
        hipLaunchKernelGGL((k_dist_params<T, false>), dim3(1), dim3(PT), 0, st, a);
        hipLaunchKernelGGL((k_build_tile<T, false>), grid, dim3(BT), 0, st, a, vec);
        hipLaunchKernelGGL((k_fixup<T, false>), fixgrid, dim3(BT), 0, st, a);
    }
}

hipError_t launch_build(const BuildArgs &a, hipStream_t st) {
    if (a.tile == Tile1024::TILE) enqueue_build<Tile1024>(a, st);
    else enqueue_build<Tile2048>(a, st);
    return hipGetLastError();
}

}  // namespace rtf
