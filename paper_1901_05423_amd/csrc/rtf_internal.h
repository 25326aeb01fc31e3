// rtf_internal.h -- shared definitions of the HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rtforest.h"

namespace rtf {

// A level above every real one (0..64): a boundary merges never cross, used
// for cell changes, distribution changes, both array ends and the end of the
// weights that carry mass (Alg. 1 gives the missing neighbours past the array
// ends the largest distance).
constexpr int SENT = 65;

// Build tile shapes: BT threads x ITEMS consecutive elements per block.  The
// forest does not depend on the shape, only the speed does: 2048-element
// tiles of 512 threads suit one large distribution; batches of many uneven
// distributions build faster in 1024-element tiles of 256 threads, whose
// batched kernel then fits its registers without spills.
template <int BT_, int ITEMS_, int WAVES_ONE_, int WAVES_BATCHED_>
struct Tiling {
    static constexpr int BT = BT_;
    static constexpr int ITEMS = ITEMS_;
    // waves per SIMD the tile kernel is compiled for, one distribution and
    // batched (the batched instance needs more registers); the LDS of one
    // tile bounds it too
    static constexpr int WAVES_ONE = WAVES_ONE_;
    static constexpr int WAVES_BATCHED = WAVES_BATCHED_;
    static constexpr int TILE = BT * ITEMS;
    // Guide cells staged in LDS per tile before their coalesced store.  With
    // m proportional to n a tile's records fall in about m/n * TILE
    // consecutive cells; records past the window are stored directly.
    static constexpr int WIN = TILE + 128;
    // Deferred node records kept per tile; more make the fix-up redo the tile.
    static constexpr int DEFER_CAP = TILE / 16;
    // Tiles summed per block of the tile-sum pass: a batch's (one wave per
    // search there), and one distribution's (only sums: more bytes per block).
    static constexpr int TS_TILES = BT / 128;
    static constexpr int TS_SINGLE = BT / 64;
};
using Tile2048 = Tiling<512, 4, 8, 6>;  // 40 KB of LDS per tile: four per CU
using Tile1024 = Tiling<256, 4, 7, 6>;  // 21 KB: seven per CU
constexpr int TILE_DEFAULT = Tile2048::TILE;
// Leaves on either side of a tile whose keys are recomputed locally so that
// subtree scans near the tile edges stay in LDS.
constexpr int HALO = 32;
// Longest in-LDS subtree scan; longer ones are finished by the fix-up kernel.
constexpr int SCAN_CAP = 64;
// Longest guide-table run written by one lane; a longer run is listed for the
// fix-up kernel, whose waves split the listed runs' cells evenly.
constexpr int RUN_CAP = 64;

struct alignas(16) Node {
    uint64_t key;
    int32_t c0, c1;
};

// Collapsed node (Sec. 5: a 4-ary tree from two binary levels), 64 bytes, one
// per internal node j of a cell whose tree the samples descend (a cell with
// more than CELL_BOUNDS lower bounds), stored at index j.  k = U_j; for its
// child c on side s (0 left, 1 right): when c is a node, kc[s] = U_c and
// r[2s], r[2s+1] are c's two children; when c is a leaf, r[2s] = r[2s+1] = c
// and kc[s] = 0.  References as in Node (>= 0 node, < 0 leaf ~i).
struct alignas(64) Wide {
    uint64_t k;
    uint64_t kc[2];
    int32_t r[4];
    uint64_t pad[2];
};
static_assert(sizeof(Wide) == 64, "collapsed nodes are 64 bytes");

// Guide-table cell record, 64 bytes: one memory access per sample in the
// common case.  `ref` is the paper's guide entry (Sec. 2.5, 3.2): the cell's
// first node a, or ~i when one interval i covers the whole cell.  Beside it
// the record keeps the keys that finish a sample without the tree
// (K = CELL_KEYS - 1 = CELL_BOUNDS + 1):
//   ref = ~i < 0:  k[0] = U_i, k[1] = U_{i+1} (KEY_END at the distribution's
//                  end), aux = ref.
//   ref = a >= 0:  the cell holds the c lower bounds U_a .. U_{a+c-1};
//                  k[0] = U_{a-1} (0 at a distribution start) and
//                  k[t] = U_{a+t-1} for t = 1 .. min(c + 1, K), where
//                  U_{a+c} (KEY_END at the distribution's end) is the upper
//                  end of the cell's last interval.
//                  c <= CELL_BOUNDS: aux = ~c, and the record resolves every
//                  sample of the cell.
//                  c > CELL_BOUNDS: aux = child 1 of node a, the root of the
//                  cell's tree; the record resolves u < k[K], larger u
//                  descend the tree from aux.
// Key slots a record does not use hold 0.  (A 128-byte record with 13 bounds
// at half the cells was measured too: fewer descents, no faster sampling,
// and twice the registers per record in the kernels that hold two.)
constexpr int CELL_BOUNDS = 5;
constexpr int CELL_KEYS = CELL_BOUNDS + 2;
struct alignas(64) Cell {
    uint64_t k[CELL_KEYS];
    int32_t ref, aux;
};
static_assert(sizeof(Cell) == 64, "cell records are 64 bytes");
constexpr int CELL_WORDS = sizeof(Cell) / 16;  // 16-byte words of a record
constexpr uint64_t KEY_END = ~0ull;

// A listed guide-table run: cells [lo, lo + len) are all covered by interval
// i, whose keys are k0 and k1.  `off` is the number of cells of the runs
// listed before it, so the listed cells form one sequence [0, total).
struct alignas(32) Run {
    uint64_t k0, k1;
    int32_t lo, len, i;
    uint32_t off;
};

// Capacity of the run list for m cells: listed runs are longer than RUN_CAP
// cells and disjoint.
__host__ __device__ inline int64_t run_cap(int64_t m) { return m / (RUN_CAP + 1) + 1; }

// Per-distribution parameters, written by the build's scan kernel.
struct alignas(64) Dist {
    uint64_t W;   // total weight
    uint64_t v;   // reciprocal of the normalised divisor W << s
    uint64_t G0;  // global prefix sum at the distribution's first element
    int64_t eo;   // first element
    int64_t n;    // elements
    int64_t co;   // first guide cell
    int64_t m;    // guide cells
    uint32_t s;   // clz(W)
    uint32_t flags;
};
constexpr uint32_t DIST_ZERO = 1u;
// bits 8..15 of Dist::flags: 64 - log2(m) when m is a power of two >= 2, else 0
constexpr int DIST_SHIFT_BIT = 8;

// status word bits: 1 << rtf_status
__host__ __device__ inline uint32_t status_bit(int code) { return 1u << code; }

struct BuildArgs {
    const uint32_t *w;
    const int64_t *src_elem_off;  // the caller's offsets (null for one distribution)
    const int64_t *src_cell_off;
    int64_t *elem_off;            // workspace copy, D+1
    int64_t *cell_off;            // workspace copy, D+1
    int32_t D;
    int64_t n_total;
    int64_t m_total;
    int32_t tile;                 // elements per tile: Tile2048::TILE or Tile1024::TILE
    int64_t ntiles;
    Node *nodes;
    Cell *cells;
    Dist *dists;
    uint32_t *status;
    uint64_t *tile_sum;     // [ntiles]
    uint64_t *tile_prefix;  // [ntiles + 1], the last the grand total
    uint64_t *dist_local;   // [D]: in-tile prefix at each distribution start
    int32_t *defer_count;   // [ntiles]
    int32_t *defer_items;   // [ntiles * DEFER_CAP]: the deferred nodes of all tiles, one list
    uint32_t *item_count;   // length of that list
    int32_t *tile_dist;     // [ntiles + 2]: distribution of element min(t tile, n - 1)
    uint64_t *run_count;    // (runs listed << 32) | cells they cover
    Run *runs;              // [run_cap(m_total)]
};

// ---- exact 64-bit fixed-point helpers ----------------------------------

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

__host__ __device__ inline int clz64(uint64_t x) { return x ? __builtin_clzll(x) : 64; }

// floor((2^128 - 1) / d) - 2^64 for a normalised d (top bit set): the
// reciprocal of the 2-by-1 division of Moller and Granlund, "Improved
// division by invariant integers" (IEEE Trans. Computers, 2011).  An FP64
// quotient 2^128 / d (a multiple of 2^12 in (2^64, 2^65], so its excess over
// 2^64 converts exactly) is within 2^13 + 2 of it.  The exact remainder r of
// (2^128 - 1) against (2^64 + v) d is then below 2^78 in magnitude; dividing
// it by d once more in FP64 is off by at most one, and one comparison on
// each side settles that.  A few dozen instructions instead of a 64-step
// bit-serial division on the one thread that computes it per distribution.
__host__ __device__ inline uint64_t reciprocal_2by1(uint64_t d) {
    typedef unsigned __int128 u128;
    typedef __int128 i128;
    const double dd = (double)d;
    const double z = 0x1p128 / dd - 0x1p64;  // exact subtraction, z in [0, 2^64]
    uint64_t v = z >= 0x1p64 ? ~0ull : (uint64_t)z;
    // r = (2^128 - 1) - (2^64 + v) d, computed modulo 2^128 (the complement)
    i128 r = (i128)(~((((u128)1 << 64) | v) * d));
    const double rd = (double)(int64_t)(r >> 64) * 0x1p64 + (double)(uint64_t)r;
    const int64_t q = (int64_t)__builtin_floor(rd / dd);  // |q| <= 2^13 + 3
    v += (uint64_t)q;
    r -= (i128)q * (i128)d;
    while (r < 0) {  // at most once
        v -= 1;
        r += d;
    }
    while (r >= (i128)d) {  // at most once
        v += 1;
        r -= d;
    }
    return v;
}

// Key U = ceil(C * 2^64 / W) for 0 <= C < W, given s = clz(W), d = W << s
// and v = reciprocal_2by1(d): one 2-by-1 division (Moller-Granlund, Alg. 4)
// of (C << s) * 2^64 by d, then rounding up on a non-zero remainder.
__host__ __device__ inline uint64_t fixed_point_key(uint64_t C, uint64_t d, uint64_t v,
                                                     uint32_t s) {
    uint64_t u1 = C << s;  // < d
    uint64_t q0 = v * u1;
    uint64_t q1 = mulhi64(v, u1) + u1 + 1;
    uint64_t r = 0 - q1 * d;
    if (r > q0) {
        q1 -= 1;
        r += d;
    }
    if (r >= d) {
        q1 += 1;
        r -= d;
    }
    return q1 + (r != 0 ? 1 : 0);
}

// Level of the boundary between two neighbouring leaves: 64 - clz(a ^ b).
__host__ __device__ inline int level_of(uint64_t a, uint64_t b) { return 64 - clz64(a ^ b); }

// 1 / b in FP64 for 1 <= b < 2^32: the hardware reciprocal refined by two
// Newton steps, within about an ulp.  Operands of this range never need the
// exponent scaling and special cases of a general division.
__device__ inline double recip_small(double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-b, r, 1.0);
    return __builtin_fma(r, e, r);
}

// a / b in FP64 for 0 <= a <= 2^32 and 1 <= b < 2^32: a times the refined
// reciprocal, then one correction of the quotient; within an ulp or two of
// the rounded quotient.
__device__ inline double div_small(double a, double b) {
    const double r = recip_small(b);
    const double q = a * r;
    return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}

// The blocks of a launch are dispatched to the 8 XCDs in turn (block b to XCD
// b mod 8), and each XCD has its own L2.  xcd_block() renumbers the blocks so
// that each XCD's blocks carry consecutive numbers (a bijection on
// [0, gridDim.x)): work handed out in contiguous ranges of the new number
// then keeps neighbouring ranges, and the data they share, on one XCD.
constexpr int NXCD = 8;
__device__ inline int64_t xcd_block() {
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t q = G / NXCD, r = G % NXCD, x = b % NXCD;
    return x * q + (x < r ? x : r) + b / NXCD;
}

// The first d in [0, D] with off[d] > i (D + 1 if none; off[0..D]
// non-decreasing), found by one wave (uniform i): each step probes 64 evenly
// spaced offsets and keeps the bracket between the last one at or below i
// and the first above it.  Every lane of the wave must call it.
__device__ inline int32_t wave_upper_bound(const int64_t *off, int32_t D, int64_t i) {
    const int32_t lane = threadIdx.x & 63;
    int32_t lo = 0, hi = D + 1;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const int32_t step = (hi - lo + 63) / 64;
        const int32_t p = lo + lane * step;
        const int32_t cnt = __popcll(__ballot(p < hi && off[p] <= i));  // a prefix of the lanes
        if (cnt == 0) {
            hi = lo;
        } else {
            const int32_t last = lo + (cnt - 1) * step;  // off[last] <= i
            const int32_t next = lo + cnt * step;       // off[next] > i, or next >= hi
            lo = last + 1;
            hi = next < hi ? next : hi;
        }
    }
    return lo;
}

// ---- launchers (defined in the .hip files) ----------------------------------

hipError_t launch_build(const BuildArgs &a, hipStream_t st);
hipError_t launch_sample(const Node *nodes, const Wide *wide, const Cell *cells, const Dist *dists,
                         const int64_t *sample_off, int32_t D, int64_t n_total, int64_t m_total,
                         const uint64_t *u, int64_t S, int32_t *idx, double *x,
                         hipStream_t st);
hipError_t launch_sample_2d(const Node *nodes, const Wide *wide, const Cell *cells, const Dist *dists,
                            int32_t D, int64_t n_total, const uint64_t *u2, int64_t S,
                            int32_t *rc, double *xy, hipStream_t st);
hipError_t launch_sample_bsearch(const Node *nodes, const Cell *cells,
                                 const Dist *dists, bool cutpoint, const uint64_t *u,
                                 int64_t S, int32_t *idx, double *x, hipStream_t st);
hipError_t launch_widen(const Node *nodes, const Cell *cells, const Dist *dists,
                        const int64_t *elem_off, int32_t D, int64_t n_total, Wide *wide,
                        hipStream_t st);
hipError_t launch_depth(const Node *nodes, const Cell *cells, const Dist *dists,
                        const int64_t *elem_off, int32_t D, int64_t n_total, uint32_t *depth,
                        hipStream_t st);
// the depth word of the status block
constexpr int STATUS_DEPTH_OFFSET = 128;
// the count of cells the depth fallback rebuilt, in the status block
constexpr int STATUS_BALANCE_OFFSET = 136;
hipError_t launch_balance(Node *nodes, Cell *cells, const Dist *dists, const int64_t *elem_off,
                          int32_t D, int64_t n_total, int64_t m_total, int32_t *deep,
                          int32_t *last, uint32_t *count, hipStream_t st);
hipError_t launch_quantize(const float *v, const int64_t *elem_off, int32_t D,
                           int64_t n_total, uint32_t *out, double *scale,
                           uint32_t *status, hipStream_t st);
// Scratch of the backward pass: per element the sums B and D, per
// distribution A, per chunk of BACKWARD_CHUNK elements the combining pass's
// head sum, link bits and carry.
constexpr int64_t BACKWARD_CHUNK = 4096;
__host__ __device__ constexpr int64_t backward_chunks(int64_t n_total) {
    return (n_total + BACKWARD_CHUNK - 1) / BACKWARD_CHUNK;
}
struct BackwardScratch {
    double *B, *Dv, *A, *head, *carry;
    int32_t *link;
};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Backward scratch layout from base: B[n], D[n], A[D], head[nch], carry[nch],
// link[nch], each 256-byte aligned; returns the bytes it spans (w may be null).
constexpr size_t backward_layout(int32_t D, int64_t n, char *base, BackwardScratch *w) {
    const int64_t nch = backward_chunks(n);
    size_t off[7] = {};
    const size_t bytes[6] = {sizeof(double) * (size_t)n,   sizeof(double) * (size_t)n,
                             sizeof(double) * (size_t)D,   sizeof(double) * (size_t)nch,
                             sizeof(double) * (size_t)nch, sizeof(int32_t) * (size_t)nch};
    for (int k = 0; k < 6; ++k) off[k + 1] = align256(off[k] + bytes[k]);
    if (w) {
        w->B = reinterpret_cast<double *>(base + off[0]);
        w->Dv = reinterpret_cast<double *>(base + off[1]);
        w->A = reinterpret_cast<double *>(base + off[2]);
        w->head = reinterpret_cast<double *>(base + off[3]);
        w->carry = reinterpret_cast<double *>(base + off[4]);
        w->link = reinterpret_cast<int32_t *>(base + off[5]);
    }
    return off[6];
}
// Argument checks and launches of a backward pass over scratch w (rtf_abi.hip).
rtf_status backward_enqueue(const rtf_forest *f, const int64_t *sample_off, const uint64_t *u,
                            const int32_t *idx, const double *grad_x, int64_t S,
                            const double *scale, double *grad_w, const BackwardScratch &w,
                            hipStream_t stream);
hipError_t launch_backward(const Node *nodes, const Dist *dists, const int64_t *elem_off,
                           int32_t D, int64_t n_total, const int64_t *sample_off,
                           const uint64_t *u, const int32_t *idx, const double *gx, int64_t S,
                           const double *scale, double *grad_w, const BackwardScratch &w,
                           hipStream_t st);

}  // namespace rtf
