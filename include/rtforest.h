/*
 * rtforest.h -- C ABI of the MI355X (gfx950) radix-tree-forest sampler.
 *
 * Method: Binder & Keller, "Massively Parallel Construction of Radix Tree
 * Forests for the Efficient Sampling of Discrete or Piecewise Constant
 * Probability Distributions" (arXiv:1901.05423).
 *
 * Problem (Sec. 1): given weights w_0..w_{n-1} >= 0 with positive sum, map a
 * uniform xi in [0,1) to the index i with P_i <= xi < P_{i+1}, where P_k is
 * the normalised partial sum of the first k weights.  The library builds the
 * auxiliary structure of Sec. 3 -- a guide table of m equal cells (Sec. 2.5)
 * plus one radix tree per cell (the radix tree forest, Sec. 3.2, Alg. 1) --
 * and evaluates Alg. 2 for batches of samples.
 *
 * Number formats.  Weights are uint32.  Partial sums C_i are exact uint64.  A
 * uniform is a uint64 u standing for xi = u * 2^-64.  Interval i's lower bound
 * is stored as the 0.64 fixed-point key U_i = ceil(C_i * 2^64 / W), W = C_n;
 * then U_i <= u exactly when C_i <= floor(u*W / 2^64), so the sampled index
 * equals the exact real-number inverse CDF, bit for bit.  Indices are 0-based
 * int32.  The continuous position x (Sec. 5) is FP64 in [0,1]:
 *     x = (i + ((t - C_i) + lo * 2^-64) / w_i) / n,   t:lo = u * W (128 bit).
 *
 * Conventions.
 *  - Every array argument is a DEVICE pointer owned by the caller unless its
 *    name starts with h_ (host pointer).  The library never allocates device
 *    memory and never frees any.
 *  - All calls are asynchronous on the given stream and return once the work
 *    is enqueued, except rtf_check and rtf_forest_export, which synchronise
 *    the stream.
 *  - Errors are returned as rtf_status; nothing is thrown across the ABI.
 *    Argument errors are detected on the host before anything is enqueued.
 *    Errors in the data (a distribution whose weights are all zero, a negative
 *    or non-finite weight) are detected on the device, recorded in the
 *    forest's status word and reported by rtf_check.
 *  - Pointers to 64-bit element arrays must be 8-byte aligned, to 32-bit
 *    element arrays 4-byte aligned; workspaces 256-byte aligned.
 */
#ifndef RTFOREST_H
#define RTFOREST_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rtf_status {
    RTF_OK = 0,
    RTF_ERR_INVALID_ARG = 1, /* null or misaligned pointer, n < 1, m < 1, D < 1 */
    RTF_ERR_SIZE = 2,        /* a size beyond 2^31 - 1 (int32 leaf references) */
    RTF_ERR_WORKSPACE = 3,   /* workspace smaller than the *_workspace_bytes call */
    RTF_ERR_HIP = 4,         /* a HIP launch or runtime error */
    RTF_ERR_ZERO_TOTAL = 5,  /* a distribution whose weights sum to zero */
    RTF_ERR_VALUE = 6        /* rtf_quantize_f32: negative, NaN or infinite weight */
} rtf_status;

/*
 * Descriptor of a built forest.  Plain data: it holds pointers into the
 * caller's workspace and is valid while that workspace lives and is not used
 * for another build.
 *
 * Node array: n_total 16-byte records { uint64 key U_j; int32 child[2]; }
 * where node j splits between leaf j-1 and leaf j and compares against U_j
 * (Sec. 3.1).  A reference r >= 0 is a node, a reference r < 0 is leaf ~r.
 *
 * Guide table: m_total 64-byte cell records
 *   { uint64 k[7]; int32 ref; int32 aux; }.
 * ref is the guide entry of Sec. 2.5 and 3.2: the first node a of cell g
 * (whose child 1 roots the cell's tree and whose child 0 is the interval
 * overlapping the cell from the left) or, for a cell that no lower bound falls
 * in, the complement ~i of the one leaf covering it.  The keys repeat the
 * bounds a sample of the cell compares against, so that most samples need
 * this record only:
 *   ref = ~i:  k[0] = U_i, k[1] = U_{i+1}, aux = ref;
 *   ref = a, the cell holding c lower bounds U_a .. U_{a+c-1}:
 *     k[0] = U_{a-1} (0 at a distribution start), k[t] = U_{a+t-1} for
 *     t = 1 .. min(c+1, 6), so that k[c+1] = U_{a+c} is the upper end of the
 *     cell's last interval when c <= 5;
 *     c <= 5: aux = ~c and the sample is leaf a-1+j, j the number of
 *     k[1..c] at or below u;
 *     c > 5: aux = child 1 of node a (the cell tree's root); u < k[6] is
 *     resolved as above with j counted over k[1..5], a larger u descends
 *     the tree from aux.
 * Unused key slots hold 0.  A key of all ones stands for the end of the
 * distribution.
 */
typedef struct rtf_forest {
    int32_t D;          /* number of distributions */
    int32_t tile;       /* elements per build tile */
    int64_t n_total;    /* leaves = nodes over all distributions */
    int64_t m_total;    /* guide cells over all distributions */
    void *nodes;        /* device: n_total node records */
    void *cells;        /* device: m_total guide cell records */
    void *dists;        /* device: D per-distribution parameter records */
    int64_t *elem_off;  /* device: D+1 element offsets (copied at build) */
    int64_t *cell_off;  /* device: D+1 cell offsets (copied at build) */
    uint32_t *status;   /* device: status word (bit set per rtf_status code) */
    void *scratch;      /* device: build scratch */
    size_t scratch_bytes;
    void *wide;         /* device: collapsed nodes (rtf_forest_widen), or NULL */
} rtf_forest;

/* ---- workspace sizing ------------------------------------------------- */

/* Bytes of workspace for rtf_build of one distribution of n weights and m
 * guide cells; 0 if n or m is out of range. */
size_t rtf_workspace_bytes(int64_t n, int64_t m);

/* Bytes of workspace for rtf_build_batched of D distributions holding
 * n_total weights and m_total guide cells in all; 0 if out of range. */
size_t rtf_workspace_bytes_batched(int32_t D, int64_t n_total, int64_t m_total);

/* ---- construction (Sec. 3.1-3.2, Alg. 1; Sec. 5 for many at once) -------- */

/*
 * Build the guide table and radix tree forest of one distribution.
 *   w        uint32[n] weights (zeros allowed; not all zero)
 *   n        number of weights, 1 <= n <= 2^31 - 1
 *   m        number of guide cells, 1 <= m <= 2^31 - 1 (Sec. 3: "proportional
 *            to n" -- m = n is the usual choice)
 *   ws       workspace of at least rtf_workspace_bytes(n, m) bytes, 256-byte
 *            aligned; it holds the forest afterwards
 *   out      host pointer; receives the descriptor
 * The weights are read during the call's kernels only.  An all-zero w is
 * reported by rtf_check as RTF_ERR_ZERO_TOTAL; sampling it gives idx -1 and
 * x NaN.  Bit-exact and deterministic: the forest depends only on (w, m).
 */
rtf_status rtf_build(const uint32_t *w, int64_t n, int64_t m, void *ws,
                     size_t ws_bytes, hipStream_t stream, rtf_forest *out);

/*
 * Build the forests of D distributions stored back to back in one launch
 * sequence (Sec. 5: a distribution's index range is one more boundary that
 * merges never cross).
 *   w         uint32[n_total] weights, distribution d at [elem_off[d], elem_off[d+1])
 *   elem_off  int64[D+1] device offsets, elem_off[0] = 0, strictly increasing,
 *             elem_off[D] = n_total (every distribution has >= 1 weight)
 *   cell_off  int64[D+1] device offsets of the guide cells, cell_off[0] = 0,
 *             strictly increasing, cell_off[D] = m_total
 * Node and leaf references are global (leaf i of distribution d is
 * elem_off[d] + i); the sampling calls return indices local to d.  Offsets
 * are copied into the workspace.  They are not read back to the host, so
 * offsets that break the rules above are found on the device: rtf_check then
 * reports RTF_ERR_INVALID_ARG, the forest's contents are unspecified, and
 * the build and every later call on the forest stay within its workspace.
 */
rtf_status rtf_build_batched(const uint32_t *w, const int64_t *elem_off,
                             const int64_t *cell_off, int32_t D,
                             int64_t n_total, int64_t m_total, void *ws,
                             size_t ws_bytes, hipStream_t stream,
                             rtf_forest *out);

/*
 * rtf_build and rtf_build_batched with the build tile chosen by the caller
 * (Sec. 5 leaves the work split open; the autotuner picks it per workload):
 *   tile  elements per build tile, 1024 or 2048 (2048 is what rtf_build and
 *         rtf_build_batched use); anything else is RTF_ERR_INVALID_ARG
 * The forest is the same for either tile, bit for bit; only the speed
 * differs (1024-element tiles suit batches of many small distributions).
 * The workspace sizes above cover both tiles.  The descriptor's tile field
 * records the choice.
 */
rtf_status rtf_build_tiled(const uint32_t *w, int64_t n, int64_t m, int32_t tile,
                           void *ws, size_t ws_bytes, hipStream_t stream,
                           rtf_forest *out);
rtf_status rtf_build_batched_tiled(const uint32_t *w, const int64_t *elem_off,
                                   const int64_t *cell_off, int32_t D,
                                   int64_t n_total, int64_t m_total, int32_t tile,
                                   void *ws, size_t ws_bytes, hipStream_t stream,
                                   rtf_forest *out);

/* ---- collapsed nodes (Sec. 2.4 k-ary trees; Sec. 5) --------------------- */

/* Bytes of workspace for rtf_forest_widen of a forest with n_total nodes;
 * 0 if out of range. */
size_t rtf_wide_workspace_bytes(int64_t n_total);

/*
 * Collapse two binary levels of the descended trees into one 64-byte record
 * (a 4-ary tree, Sec. 5; memory transfer granularity, Sec. 2.4), so that a
 * sample past its cell record reads one record per two levels.  Records are
 * written for the internal nodes of every cell holding more than five lower
 * bounds (the cells whose samples descend), at the node's index:
 *   { uint64 k = U_j; uint64 kc[2]; int32 r[4]; 16 bytes unused }
 * For child c of node j on side s (0: u < U_j, 1: u >= U_j): when c is a node,
 * kc[s] = U_c and r[2s], r[2s+1] are c's children; when c is leaf ~i,
 * r[2s] = r[2s+1] = c and kc[s] = 0.
 *   f        a built forest (rtf_build / rtf_build_batched); on success its
 *            `wide` field points at ws and every later sampling call on f
 *            descends the collapsed records (same indices and positions)
 *   ws       rtf_wide_workspace_bytes(f->n_total) bytes, 256-byte aligned,
 *            owned by the caller; it must outlive the forest's use
 * Asynchronous on the stream, after the build in stream order.  A rebuild
 * into f's workspace clears f->wide (call rtf_forest_widen again).
 */
rtf_status rtf_forest_widen(rtf_forest *f, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---- depth fallback (Sec. 3) ------------------------------------------- */

/* Bytes of workspace for rtf_forest_balance of a forest with m_total guide
 * cells; 0 if out of range. */
size_t rtf_balance_workspace_bytes(int64_t m_total);

/*
 * The fallback of Sec. 3 for degenerate trees: the tree of a guide cell
 * holding c lower bounds (leaves a..a+c-1, child 1 of node a) is replaced
 * when a leaf with positive weight lies more than 2 ceil(log2 c) internal
 * nodes deep in it, by the balanced tree over the same leaves (the range
 * [lo, hi] splits at node ceil((lo + hi) / 2)).  Keys and guide entries stay,
 * so every search gives the same index as before; the cell record's aux
 * follows the new root.  With 64-bit keys a search never exceeds
 * 68 - floor(log2 m) reads (rtf_forest_depth), but a cell of geometrically
 * falling weights forms a comb as deep as its leaf count up to that bound;
 * after this call such a cell costs ceil(log2 c) + 2 reads.
 *   f          a built forest; its `wide` field is cleared (call
 *              rtf_forest_widen afterwards to collapse the new trees)
 *   ws         rtf_balance_workspace_bytes(f->m_total) bytes, 256-byte
 *              aligned (per-cell scratch, free after the call's kernels)
 *   h_rebuilt  host pointer receiving the number of cells rebuilt, or NULL;
 *              when given, the call synchronises the stream
 * Asynchronous otherwise, after the build in stream order.
 */
rtf_status rtf_forest_balance(rtf_forest *f, void *ws, size_t ws_bytes, int64_t *h_rebuilt,
                              hipStream_t stream);

/* ---- sampling (Alg. 2, Sec. 5) ---------------------------------------- */

/*
 * Alg. 2 for S uniforms of distribution 0 of f:
 *   u        uint64[S] uniforms (xi = u * 2^-64)
 *   out_idx  int32[S]: the i with P_i <= xi < P_{i+1}
 *   out_x    double[S] continuous position x, or NULL to skip it
 * S may be 0 (nothing is launched).
 */
rtf_status rtf_sample(const rtf_forest *f, const uint64_t *u, int64_t S,
                      int32_t *out_idx, double *out_x, hipStream_t stream);

/*
 * Alg. 2 for a batch: samples [sample_off[d], sample_off[d+1]) of u belong to
 * distribution d (int64[D+1] device offsets, non-decreasing, sample_off[D] = S;
 * empty ranges allowed).  Indices are local to each distribution.  Offsets
 * that break those rules (they are not read back to the host) give
 * unspecified indices, but every sample is still written once, the kernels
 * stay within the forest, u and the outputs, and they finish.
 */
rtf_status rtf_sample_batched(const rtf_forest *f, const int64_t *sample_off,
                              const uint64_t *u, int64_t S, int32_t *out_idx,
                              double *out_x, hipStream_t stream);

/*
 * Two-dimensional inversion (Sec. 5): distribution 0 of f is the marginal
 * over R rows and distributions 1..R are the rows (so D = R + 1 and the
 * marginal has R weights).  For pair s, u2[2s] picks the row r from the
 * marginal and u2[2s+1] the column c from row r.
 *   out_rc   int32[2S]: (r, c) per pair
 *   out_xy   double[2S]: (y, x) continuous positions of the row and the
 *            column, or NULL
 * u2 and out_xy must be 16-byte aligned and out_rc 8-byte aligned (pairs
 * move as vectors); otherwise RTF_ERR_INVALID_ARG.
 */
rtf_status rtf_sample_2d(const rtf_forest *f, const uint64_t *u2, int64_t S,
                         int32_t *out_rc, double *out_xy, hipStream_t stream);

/* Baseline of the same mapping by plain binary search over the forest's keys
 * (Sec. 2.2); identical output to rtf_sample (Sec. 4). */
rtf_status rtf_sample_bsearch(const rtf_forest *f, const uint64_t *u,
                              int64_t S, int32_t *out_idx, double *out_x,
                              hipStream_t stream);

/* Baseline of the same mapping by the guide table plus binary search inside
 * the cell (the Cutpoint Method with bisection, Sec. 2.5); identical output. */
rtf_status rtf_sample_cutpoint_bsearch(const rtf_forest *f, const uint64_t *u,
                                       int64_t S, int32_t *out_idx,
                                       double *out_x, hipStream_t stream);

/* ---- quantisation and differentiation (extensions) ---------------------- */

/*
 * Quantise non-negative float weights to uint32, per distribution:
 * s_d = (2^32-1) / max(v over d) in FP64, q = rint(v * s_d) clamped to
 * [1, 2^32-1] for v > 0, q = 0 for v == 0; scale[d] = s_d (0 if all zero).
 *   v         float[n_total]; elem_off int64[D+1] device offsets as in
 *             rtf_build_batched (NULL with D == 1 means [0, n_total])
 *   out       uint32[n_total]; scale double[D]
 *   status    uint32 device status word that receives RTF_ERR_VALUE for a
 *             negative, NaN or infinite weight (may be NULL)
 * Offsets that break those rules (they are not read back to the host) give
 * unspecified q and scale, but the kernels stay within v, out, scale and
 * elem_off and finish.
 */
rtf_status rtf_quantize_f32(const float *v, const int64_t *elem_off, int32_t D,
                            int64_t n_total, uint32_t *out, double *scale,
                            uint32_t *status, hipStream_t stream);

/* Bytes of workspace rtf_backward needs for a forest of D distributions and
 * n_total weights. */
size_t rtf_backward_workspace_bytes(int32_t D, int64_t n_total);

/*
 * Adjoint of x with respect to the real weights v = q / scale (the sampled
 * index is piecewise constant and held fixed).  For distribution d with n_d
 * weights and a_s = grad_x[s] / (n_d * w_{i_s}):
 *   grad_w[k] = sum_s a_s xi_s - sum_{s: i_s > k} a_s - sum_{s: i_s = k} a_s frac_s
 * over the samples s of d, where frac_s = x_s * n_d - i_s.
 *   sample_off int64[D+1] as in rtf_sample_batched (NULL with D == 1)
 *   u, idx     the forward call's uniforms and local indices
 *   grad_x     double[S]; scale double[D] from rtf_quantize_f32
 *   grad_w     double[n_total] (written, not accumulated)
 *   ws         rtf_backward_workspace_bytes(D, n_total) bytes, 256-aligned
 * Samples with idx < 0 are ignored.
 */
rtf_status rtf_backward(const rtf_forest *f, const int64_t *sample_off,
                        const uint64_t *u, const int32_t *idx,
                        const double *grad_x, int64_t S, const double *scale,
                        double *grad_w, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/*
 * rtf_backward with its scratch in a fixed device array of the library
 * instead of a caller workspace.  For callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the call allocates and frees nothing, on the device or
 * through any allocating library routine.  Arguments, results and errors are
 * those of rtf_backward, less the workspace, plus:
 *   RTF_ERR_SIZE  f->n_total > RTF_BACKWARD_STATIC_MAX_N or
 *                 f->D > RTF_BACKWARD_STATIC_MAX_D (nothing is enqueued)
 *   RTF_ERR_HIP   the array's device address could not be obtained
 * Each GPU holds one copy of the array (about 16.5 MiB at these limits) from
 * the first call on it until the process ends.  Every call on one GPU uses
 * that same copy, and the pass clears what it accumulates before use, so
 * calls in stream order are independent; calls that overlap on one GPU (on
 * different streams, or from several threads without ordering) race on it
 * and give undefined results.
 */
#define RTF_BACKWARD_STATIC_MAX_N (1 << 20)
#define RTF_BACKWARD_STATIC_MAX_D (1 << 16)
rtf_status rtf_backward_static(const rtf_forest *f, const int64_t *sample_off,
                               const uint64_t *u, const int32_t *idx,
                               const double *grad_x, int64_t S,
                               const double *scale, double *grad_w,
                               hipStream_t stream);

/* ---- the Alias Method: the non-monotone comparison mapping (Sec. 2.6) ---- */

/*
 * Walker's alias table (Sec. 2.6, Fig. alias_map), the mapping the paper's
 * quality study compares the inverse against (Figs. results_sine64, 2d_zoom,
 * convergence).  It maps uniforms to the same distribution, but not
 * monotonically, so it does not preserve the uniformity of a low-discrepancy
 * sequence.  Exact integers: item i of a distribution of n weights carries
 * the mass w_i n, each of the n cells holds W = sum w.  Record j is
 * { uint64 thr_j; int32 alias_j; int32 unused; }: item j keeps the part thr_j
 * of cell j, alias_j the rest.  Built by Vose's two-worklist method in a
 * fixed order (small items, of mass below W, and large ones on two stacks in
 * increasing index order; each step pairs the top of both and pushes the
 * large item back by its remaining mass), serial per distribution as the
 * paper notes known setups are.
 */
typedef struct rtf_alias_table {
    int32_t D;
    int64_t n_total;
    void *recs;         /* device: n_total 16-byte records */
    uint64_t *W;        /* device: D totals */
    int64_t *elem_off;  /* device: D+1 offsets (copied at build) */
    uint32_t *status;   /* device: status word */
} rtf_alias_table;

/* Bytes of workspace for rtf_alias_build; 0 if out of range. */
size_t rtf_alias_workspace_bytes(int32_t D, int64_t n_total);

/*
 * Build the alias tables of D distributions stored back to back.
 *   w         uint32[n_total] weights; elem_off int64[D+1] device offsets as
 *             in rtf_build_batched (NULL with D == 1)
 *   ws        rtf_alias_workspace_bytes(D, n_total) bytes, 256-byte aligned;
 *             it holds the tables afterwards
 * One thread per distribution runs the serial setup, so a distribution of n
 * items costs n dependent steps on one thread: the call suits many small or
 * medium tables (the rows of a 2D map), not one table of millions of items.
 * A distribution with W = 0 is reported by rtf_alias_export as
 * RTF_ERR_ZERO_TOTAL and samples to -1.
 */
rtf_status rtf_alias_build(const uint32_t *w, const int64_t *elem_off, int32_t D,
                           int64_t n_total, void *ws, size_t ws_bytes,
                           hipStream_t stream, rtf_alias_table *out);

/*
 * Sample: xi = u 2^-64 lies in cell j = floor(u n / 2^64) at the offset
 * r = u n mod 2^64; the item is j if floor(r W / 2^64) < thr_j, else
 * alias_j (an exact test).  sample_off int64[D+1] as in rtf_sample_batched
 * (NULL with D == 1); indices are local to each distribution.
 */
rtf_status rtf_alias_sample(const rtf_alias_table *t, const int64_t *sample_off,
                            const uint64_t *u, int64_t S, int32_t *out_idx,
                            hipStream_t stream);

/* Pairs as rtf_sample_2d: table 0 is the marginal over R = D - 1 rows,
 * table r + 1 is row r; u2[2s] picks the row, u2[2s+1] the column.  u2 must
 * be 16-byte and out_rc 8-byte aligned.  A pair whose row has no table (a
 * marginal with more than D - 1 items) gets (-1, -1). */
rtf_status rtf_alias_sample_2d(const rtf_alias_table *t, const uint64_t *u2, int64_t S,
                               int32_t *out_rc, hipStream_t stream);

/* Synchronise and copy the tables to host buffers (each may be NULL):
 * h_thr uint64[n_total], h_alias int32[n_total] (local indices), h_W
 * uint64[D]; returns the first error the build recorded. */
rtf_status rtf_alias_export(const rtf_alias_table *t, uint64_t *h_thr, int32_t *h_alias,
                            uint64_t *h_W, hipStream_t stream);

/* ---- inspection --------------------------------------------------------- */

/* Synchronise the stream and return the first error recorded in the forest's
 * status word (RTF_OK if none). */
rtf_status rtf_check(const rtf_forest *f, hipStream_t stream);

/* Synchronise and copy the forest to host buffers (each may be NULL):
 * h_nodes receives the n_total 16-byte node records as stored, h_cells the
 * m_total 64-byte guide cell records as stored, h_W uint64[D] the
 * distributions' total weights. */
rtf_status rtf_forest_export(const rtf_forest *f, void *h_nodes, void *h_cells,
                             uint64_t *h_W, hipStream_t stream);

/*
 * The inverse of rtf_forest_export, for tests: a forest built elsewhere (for
 * instance by a CPU reference) is copied into a workspace so that the
 * sampling and backward calls can run on it.
 *   h_nodes     host: n_total 16-byte node records, as rtf_forest_export gives
 *   h_cells     host: m_total 64-byte guide cell records, as rtf_forest_export
 *               gives (keys and aux must follow the record layout above)
 *   h_W         host: uint64[D] totals
 *   h_elem_off, h_cell_off  host: int64[D+1] offsets as in rtf_build_batched
 *               (NULL with D == 1)
 *   ws          rtf_workspace_bytes_batched(D, n_total, m_total) bytes,
 *               256-byte aligned (rtf_workspace_bytes(n, m) with D == 1)
 * The per-distribution parameters are derived from the totals as the build
 * derives them.  Offsets that are not strictly increasing from 0 to n_total
 * (m_total) give RTF_ERR_INVALID_ARG.  Synchronises the stream.  The records
 * are not checked: a forest that breaks the layout samples undefined values
 * (but a reference outside the forest yields index -1, not a fault).
 */
rtf_status rtf_forest_import(const void *h_nodes, const void *h_cells, const uint64_t *h_W,
                             const int64_t *h_elem_off, const int64_t *h_cell_off, int32_t D,
                             int64_t n_total, int64_t m_total, void *ws, size_t ws_bytes,
                             hipStream_t stream, rtf_forest *out);

/*
 * The deepest search of the forest, counted as Alg. 2 counts memory reads:
 * the guide entry plus the nodes visited down to the leaf, maximised over
 * every uniform (over the leaves with positive weight, each from the cell
 * holding its lower bound).  Written to the forest's status block and to
 * *h_depth (host); synchronises the stream.  One distribution's bound: the
 * keys of a cell differ below bit 65 - floor(log2 m) and the levels fall
 * strictly along a path through distinct keys, while a run of zero weights
 * (equal keys) is left at its first node, so the depth never exceeds
 * 68 - floor(log2 m) whatever the weights -- the degenerate O(n) trees of
 * Sec. 3 cannot be reached by a search here (the chains that zero runs form
 * exist but no uniform descends them).
 */
rtf_status rtf_forest_depth(const rtf_forest *f, int32_t *h_depth, hipStream_t stream);

/* Static string naming a status code. */
const char *rtf_status_string(rtf_status s);

#ifdef __cplusplus
}
#endif

#endif /* RTFOREST_H */
