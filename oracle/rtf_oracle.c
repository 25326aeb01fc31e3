/*
 * rtf_oracle.c -- CPU oracle for radix-tree-forest inverse-CDF sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference against which the HIP library is checked.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * Source: Binder & Keller, "Massively Parallel Construction of Radix Tree
 * Forests for the Efficient Sampling of Discrete or Piecewise Constant
 * Probability Distributions" (arXiv:1901.05423).  Each function names the
 * passage it follows.
 *
 * Number formats (the paper works in [0,1) floats; we fix exact integers):
 *   w_i  uint32 weights, C_i = sum_{k<i} w_k (uint64), W = C_n.
 *   u    uint64, standing for xi = u * 2^-64 in [0,1).
 *   U_i  = ceil(C_i * 2^64 / W), the 0.64 fixed-point lower bound of
 *        interval i, so that  U_i <= u  <=>  C_i <= floor(u*W / 2^64).
 *   Leaf references are bitwise complements ~i (MSB set); node references
 *   are non-negative node indices.
 *
 * Pins (tests/): brute-force linear search, monotonicity, closed forms for
 * equal weights and regular grids, the worked forest figure, the printed
 * sine^2 histograms, Algorithm 1 under random schedules, finite differences,
 * a hand-built balanced tree for the depth fallback.
 * No function here is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_ZERO_TOTAL 2
#define ORC_ERR_VALUE 3

#define SENT 65 /* "distance = maximum": above any real level 0..64 */

/* ------------------------------------------------------------------------ */
/* Quantisation of non-negative real weights to uint32 (not in the paper;   */
/* the paper assumes given p_i > 0, Sec. 1).  Rule: s = (2^32-1)/max v in   */
/* FP64, q = rint(v*s) clamped to [1, 2^32-1] for v > 0, q = 0 for v == 0.  */
/* Returns ORC_ERR_VALUE for negative, NaN or infinite input.               */
/* ------------------------------------------------------------------------ */
int oracle_quantize(const float *v, int64_t n, uint32_t *q, double *scale)
{
    float mx = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        if (!(v[i] >= 0.0f) || isinf(v[i]))
            return ORC_ERR_VALUE;
        if (v[i] > mx)
            mx = v[i];
    }
    if (mx == 0.0f) {
        for (int64_t i = 0; i < n; ++i)
            q[i] = 0;
        *scale = 0.0;
        return ORC_OK;
    }
    double s = 4294967295.0 / (double)mx;
    for (int64_t i = 0; i < n; ++i) {
        if (v[i] == 0.0f) {
            q[i] = 0;
            continue;
        }
        double y = rint((double)v[i] * s);
        if (y < 1.0)
            y = 1.0;
        if (y > 4294967295.0)
            y = 4294967295.0;
        q[i] = (uint32_t)y;
    }
    *scale = s;
    return ORC_OK;
}

/* Partial sums P_k of Sec. 1, in integers: C[0] = 0, C[i+1] = C[i] + w[i]. */
void oracle_prefix(const uint32_t *w, int64_t n, uint64_t *C)
{
    C[0] = 0;
    for (int64_t i = 0; i < n; ++i)
        C[i + 1] = C[i] + (uint64_t)w[i];
}

/* floor(u*W / 2^64) and the low 64 bits of u*W. */
static void mul_split(uint64_t u, uint64_t W, uint64_t *t, uint64_t *lo)
{
    u128 p = (u128)u * (u128)W;
    *t = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Continuous position inside the sampled interval, rescaled to [0,1]
 * (Sec. 5, sub-pixel position): x = (i + ((t - C_i) + lo*2^-64) / w_i) / n. */
static double position(int64_t i, int64_t n, uint64_t t, uint64_t lo,
                       uint64_t Ci, uint64_t wi)
{
    double frac = ((double)(t - Ci) + ldexp((double)lo, -64)) / (double)wi;
    return ((double)i + frac) / (double)n;
}

/*
 * Inverse CDF by binary search (Sec. 2.2) on the integer partial sums:
 * idx[s] = the i with C_i <= t < C_{i+1}, t = floor(u*W/2^64), i.e. the
 * 0-based form of P_{i-1} <= xi < P_i (Sec. 1).  x (nullable) as above.
 * C has n+1 entries.  W == 0 gives idx = -1, x = NaN and ORC_ERR_ZERO_TOTAL.
 */
int oracle_search(const uint64_t *C, int64_t n, const uint64_t *u, int64_t S,
                  int32_t *idx, double *x)
{
    uint64_t W = C[n];
    if (W == 0) {
        for (int64_t s = 0; s < S; ++s) {
            idx[s] = -1;
            if (x)
                x[s] = NAN;
        }
        return ORC_ERR_ZERO_TOTAL;
    }
    for (int64_t s = 0; s < S; ++s) {
        uint64_t t, lo;
        mul_split(u[s], W, &t, &lo);
        /* largest i in [0, n) with C[i] <= t; C[0] = 0 <= t < W = C[n] */
        int64_t a = 0, b = n; /* invariant: C[a] <= t < C[b] */
        while (b - a > 1) {
            int64_t mid = a + (b - a) / 2;
            if (C[mid] <= t)
                a = mid;
            else
                b = mid;
        }
        idx[s] = (int32_t)a;
        if (x)
            x[s] = position(a, n, t, lo, C[a], C[a + 1] - C[a]);
    }
    return ORC_OK;
}

/* Linear search (Sec. 2.1): scan intervals in order until one holds xi. */
int oracle_linear_search(const uint64_t *C, int64_t n, const uint64_t *u,
                         int64_t S, int32_t *idx)
{
    uint64_t W = C[n];
    if (W == 0)
        return ORC_ERR_ZERO_TOTAL;
    for (int64_t s = 0; s < S; ++s) {
        uint64_t t, lo;
        mul_split(u[s], W, &t, &lo);
        int64_t i = 0;
        while (!(C[i] <= t && t < C[i + 1]))
            ++i;
        idx[s] = (int32_t)i;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Radix tree forest: reference construction from the definition.          */
/* ------------------------------------------------------------------------ */

/* Fixed-point lower bounds, trailing zero-weight leaves get UINT64_MAX. */
static void lower_bounds(const uint64_t *C, int64_t n, int64_t n_eff,
                         uint64_t *key)
{
    uint64_t W = C[n];
    for (int64_t i = 0; i < n; ++i) {
        if (i < n_eff)
            key[i] = (uint64_t)((((u128)C[i] << 64) + (u128)(W - 1)) / (u128)W);
        else
            key[i] = UINT64_MAX;
    }
}

/* Guide-table cell of a lower bound: floor(U * m / 2^64) (Alg. 1, cell). */
static int64_t cell_of(uint64_t U, int64_t m)
{
    return (int64_t)(((u128)U * (u128)(uint64_t)m) >> 64);
}

/* Level of the boundary between leaf b and b+1: the position of the most
 * significant differing bit, 64 - clz(U_b ^ U_{b+1}) (Sec. 3.1), or SENT where
 * a merge must not cross (a cell change, Sec. 3.2; the end of the weights
 * that carry mass).  Boundaries -1 and n-1 are SENT as well. */
static int level_at(const uint64_t *key, const int64_t *cell, int64_t n_eff,
                    int64_t b)
{
    if (b < 0 || b + 1 >= n_eff)
        return SENT;
    if (cell[b] != cell[b + 1])
        return SENT;
    uint64_t d = key[b] ^ key[b + 1];
    int l = 0;
    while (d) {
        ++l;
        d >>= 1;
    }
    return l;
}

/*
 * One distribution of n weights, with its leaves at global index eo and its
 * guide cells at global index co (m cells).  Writes key[eo..eo+n),
 * child[2*(eo..eo+n)], table[co..co+m) with global references.
 *
 * Tree definition (Sec. 3.1, Fig. radix_forest): node j splits between leaf
 * j-1 and leaf j and compares against U_j.  Within one cell's run of leaves
 * [a,b], the root is the boundary k in [a,b) of highest level, the rightmost
 * one among equal levels; it becomes node k+1 with left subtree [a,k] and right
 * subtree [k+1,b].  The cell's tree hangs as child 1 of node a; child 0 of
 * node a is set to the interval on its left, or to leaf a itself at the start
 * of a distribution (Fig. radix_forest caption).
 *
 * Guide table (Sec. 2.5 and the remark on complemented references in Sec.
 * 3.2): cell g holds node a when a is the first leaf whose lower bound falls
 * in g; a cell that no lower bound falls in is covered by one interval only,
 * the one to its left, and holds that leaf's complement.
 */
static int forest_one(const uint32_t *w, int64_t n, int64_t m, int64_t eo,
                      int64_t co, uint64_t *key_g, int32_t *child_g,
                      int32_t *table_g, uint64_t *W_out)
{
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n + 1));
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *stk = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)(n + 1));
    if (!C || !cell || !stk) {
        free(C);
        free(cell);
        free(stk);
        return ORC_ERR_ARG;
    }
    oracle_prefix(w, n, C);
    uint64_t W = C[n];
    *W_out = W;
    if (W == 0) {
        free(C);
        free(cell);
        free(stk);
        return ORC_ERR_ZERO_TOTAL;
    }
    int64_t n_eff = n;
    while (w[n_eff - 1] == 0)
        --n_eff;

    uint64_t *key = key_g + eo;
    int32_t *child = child_g + 2 * eo;
    int32_t *table = table_g + co;
    lower_bounds(C, n, n_eff, key);
    for (int64_t i = 0; i < n_eff; ++i)
        cell[i] = cell_of(key[i], m);

    /* leaves past the last positive weight are never part of a tree */
    for (int64_t j = n_eff; j < n; ++j) {
        child[2 * j + 0] = ~(int32_t)(eo + j);
        child[2 * j + 1] = ~(int32_t)(eo + j);
    }

    int64_t a = 0;
    while (a < n_eff) {
        int64_t b = a;
        while (b + 1 < n_eff && cell[b + 1] == cell[a])
            ++b;
        /* pseudo-root a */
        child[2 * a + 0] = (a == 0) ? ~(int32_t)(eo + a) : ~(int32_t)(eo + a - 1);
        /* recursive split of [a,b] with an explicit stack of
         * (lo, hi, slot) where slot is the child slot to fill */
        int64_t sp = 0;
        stk[sp++] = a;
        stk[sp++] = b;
        stk[sp++] = 2 * a + 1;
        while (sp > 0) {
            int64_t slot = stk[--sp];
            int64_t hi = stk[--sp];
            int64_t lo = stk[--sp];
            if (lo == hi) {
                child[slot] = ~(int32_t)(eo + lo);
                continue;
            }
            int64_t kbest = lo;
            int lbest = level_at(key, cell, n_eff, lo);
            for (int64_t k = lo + 1; k < hi; ++k) {
                int l = level_at(key, cell, n_eff, k);
                if (l >= lbest) { /* ties: the rightmost boundary */
                    lbest = l;
                    kbest = k;
                }
            }
            child[slot] = (int32_t)(eo + kbest + 1);
            stk[sp++] = lo;
            stk[sp++] = kbest;
            stk[sp++] = 2 * (kbest + 1) + 0;
            stk[sp++] = kbest + 1;
            stk[sp++] = hi;
            stk[sp++] = 2 * (kbest + 1) + 1;
        }
        a = b + 1;
    }

    /* guide table: first leaf whose cell is >= g */
    int64_t p = 0;
    for (int64_t g = 0; g < m; ++g) {
        while (p < n_eff && cell[p] < g)
            ++p;
        if (p < n_eff && cell[p] == g)
            table[g] = (int32_t)(eo + p);
        else
            table[g] = ~(int32_t)(eo + p - 1);
    }
    free(C);
    free(cell);
    free(stk);
    return ORC_OK;
}

/*
 * Forest over D distributions stored back to back (Sec. 5: building many
 * tables and trees at once treats each distribution's index range as one
 * more boundary).  elem_off and cell_off hold D+1 offsets each.  key[n_total],
 * child[2*n_total], table[m_total], W[D].  Returns the first error met;
 * a distribution with W == 0 leaves its outputs untouched.
 */
int oracle_forest(const uint32_t *w, const int64_t *elem_off,
                  const int64_t *cell_off, int32_t D, uint64_t *key,
                  int32_t *child, int32_t *table, uint64_t *W)
{
    int rc = ORC_OK;
    for (int32_t d = 0; d < D; ++d) {
        int64_t eo = elem_off[d], n = elem_off[d + 1] - eo;
        int64_t co = cell_off[d], m = cell_off[d + 1] - co;
        if (n < 1 || m < 1)
            return ORC_ERR_ARG;
        int r = forest_one(w + eo, n, m, eo, co, key, child, table, &W[d]);
        if (r != ORC_OK && rc == ORC_OK)
            rc = r;
    }
    return rc;
}

/*
 * Alg. 2: guide lookup g = floor(xi*m), then descend while the reference is a
 * node, going to child 0 when xi < U_j and to child 1 otherwise; the leaf is
 * the complement of the final reference.  For distribution d the cell is
 * cell_off[d] + floor(u*m_d/2^64) and the returned index is local to d.
 */
void oracle_descend(const uint64_t *key, const int32_t *child,
                    const int32_t *table, int64_t eo, int64_t co, int64_t m,
                    const uint64_t *u, int64_t S, int32_t *idx)
{
    for (int64_t s = 0; s < S; ++s) {
        int32_t j = table[co + cell_of(u[s], m)];
        while (j >= 0)
            j = (u[s] < key[j]) ? child[2 * (int64_t)j + 0]
                                : child[2 * (int64_t)j + 1];
        idx[s] = (int32_t)((int64_t)(~j) - eo);
    }
}

/*
 * Depth fallback (Sec. 3: a degenerate tree would cost O(n) per search, so a
 * fallback builds a structure with logarithmic depth when one is detected).
 * Reading: the tree of a guide cell holding c lower bounds (leaves a..a+c-1,
 * hung as child 1 of node a) is degenerate when some leaf with positive
 * weight lies more than 2 ceil(log2 c) internal nodes below that tree's root,
 * i.e. when Alg. 2, entering at node a, visits more than 1 + 2 ceil(log2 c)
 * nodes for it.  Such a tree is replaced by the balanced one over the same
 * leaves: split(lo, hi) is leaf ~lo when lo == hi, else node mid with
 * mid = ceil((lo + hi) / 2), left subtree split(lo, mid-1) and right
 * subtree split(mid, hi).  Every node keeps its key U_j and still splits
 * between leaf j-1 and j, so any search gives the index binary search gives.
 * Works in place on a forest from oracle_forest; *rebuilt receives the number
 * of cells replaced.
 */
static int ceil_log2(int64_t c)
{
    int l = 0;
    while (((int64_t)1 << l) < c)
        ++l;
    return l;
}

static int32_t balanced_split(int32_t *child, int64_t lo, int64_t hi)
{
    if (lo == hi)
        return ~(int32_t)lo;
    int64_t mid = (lo + hi + 1) / 2;
    child[2 * mid + 0] = balanced_split(child, lo, mid - 1);
    child[2 * mid + 1] = balanced_split(child, mid, hi);
    return (int32_t)mid;
}

int oracle_balance(const int64_t *elem_off, const int64_t *cell_off, int32_t D,
                   const uint64_t *key, int32_t *child, const int32_t *table,
                   int64_t *rebuilt)
{
    int64_t count = 0;
    for (int32_t d = 0; d < D; ++d) {
        int64_t end = elem_off[d + 1];
        int64_t co = cell_off[d], m = cell_off[d + 1] - co;
        for (int64_t g = 0; g < m; ++g) {
            int64_t a = table[co + g];
            if (a < 0)
                continue; /* covered by one interval: no tree */
            int64_t b = a; /* last leaf whose lower bound lies in cell g */
            while (b + 1 < end && key[b + 1] != UINT64_MAX && cell_of(key[b + 1], m) == g)
                ++b;
            int64_t c = b - a + 1;
            int64_t deepest = 0; /* nodes Alg. 2 visits from node a */
            for (int64_t i = a; i <= b; ++i) {
                int live = (i + 1 == end) || key[i + 1] == UINT64_MAX || key[i + 1] != key[i];
                if (!live)
                    continue; /* zero weight: no uniform reaches it */
                int64_t visits = 0;
                int32_t j = (int32_t)a;
                while (j >= 0) {
                    ++visits;
                    j = key[i] < key[j] ? child[2 * (int64_t)j] : child[2 * (int64_t)j + 1];
                }
                if (visits > deepest)
                    deepest = visits;
            }
            if (deepest - 1 > 2 * ceil_log2(c)) {
                child[2 * a + 1] = balanced_split(child, a, b);
                ++count;
            }
        }
    }
    *rebuilt = count;
    return ORC_OK;
}

/* Levels of all boundaries of one distribution (for tests): lvl[b] for
 * b in [0, n-1), the level between leaf b and b+1. */
int oracle_levels(const uint32_t *w, int64_t n, int64_t m, int32_t *lvl)
{
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n + 1));
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    oracle_prefix(w, n, C);
    if (C[n] == 0) {
        free(C);
        free(key);
        free(cell);
        return ORC_ERR_ZERO_TOTAL;
    }
    int64_t n_eff = n;
    while (w[n_eff - 1] == 0)
        --n_eff;
    lower_bounds(C, n, n_eff, key);
    for (int64_t i = 0; i < n_eff; ++i)
        cell[i] = cell_of(key[i], m);
    for (int64_t b = 0; b + 1 < n; ++b)
        lvl[b] = level_at(key, cell, n_eff, b);
    free(C);
    free(key);
    free(cell);
    return ORC_OK;
}

/*
 * Alg. 1 run as written, one distribution, as a serial simulation of its
 * parallel threads: a thread per leaf that carries mass, and at every step a
 * runnable thread picked by a caller-seeded xorshift generator executes one
 * pass of the merge loop.  The distance comparison uses the levels above
 * (highest differing bit; SENT at cell changes, both array ends and after
 * the last positive weight), with ties taking the "otherwise" branch.  The
 * atomic exchange on otherBounds is the only shared read-modify-write, so
 * interleaving whole loop passes covers every outcome the algorithm can
 * have.  Child 0 of every cell's first node is then set by hand as in the
 * caption of Fig. radix_forest.  Output layout as oracle_forest (eo=co=0);
 * the guide table is not written.
 */
int oracle_alg1(const uint32_t *w, int64_t n, int64_t m, uint64_t seed,
                uint64_t *key, int32_t *child)
{
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n + 1));
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int *lvl = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int64_t *other = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *r0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *r1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *node = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *run = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    oracle_prefix(w, n, C);
    int rc = ORC_OK;
    if (C[n] == 0) {
        rc = ORC_ERR_ZERO_TOTAL;
        goto done;
    }
    int64_t n_eff = n;
    while (w[n_eff - 1] == 0)
        --n_eff;
    lower_bounds(C, n, n_eff, key);
    for (int64_t i = 0; i < n_eff; ++i)
        cell[i] = cell_of(key[i], m);
    /* lvl[b+1] is the level between leaf b and b+1, b in [-1, n) */
    for (int64_t b = -1; b < n; ++b)
        lvl[b + 1] = (b == n - 1) ? SENT : level_at(key, cell, n_eff, b);
    for (int64_t i = 0; i < n; ++i) {
        other[i] = -1;
        child[2 * i] = child[2 * i + 1] = 0x7fffffff; /* "unset" */
    }
    int64_t nrun = 0;
    for (int64_t i = 0; i < n_eff; ++i) {
        r0[i] = r1[i] = i;
        node[i] = ~i;
        run[nrun++] = i;
    }
    uint64_t z = seed ? seed : 0x9e3779b97f4a7c15ull;
    while (nrun > 0) {
        z ^= z << 13;
        z ^= z >> 7;
        z ^= z << 17;
        int64_t pick = (int64_t)(z % (uint64_t)nrun);
        int64_t th = run[pick];
        int low = lvl[r0[th]];      /* boundary r0-1 | r0 */
        int high = lvl[r1[th] + 1]; /* boundary r1 | r1+1 */
        int c = (low > high) ? 0 : 1;
        int64_t parent = (c == 0) ? r1[th] + 1 : r0[th];
        int64_t mine = (c == 0) ? r0[th] : r1[th]; /* range[child] */
        child[2 * parent + c] = (int32_t)node[th];
        int64_t ob = other[parent];
        other[parent] = mine; /* atomicExch */
        if (ob != -1) { /* range[1 - child] <- the sibling's far end */
            if (c == 0)
                r1[th] = ob;
            else
                r0[th] = ob;
            node[th] = parent;
        } else {
            run[pick] = run[--nrun];
        }
    }
    for (int64_t a = 0; a < n_eff; ++a)
        if (lvl[a] == SENT) /* boundary a-1 | a: a cell starts at a */
            child[2 * a + 0] = (a == 0) ? ~(int32_t)0 : ~(int32_t)(a - 1);
    for (int64_t j = n_eff; j < n; ++j)
        child[2 * j + 0] = child[2 * j + 1] = ~(int32_t)j;
done:
    free(C);
    free(cell);
    free(lvl);
    free(other);
    free(r0);
    free(r1);
    free(node);
    free(run);
    return rc;
}

/*
 * Reference gradient of x with respect to the real weights v of one
 * distribution, the sampled index held fixed (it is piecewise constant).
 * With w_k = q_k / scale, xi = u*2^-64, frac as in position() and
 * a_s = g_s / (n * w_{i_s}):
 *   dL/dv_k = sum_s a_s * (xi_s - [k < i_s] - [k == i_s] * frac_s)
 *           = A - sum_{j > k} B_j - D_k,
 *   A = sum_s a_s xi_s,  B_j = sum_{i_s = j} a_s,  D_j = sum_{i_s = j} a_s frac_s.
 * Derived from x = (i + (xi*W - C_i)/w_i)/n (Sec. 5, sub-pixel position).
 */
int oracle_grad(const uint32_t *q, int64_t n, double scale, const uint64_t *u,
                const double *g, int64_t S, double *grad)
{
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n + 1));
    double *B = (double *)calloc((size_t)n, sizeof(double));
    double *Dv = (double *)calloc((size_t)n, sizeof(double));
    oracle_prefix(q, n, C);
    uint64_t W = C[n];
    if (W == 0 || !(scale > 0.0)) {
        free(C);
        free(B);
        free(Dv);
        return ORC_ERR_ZERO_TOTAL;
    }
    double A = 0.0;
    for (int64_t s = 0; s < S; ++s) {
        int32_t i;
        double xs;
        oracle_search(C, n, &u[s], 1, &i, &xs);
        uint64_t t, lo;
        mul_split(u[s], W, &t, &lo);
        uint64_t wi = C[i + 1] - C[i];
        double frac = ((double)(t - C[i]) + ldexp((double)lo, -64)) / (double)wi;
        double xi = ldexp((double)u[s], -64);
        double a = g[s] / ((double)n * ((double)wi / scale));
        A += a * xi;
        B[i] += a;
        Dv[i] += a * frac;
    }
    double suffix = 0.0; /* sum_{j > k} B_j */
    for (int64_t k = n - 1; k >= 0; --k) {
        grad[k] = A - suffix - Dv[k];
        suffix += B[k];
    }
    free(C);
    free(B);
    free(Dv);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The Alias Method (Sec. 2.6 "The Alias Method", Fig. alias_map: Walker's  */
/* table of cells holding at most two intervals, the cell's own and one     */
/* alias), built by the two-worklist construction of Vose (IEEE TSE 1991)   */
/* in exact integers.  The comparison mapping of the paper's quality study  */
/* (Figs. results_sine64, 2d_zoom, convergence); it is not monotone.        */
/*                                                                          */
/* Units: item i carries a_i = w_i * n, a cell holds W = sum w, so the n    */
/* cells hold exactly the total mass.  thr[j] in [0, W] is the part of cell */
/* j kept by item j; the rest, W - thr[j], belongs to alias[j].             */
/* Order (fixed so that any implementation can reproduce the table): the    */
/* items with a_i < W ("small") and a_i >= W ("large") are pushed onto two  */
/* stacks in increasing index order; each step pops the top of both, gives  */
/* the small item's cell its remainder to the large item, and pushes the    */
/* large item back onto the stack its remaining mass now belongs to.  With  */
/* exact integers the stacks run empty together, or the large one is left   */
/* holding items of mass exactly W (their cells keep all of it).            */
/* work: 2n int64 entries of scratch.  Returns ORC_ERR_ZERO_TOTAL if W = 0. */
/* ------------------------------------------------------------------------ */
int oracle_alias_build(const uint32_t *w, int64_t n, uint64_t *thr, int32_t *alias,
                       int64_t *work)
{
    if (n < 1)
        return ORC_ERR_ARG;
    uint64_t W = 0;
    for (int64_t i = 0; i < n; ++i)
        W += w[i];
    if (W == 0)
        return ORC_ERR_ZERO_TOTAL;
    int64_t *small = work, *large = work + n;
    int64_t ns = 0, nl = 0;
    for (int64_t i = 0; i < n; ++i) {
        thr[i] = (uint64_t)w[i] * (uint64_t)n; /* the mass still to place */
        alias[i] = (int32_t)i;
        if (thr[i] < W)
            small[ns++] = i;
        else
            large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        int64_t s = small[--ns], l = large[--nl];
        alias[s] = (int32_t)l;                 /* thr[s] = a_s stays */
        thr[l] -= W - thr[s];                  /* >= a_s >= 0 since a_l >= W */
        if (thr[l] < W)
            small[ns++] = l;
        else
            large[nl++] = l;
    }
    while (nl > 0) { /* mass exactly W: the cell is the item's own */
        int64_t l = large[--nl];
        thr[l] = W;
        alias[l] = (int32_t)l;
    }
    if (ns > 0) /* impossible with exact sums */
        return ORC_ERR_ARG;
    return ORC_OK;
}

/* Sample the alias table: xi = u 2^-64 falls in cell j = floor(xi n) at
 * relative position f = xi n - j; the item is j when f < thr[j] / W, else
 * alias[j].  In integers: j:r = u * n (high:low 64 bits), f = r 2^-64, and
 * f < thr/W  <=>  r W < thr 2^64  <=>  floor(r W / 2^64) < thr (thr is an
 * integer), so the test is exact. */
void oracle_alias_sample(const uint64_t *thr, const int32_t *alias, int64_t n, uint64_t W,
                         const uint64_t *u, int64_t S, int32_t *idx)
{
    for (int64_t s = 0; s < S; ++s) {
        u128 p = (u128)u[s] * (u128)(uint64_t)n;
        int64_t j = (int64_t)(p >> 64);
        uint64_t r = (uint64_t)p;
        uint64_t t = (uint64_t)(((u128)r * (u128)W) >> 64);
        idx[s] = t < thr[j] ? (int32_t)j : alias[j];
    }
}
