/*
 * Driver for a sanitizer build of the CPU oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, gcc): every oracle routine runs on small seeded
 * inputs with zero runs, leading and trailing zeros, one-weight and all-equal
 * distributions and several guide sizes, and the routines that must agree are
 * compared (binary search with linear search, the forest's Alg. 2 descent with
 * the search, Alg. 1 under random schedules with the forest, the alias table's
 * mass with the weights).  Any sanitizer report or mismatch exits non-zero.
 */
#include "../../oracle/rtf_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) { /* xorshift64* (Marsaglia; Vigna) */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545F4914F6CDD1Dull;
}

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);     \
            return 1;                                                            \
        }                                                                        \
    } while (0)

static int one_case(int64_t n, int64_t m, int kind) {
    uint32_t *w = malloc(sizeof(uint32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t r = next_u64();
        w[i] = kind == 0 ? (uint32_t)(r >> 32) : (kind == 1 ? 7u : (uint32_t)(r >> (32 + r % 31)));
        if (kind == 2 && r % 5 == 0) w[i] = 0; /* zero runs */
    }
    if (n > 2 && kind == 2) {
        w[0] = 0;     /* a leading zero */
        w[n - 1] = 0; /* a trailing zero */
    }
    w[n / 2] |= 1u; /* never all zero */
    uint64_t *C = malloc(sizeof(uint64_t) * (size_t)(n + 1));
    oracle_prefix(w, n, C);
    const int64_t S = 4 * n + 16;
    uint64_t *u = malloc(sizeof(uint64_t) * (size_t)S);
    for (int64_t s = 0; s < S; ++s) u[s] = next_u64();
    u[0] = 0;
    u[1] = ~0ull;
    int32_t *i1 = malloc(sizeof(int32_t) * (size_t)S), *i2 = malloc(sizeof(int32_t) * (size_t)S);
    int32_t *i3 = malloc(sizeof(int32_t) * (size_t)S);
    double *x = malloc(sizeof(double) * (size_t)S);
    CHECK(oracle_search(C, n, u, S, i1, x) == ORC_OK);
    CHECK(oracle_linear_search(C, n, u, S, i2) == ORC_OK);
    for (int64_t s = 0; s < S; ++s) CHECK(i1[s] == i2[s] && x[s] >= 0.0 && x[s] <= 1.0);

    uint64_t *key = malloc(sizeof(uint64_t) * (size_t)n), *key2 = malloc(sizeof(uint64_t) * (size_t)n);
    int32_t *child = malloc(sizeof(int32_t) * 2 * (size_t)n), *child2 = malloc(sizeof(int32_t) * 2 * (size_t)n);
    int32_t *table = malloc(sizeof(int32_t) * (size_t)m);
    uint64_t W = 0;
    int64_t eo[2] = {0, n}, co[2] = {0, m};
    CHECK(oracle_forest(w, eo, co, 1, key, child, table, &W) == ORC_OK);
    CHECK(W == C[n]);
    oracle_descend(key, child, table, 0, 0, m, u, S, i3);
    for (int64_t s = 0; s < S; ++s) CHECK(i3[s] == i1[s]);
    for (uint64_t seed = 1; seed <= 3; ++seed) {
        CHECK(oracle_alg1(w, n, m, seed, key2, child2) == ORC_OK);
        for (int64_t j = 0; j < n; ++j) CHECK(key2[j] == key[j]);
        for (int64_t j = 0; j < 2 * n; ++j) CHECK(child2[j] == child[j]);
    }
    int32_t *lvl = malloc(sizeof(int32_t) * (size_t)(n > 1 ? n - 1 : 1));
    CHECK(oracle_levels(w, n, m, lvl) == ORC_OK);
    for (int64_t b = 0; b + 1 < n; ++b) CHECK(lvl[b] >= 0 && lvl[b] <= SENT);

    double *g = malloc(sizeof(double) * (size_t)S), *grad = malloc(sizeof(double) * (size_t)n);
    for (int64_t s = 0; s < S; ++s) g[s] = (double)(int64_t)(next_u64() >> 40) / 1e6 - 8.0;
    CHECK(oracle_grad(w, n, 0.5, u, g, S, grad) == ORC_OK);

    uint64_t *thr = malloc(sizeof(uint64_t) * (size_t)n);
    int32_t *alias = malloc(sizeof(int32_t) * (size_t)n);
    int64_t *work = malloc(sizeof(int64_t) * 2 * (size_t)n);
    CHECK(oracle_alias_build(w, n, thr, alias, work) == ORC_OK);
    /* the table holds each item's mass w_i n exactly */
    uint64_t *mass = calloc((size_t)n, sizeof(uint64_t));
    for (int64_t j = 0; j < n; ++j) {
        CHECK(thr[j] <= W && alias[j] >= 0 && alias[j] < n);
        mass[j] += thr[j];
        mass[alias[j]] += W - thr[j];
    }
    for (int64_t i = 0; i < n; ++i) CHECK(mass[i] == (uint64_t)w[i] * (uint64_t)n);
    oracle_alias_sample(thr, alias, n, W, u, S, i3);
    for (int64_t s = 0; s < S; ++s) CHECK(i3[s] >= 0 && i3[s] < n && w[i3[s]] > 0);

    free(w); free(C); free(u); free(i1); free(i2); free(i3); free(x); free(key); free(key2);
    free(child); free(child2); free(table); free(lvl); free(g); free(grad); free(thr);
    free(alias); free(work); free(mass);
    return 0;
}

int main(void) {
    /* quantisation: zeros, -0.0, subnormals, the maximum, a negative and a NaN */
    float v[8] = {0.0f, -0.0f, 1e-40f, 3.5f, 1.0f, 2.0f, 3.4e38f, 0.25f};
    uint32_t q[8];
    double scale = 0.0;
    CHECK(oracle_quantize(v, 8, q, &scale) == ORC_OK);
    CHECK(q[0] == 0 && q[1] == 0 && q[2] >= 1 && q[6] == 0xFFFFFFFFu);
    v[3] = -1.0f;
    CHECK(oracle_quantize(v, 8, q, &scale) == ORC_ERR_VALUE);
    v[3] = NAN;
    CHECK(oracle_quantize(v, 8, q, &scale) == ORC_ERR_VALUE);

    const int64_t ns[] = {1, 2, 3, 5, 64, 257, 1000, 4097};
    for (size_t a = 0; a < sizeof ns / sizeof ns[0]; ++a) {
        const int64_t n = ns[a];
        const int64_t ms[] = {1, 3, n, 2 * n + 1};
        for (int b = 0; b < 4; ++b)
            for (int kind = 0; kind < 3; ++kind)
                if (one_case(n, ms[b], kind)) {
                    fprintf(stderr, "case n=%lld m=%lld kind=%d\n", (long long)n,
                            (long long)ms[b], kind);
                    return 1;
                }
    }
    printf("oracle sanitizer run ok\n");
    return 0;
}
