/*
 * Runs every entry point of the CPU oracle on small seeded inputs and checks
 * the results against one another.  The test suite builds this file together
 * with oracle/gf2e_oracle.c under AddressSanitizer and UndefinedBehavior-
 * Sanitizer, so an out-of-bounds access or an undefined operation anywhere in
 * the oracle fails the suite.  Exit status 0: every check passed.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int gf2e_oracle_is_irreducible(int e, uint32_t f);
uint32_t gf2e_oracle_mul_def(int e, uint32_t f, uint32_t a, uint32_t b);
int gf2e_oracle_tables(int e, uint32_t f, uint32_t* gen, uint16_t* exp_out);
int gf2e_oracle_matmul(int e, uint32_t f, int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
                       const void* B, int64_t ldb, void* C, int64_t ldc, int64_t row0, int64_t row1,
                       int nthreads);
int gf2e_oracle_entries(int e, uint32_t f, int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
                        const void* B, int64_t ldb, const int64_t* I, const int64_t* J, int64_t count,
                        uint32_t* out, int nthreads);
int64_t gf2e_oracle_freivalds(int e, uint32_t f, int64_t m, int64_t k, int64_t n, const void* A, int64_t lda,
                              const void* B, int64_t ldb, const void* C, int64_t ldc, const void* R, int64_t t,
                              int nthreads);
int gf2e_oracle_trsm(int e, uint32_t f, int lower, int unit, int64_t m, int64_t n, const void* Tm, int64_t ldt,
                     void* B, int64_t ldb, int nthreads);
int gf2e_oracle_echelon(int e, uint32_t f, int full, int64_t m, int64_t n, void* A, int64_t lda, int64_t* rank,
                        int64_t* pivots);
int gf2e_oracle_ple(int e, uint32_t f, int64_t m, int64_t n, void* A, int64_t lda, void* L, int64_t ldl,
                    int64_t* P, int64_t* Q, int64_t* rank);

static int failures = 0;
#define CHECK(cond, ...)                                              \
    do {                                                              \
        if (!(cond)) {                                                \
            ++failures;                                               \
            fprintf(stderr, "%s:%d: ", __FILE__, __LINE__);           \
            fprintf(stderr, __VA_ARGS__);                             \
            fputc('\n', stderr);                                      \
        }                                                             \
    } while (0)

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)  /* splitmix64 */
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)((z ^ (z >> 31)) >> 16);
}

/* Matrices are exact-size heap blocks, so any access past an edge is caught. */
static int wide_of(int e) { return e > 8; }
static void* alloc(int e, int64_t count) { return calloc(count > 0 ? (size_t)count : 1, wide_of(e) ? 2 : 1); }
static uint32_t get(int e, const void* M, int64_t i)
{
    return wide_of(e) ? ((const uint16_t*)M)[i] : ((const uint8_t*)M)[i];
}
static void put(int e, void* M, int64_t i, uint32_t v)
{
    if (wide_of(e)) ((uint16_t*)M)[i] = (uint16_t)v;
    else ((uint8_t*)M)[i] = (uint8_t)v;
}
static void* random_matrix(int e, int64_t count)
{
    void* M = alloc(e, count);
    for (int64_t i = 0; i < count; ++i) put(e, M, i, rnd() & ((1u << e) - 1u));
    return M;
}

static void check_products(int e, uint32_t f, int64_t m, int64_t k, int64_t n)
{
    void* A = random_matrix(e, m * k);
    void* B = random_matrix(e, k * n);
    void* C = alloc(e, m * n);
    void* C2 = alloc(e, m * n);
    CHECK(gf2e_oracle_matmul(e, f, m, k, n, A, k, B, n, C, n, 0, m, 2) == 0, "matmul e=%d", e);
    /* the same product in two row ranges */
    const int64_t half = m / 2;
    CHECK(gf2e_oracle_matmul(e, f, m, k, n, A, k, B, n, C2, n, 0, half, 1) == 0, "matmul rows");
    CHECK(gf2e_oracle_matmul(e, f, m, k, n, A, k, B, n, C2, n, half, m, 3) == 0, "matmul rows");
    CHECK(memcmp(C, C2, (size_t)(m * n) * (wide_of(e) ? 2 : 1)) == 0, "row ranges e=%d", e);
    /* every entry one by one, against the definition of the field product */
    const int64_t count = m * n;
    int64_t* I = malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    int64_t* J = malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    uint32_t* out = malloc(sizeof(uint32_t) * (size_t)(count > 0 ? count : 1));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            I[i * n + j] = i;
            J[i * n + j] = j;
        }
    CHECK(gf2e_oracle_entries(e, f, m, k, n, A, k, B, n, I, J, count, out, 2) == 0, "entries");
    for (int64_t s = 0; s < count; ++s) {
        uint32_t ref = 0;
        for (int64_t l = 0; l < k; ++l)
            ref ^= gf2e_oracle_mul_def(e, f, get(e, A, I[s] * k + l), get(e, B, l * n + J[s]));
        CHECK(out[s] == ref && get(e, C, s) == ref, "entry %lld e=%d", (long long)s, e);
    }
    /* Freivalds: passes on C, fails once an entry is changed */
    const int64_t t = (64 + e - 1) / e;
    void* R = random_matrix(e, n * t);
    CHECK(gf2e_oracle_freivalds(e, f, m, k, n, A, k, B, n, C, n, R, t, 2) == 0, "freivalds e=%d", e);
    if (count > 0) {
        put(e, C, count / 2, get(e, C, count / 2) ^ 1u);
        int found = 0;
        for (int trial = 0; trial < 8 && !found; ++trial) {
            free(R);
            R = random_matrix(e, n * t);
            found = gf2e_oracle_freivalds(e, f, m, k, n, A, k, B, n, C, n, R, t, 2) > 0;
        }
        CHECK(found, "freivalds missed a changed entry e=%d", e);
    }
    free(R); free(out); free(J); free(I); free(C2); free(C); free(B); free(A);
}

static void check_trsm(int e, uint32_t f, int64_t m, int64_t n)
{
    for (int lower = 0; lower < 2; ++lower)
        for (int unit = 0; unit < 2; ++unit) {
            void* T = random_matrix(e, m * m);
            for (int64_t i = 0; i < m; ++i)
                for (int64_t j = 0; j < m; ++j) {
                    const int64_t idx = i * m + j;
                    if (lower ? j > i : j < i) put(e, T, idx, 0);
                    if (i == j) {
                        uint32_t d = get(e, T, idx);
                        put(e, T, idx, unit ? 1u : (d ? d : 1u));
                    }
                }
            void* X = random_matrix(e, m * n);
            void* B = alloc(e, m * n);
            CHECK(gf2e_oracle_matmul(e, f, m, m, n, T, m, X, n, B, n, 0, m, 1) == 0, "trsm rhs");
            if (unit)  /* a unit solve must not read the diagonal */
                for (int64_t i = 0; i < m; ++i) put(e, T, i * m + i, 0);
            CHECK(gf2e_oracle_trsm(e, f, lower, unit, m, n, T, m, B, n, 2) == 0, "trsm");
            CHECK(memcmp(B, X, (size_t)(m * n) * (wide_of(e) ? 2 : 1)) == 0, "trsm e=%d lower=%d unit=%d", e,
                  lower, unit);
            free(B); free(X); free(T);
        }
}

static void check_echelon_and_ple(int e, uint32_t f, int64_t m, int64_t n)
{
    /* rank-deficient input: the last rows are sums of multiples of the first */
    void* A = random_matrix(e, m * n);
    for (int64_t i = m - 3; i >= 0 && i < m; ++i)
        for (int64_t c = 0; c < n; ++c)
            put(e, A, i * n + c, get(e, A, c) ^ gf2e_oracle_mul_def(e, f, 3u, get(e, A, n + c)));
    void* R = alloc(e, m * n);
    memcpy(R, A, (size_t)(m * n) * (wide_of(e) ? 2 : 1));
    int64_t rank_r = -1, rank_e = -1, rank_p = -1;
    int64_t* piv = malloc(sizeof(int64_t) * (size_t)(m + 1));
    CHECK(gf2e_oracle_echelon(e, f, 1, m, n, R, n, &rank_r, piv) == 0, "rref");
    void* E = alloc(e, m * n);
    memcpy(E, A, (size_t)(m * n) * (wide_of(e) ? 2 : 1));
    CHECK(gf2e_oracle_echelon(e, f, 0, m, n, E, n, &rank_e, NULL) == 0, "ref");
    const int64_t mn = m < n ? m : n;
    void* L = alloc(e, m * mn);
    void* W = alloc(e, m * n);
    memcpy(W, A, (size_t)(m * n) * (wide_of(e) ? 2 : 1));
    int64_t* P = malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t* Q = malloc(sizeof(int64_t) * (size_t)(m + 1));
    CHECK(gf2e_oracle_ple(e, f, m, n, W, n, L, mn, P, Q, &rank_p) == 0, "ple");
    CHECK(rank_r == rank_e && rank_e == rank_p && rank_p <= m - 2, "ranks %lld %lld %lld",
          (long long)rank_r, (long long)rank_e, (long long)rank_p);
    for (int64_t t = 0; t < rank_p; ++t) CHECK(Q[t] == piv[t], "pivot %lld", (long long)t);
    /* A[P[i]] = row i of L * E */
    void* LE = alloc(e, m * n);
    CHECK(gf2e_oracle_matmul(e, f, m, mn, n, L, mn, W, n, LE, n, 0, m, 1) == 0, "L*E");
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < n; ++c)
            CHECK(get(e, LE, i * n + c) == get(e, A, P[i] * n + c), "A = P L E at (%lld, %lld) e=%d",
                  (long long)i, (long long)c, e);
    free(LE); free(Q); free(P); free(W); free(L); free(E); free(piv); free(R); free(A);
}

static void check_errors(void)
{
    uint8_t a[4] = {1, 2, 3, 4}, c[4];
    /* 4 is not an element of F_4; x^2 + 1 is reducible; f = 0 has no degree */
    CHECK(gf2e_oracle_matmul(2, 0x7, 2, 2, 2, a, 2, a, 2, c, 2, 0, 2, 1) < 0, "range");
    CHECK(gf2e_oracle_matmul(2, 0x5, 2, 2, 2, a, 2, a, 2, c, 2, 0, 2, 1) < 0, "reducible");
    CHECK(gf2e_oracle_matmul(2, 0x0, 2, 2, 2, a, 2, a, 2, c, 2, 0, 2, 1) < 0, "zero f");
    CHECK(gf2e_oracle_matmul(2, 0x7, 2, 2, 2, a, 2, a, 2, c, 2, 1, 3, 1) < 0, "rows past m");
    uint8_t T[4] = {0, 1, 0, 1};
    CHECK(gf2e_oracle_trsm(2, 0x7, 0, 0, 2, 2, T, 2, c, 2, 1) < 0, "singular");
}

int main(void)
{
    static const struct { int e; uint32_t f; } fields[] = {
        {2, 0x7}, {3, 0xB}, {4, 0x13}, {8, 0x11D}, {8, 0x11B}, {10, 0x409}, {16, 0x1002B},
    };
    static const int64_t shapes[][3] = {{0, 3, 4}, {3, 0, 4}, {1, 1, 1}, {5, 7, 3}, {17, 33, 9}, {40, 65, 70}};
    for (size_t i = 0; i < sizeof fields / sizeof fields[0]; ++i) {
        const int e = fields[i].e;
        const uint32_t f = fields[i].f;
        CHECK(gf2e_oracle_is_irreducible(e, f), "irreducible e=%d", e);
        uint32_t gen = 0;
        uint16_t* ex = malloc(sizeof(uint16_t) << e);
        CHECK(gf2e_oracle_tables(e, f, &gen, ex) == 0, "tables e=%d", e);
        free(ex);
        for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
            check_products(e, f, shapes[s][0], shapes[s][1], shapes[s][2]);
        check_trsm(e, f, 13, 6);
        check_trsm(e, f, 1, 3);
        check_echelon_and_ple(e, f, 9, 14);
        check_echelon_and_ple(e, f, 16, 7);
    }
    check_errors();
    if (failures) fprintf(stderr, "%d checks failed\n", failures);
    else printf("oracle checks passed\n");
    return failures ? 1 : 0;
}
