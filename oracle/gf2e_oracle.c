/*
 * gf2e_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for dense matrix
 * multiplication over F_{2^e} = F_2[x]/<f>, 2 <= e <= 16.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library; the GPU product path never calls it and shares no code with it.
 *
 * What it follows (M4RIE paper):
 *   - Section 2 (Notation): an element is a polynomial sum a_i x^i of degree
 *     < e, identified with the integer sum a_i 2^i; f has degree e and is
 *     irreducible.  Field multiplication is polynomial multiplication
 *     followed by reduction modulo f.
 *   - Section 4, Algorithm 1 (cubic matrix multiplication), read as
 *     C = A * B with row i of C accumulating A[i][l] * (row l of B) for every
 *     l: m*l*n field multiplications and as many additions (XOR).
 *   - The log/antilog-table form of the field product (a generator g, every
 *     nonzero element is g^i) is the classic table method the paper's
 *     appendix names for other systems; it is used here only because it is
 *     fast enough for the larger test sizes.  Every table entry is checked
 *     against the shift-and-add definition by the test suite.
 *
 * Elements are stored one per uint8_t when e <= 8 and one per uint16_t when
 * e is 9..16, row-major with a leading dimension counted in elements.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EFIELD (-2)
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-5)
#define ORC_ESINGULAR (-9)

/* ---------------------------------------------------------------------- */
/* Polynomials over F_2, held in the bits of an unsigned integer.           */
/* ---------------------------------------------------------------------- */

static int poly_degree(uint64_t p)
{
    int d = -1;
    while (p) { ++d; p >>= 1; }
    return d;
}

/* Remainder of a modulo b (b != 0) in F_2[x]: long division. */
static uint64_t poly_rem(uint64_t a, uint64_t b)
{
    int db = poly_degree(b);
    for (int d = poly_degree(a); d >= db; d = poly_degree(a))
        a ^= b << (d - db);
    return a;
}

/* Carry-less product a(x)*b(x) in F_2[x]: shift-and-add. */
static uint64_t poly_mul(uint64_t a, uint64_t b)
{
    uint64_t r = 0;
    for (int i = 0; b >> i; ++i)
        if ((b >> i) & 1u) r ^= a << i;
    return r;
}

/* f is accepted when deg f = e and no polynomial of degree 1..e/2 divides it
 * (Section 2 asks for an irreducible f). */
int gf2e_oracle_is_irreducible(int e, uint32_t f)
{
    if (e < 1 || e > 16 || poly_degree(f) != e) return 0;
    for (uint64_t g = 2; poly_degree(g) <= e / 2; ++g)
        if (poly_rem(f, g) == 0) return 0;
    return 1;
}

/* Field product by its definition: multiply as polynomials, reduce mod f. */
uint32_t gf2e_oracle_mul_def(int e, uint32_t f, uint32_t a, uint32_t b)
{
    (void)e;
    return (uint32_t)poly_rem(poly_mul(a, b), f);
}

/* Multiplicative order of a nonzero element (0 if a is 0). */
uint32_t gf2e_oracle_order(int e, uint32_t f, uint32_t a)
{
    if (a == 0) return 0;
    uint32_t x = a, ord = 1;
    while (x != 1) {
        x = gf2e_oracle_mul_def(e, f, x, a);
        if (++ord > (1u << e)) return 0; /* f reducible: no cycle through 1 */
    }
    return ord;
}

/* 1 when x itself generates the multiplicative group (f is primitive). */
int gf2e_oracle_is_primitive(int e, uint32_t f)
{
    if (!gf2e_oracle_is_irreducible(e, f)) return 0;
    return gf2e_oracle_order(e, f, 2u) == (1u << e) - 1u;
}

/* ---------------------------------------------------------------------- */
/* Log / antilog tables.                                                   */
/* ---------------------------------------------------------------------- */

typedef struct {
    int e;
    uint32_t f, gen, q;     /* q = 2^e - 1, the group order */
    uint32_t log[65536];    /* log[0] = 2q: points into the zero tail of exp */
    uint16_t exp[4 * 65535 + 1];
} field_tables;

/* Build tables with the smallest generator g found by search (f need not be
 * primitive).  exp has length 4q+1: exp[i] = g^(i mod q) for i < 2q, zero
 * from 2q on, so log[a] + log[b] indexes 0 whenever a or b is 0. */
static int build_tables(int e, uint32_t f, field_tables* T)
{
    if (e < 2 || e > 16 || !gf2e_oracle_is_irreducible(e, f)) return ORC_EFIELD;
    memset(T, 0, sizeof *T);
    T->e = e; T->f = f; T->q = (1u << e) - 1u;
    uint32_t g = 2;
    while (gf2e_oracle_order(e, f, g) != T->q) ++g;
    T->gen = g;
    uint32_t x = 1;
    for (uint32_t i = 0; i < T->q; ++i) {
        T->exp[i] = (uint16_t)x;
        T->exp[i + T->q] = (uint16_t)x;
        T->log[x] = i;
        x = gf2e_oracle_mul_def(e, f, x, g);
    }
    T->log[0] = 2 * T->q;
    return ORC_OK;
}

static inline uint32_t tab_mul(const field_tables* T, uint32_t a, uint32_t b)
{
    return T->exp[T->log[a] + T->log[b]];
}

/* Exported for the table self-tests: returns the generator used, writes the
 * q-entry antilog table (exp_out may be NULL). */
int gf2e_oracle_tables(int e, uint32_t f, uint32_t* gen, uint16_t* exp_out)
{
    field_tables* T = (field_tables*)malloc(sizeof *T);
    if (!T) return ORC_EINVAL;
    int rc = build_tables(e, f, T);
    if (rc == ORC_OK) {
        if (gen) *gen = T->gen;
        if (exp_out) memcpy(exp_out, T->exp, T->q * sizeof(uint16_t));
    }
    free(T);
    return rc;
}

/* Table product of two scalars (for the exhaustive table-vs-definition test). */
int gf2e_oracle_mul_table_all(int e, uint32_t f, uint16_t* out /* 2^e x 2^e */)
{
    field_tables* T = (field_tables*)malloc(sizeof *T);
    if (!T) return ORC_EINVAL;
    int rc = build_tables(e, f, T);
    if (rc == ORC_OK) {
        uint32_t s = 1u << e;
        for (uint32_t a = 0; a < s; ++a)
            for (uint32_t b = 0; b < s; ++b)
                out[a * s + b] = (uint16_t)tab_mul(T, a, b);
    }
    free(T);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Matrices.                                                               */
/* ---------------------------------------------------------------------- */

static inline uint32_t get_el(const void* M, int wide, int64_t idx)
{
    return wide ? ((const uint16_t*)M)[idx] : ((const uint8_t*)M)[idx];
}

static inline void put_el(void* M, int wide, int64_t idx, uint32_t v)
{
    if (wide) ((uint16_t*)M)[idx] = (uint16_t)v;
    else ((uint8_t*)M)[idx] = (uint8_t)v;
}

/* Rows [row0, row1) of C = A * B by the cubic algorithm (Algorithm 1):
 * C_i starts at zero and, for every l, receives A[i][l] * B_l.
 * A is m x k (lda), B is k x n (ldb), C is m x n (ldc).  Rows are split
 * across nthreads OpenMP threads (nthreads <= 0: the OpenMP default).
 * Returns ORC_ERANGE if an input entry is not below 2^e. */
int gf2e_oracle_matmul(int e, uint32_t f, int64_t m, int64_t k, int64_t n,
                       const void* A, int64_t lda, const void* B, int64_t ldb,
                       void* C, int64_t ldc, int64_t row0, int64_t row1,
                       int nthreads)
{
    if (m < 0 || k < 0 || n < 0 || row0 < 0 || row1 > m || row0 > row1)
        return ORC_EINVAL;
    field_tables* T = (field_tables*)malloc(sizeof *T);
    if (!T) return ORC_EINVAL;
    int rc = build_tables(e, f, T);
    if (rc != ORC_OK) { free(T); return rc; }
    const int wide = e > 8;
    const uint32_t lim = 1u << e;
    int bad = 0;
    if (nthreads <= 0) nthreads = omp_get_max_threads();

#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1) reduction(| : bad)
    for (int64_t i = row0; i < row1; ++i) {
        uint32_t* acc = (uint32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
        for (int64_t l = 0; l < k; ++l) {
            uint32_t a = get_el(A, wide, i * lda + l);
            if (a >= lim) { bad = 1; continue; }
            for (int64_t j = 0; j < n; ++j) {
                uint32_t b = get_el(B, wide, l * ldb + j);
                if (b >= lim) { bad = 1; continue; }
                acc[j] ^= tab_mul(T, a, b);
            }
        }
        for (int64_t j = 0; j < n; ++j) put_el(C, wide, i * ldc + j, acc[j]);
        free(acc);
    }
    free(T);
    return bad ? ORC_ERANGE : ORC_OK;
}

/* 1 when every entry of the rows x cols matrix M is below 2^e. */
static int all_in_field(const void* M, int wide, int64_t rows, int64_t cols, int64_t ld, uint32_t lim)
{
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t j = 0; j < cols; ++j)
            if (get_el(M, wide, i * ld + j) >= lim) return 0;
    return 1;
}

/* Single entries C[I[s]][J[s]] = sum_l A[I[s]][l] * B[l][J[s]], for checking
 * large products at sampled positions. */
int gf2e_oracle_entries(int e, uint32_t f, int64_t m, int64_t k, int64_t n,
                        const void* A, int64_t lda, const void* B, int64_t ldb,
                        const int64_t* I, const int64_t* J, int64_t count,
                        uint32_t* out, int nthreads)
{
    field_tables* T = (field_tables*)malloc(sizeof *T);
    if (!T) return ORC_EINVAL;
    int rc = build_tables(e, f, T);
    if (rc != ORC_OK) { free(T); return rc; }
    const int wide = e > 8;
    const uint32_t lim = 1u << e;
    if (!all_in_field(A, wide, m, k, lda, lim) || !all_in_field(B, wide, k, n, ldb, lim)) {
        free(T);
        return ORC_ERANGE;
    }
    int bad = 0;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(| : bad)
    for (int64_t s = 0; s < count; ++s) {
        if (I[s] < 0 || I[s] >= m || J[s] < 0 || J[s] >= n) { bad = 1; continue; }
        uint32_t acc = 0;
        for (int64_t l = 0; l < k; ++l)
            acc ^= tab_mul(T, get_el(A, wide, I[s] * lda + l),
                           get_el(B, wide, l * ldb + J[s]));
        out[s] = acc;
    }
    free(T);
    return bad ? ORC_EINVAL : ORC_OK;
}

/* Freivalds' check of C == A * B over F_{2^e}: with R an n x t matrix of
 * caller-drawn field elements, compare A * (B * R) with C * R (all products
 * by the cubic definition).  Returns the number of rows of the m x t result
 * that differ (0: the check passed), or a negative error code. */
int64_t gf2e_oracle_freivalds(int e, uint32_t f, int64_t m, int64_t k, int64_t n,
                              const void* A, int64_t lda, const void* B, int64_t ldb,
                              const void* C, int64_t ldc, const void* R, int64_t t,
                              int nthreads)
{
    field_tables* T = (field_tables*)malloc(sizeof *T);
    if (!T) return ORC_EINVAL;
    int rc = build_tables(e, f, T);
    if (rc != ORC_OK) { free(T); return rc; }
    const int wide = e > 8;
    const uint32_t lim = 1u << e;
    if (!all_in_field(A, wide, m, k, lda, lim) || !all_in_field(B, wide, k, n, ldb, lim) ||
        !all_in_field(C, wide, m, n, ldc, lim) || !all_in_field(R, wide, n, t, t, lim)) {
        free(T);
        return ORC_ERANGE;
    }
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    /* BR = B * R, then per row i of A: (A * BR)_i and (C * R)_i.  Each sum
     * is accumulated term by term in the order of its index l or j, the t
     * columns side by side (XOR is commutative, so this is the same sum).
     * Products go through the tables: a * b = exp[log a + log b], with the
     * logarithms of R and BR looked up once. */
    uint32_t* logR = (uint32_t*)malloc((size_t)(n * t + 1) * sizeof(uint32_t));
    uint32_t* BR = (uint32_t*)calloc((size_t)(k * t + 1), sizeof(uint32_t));
    if (!logR || !BR) { free(logR); free(BR); free(T); return ORC_EINVAL; }
    for (int64_t x = 0; x < n * t; ++x) logR[x] = T->log[get_el(R, wide, x)];
    int64_t diff = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t l = 0; l < k; ++l) {
        uint32_t* br = BR + l * t;
        for (int64_t j = 0; j < n; ++j) {
            const uint32_t lb = T->log[get_el(B, wide, l * ldb + j)];
            const uint32_t* lr = logR + j * t;
            for (int64_t s = 0; s < t; ++s) br[s] ^= T->exp[lb + lr[s]];
        }
        for (int64_t s = 0; s < t; ++s) br[s] = T->log[br[s]];  /* keep log(BR) */
    }
#pragma omp parallel num_threads(nthreads) reduction(+ : diff)
    {
        uint32_t* acc = (uint32_t*)calloc((size_t)(2 * t + 1), sizeof(uint32_t));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            uint32_t* lhs = acc;
            uint32_t* rhs = acc + t;
            memset(acc, 0, (size_t)(2 * t) * sizeof(uint32_t));
            for (int64_t l = 0; l < k; ++l) {
                const uint32_t la = T->log[get_el(A, wide, i * lda + l)];
                const uint32_t* lbr = BR + l * t;
                for (int64_t s = 0; s < t; ++s) lhs[s] ^= T->exp[la + lbr[s]];
            }
            for (int64_t j = 0; j < n; ++j) {
                const uint32_t lc = T->log[get_el(C, wide, i * ldc + j)];
                const uint32_t* lr = logR + j * t;
                for (int64_t s = 0; s < t; ++s) rhs[s] ^= T->exp[lc + lr[s]];
            }
            int row_bad = 0;
            for (int64_t s = 0; s < t; ++s)
                if (lhs[s] != rhs[s]) row_bad = 1;
            diff += row_bad;
        }
        free(acc);
    }
    free(logR);
    free(BR);
    free(T);
    return diff;
}

int gf2e_oracle_max_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------------- */
/* Triangular solving (Section 4.3).                                       */
/* ---------------------------------------------------------------------- */

/* X = T^{-1} B for a triangular m x m matrix T, overwriting B (m x n).
 *
 * Upper T (lower = 0), the algorithm of Section 4.3: for i from m-1 down to
 * 0, scale row i of B by the inverse of T[i][i], then add T[j][i] times that
 * row to every row j < i.  Lower T (lower = 1) is the mirror image: rows from
 * 0 up, and the scaled row i is added to every row j > i with factor T[j][i].
 * unit = 1 takes the diagonal as ones (its entries are not read).  Columns
 * are independent, so column ranges are split across nthreads threads.
 *
 * ORC_ESINGULAR if a diagonal entry is zero (unit = 0); ORC_ERANGE if an
 * entry that is read is not below 2^e (B is then left partly solved). */
int gf2e_oracle_trsm(int e, uint32_t f, int lower, int unit, int64_t m, int64_t n,
                     const void* Tm, int64_t ldt, void* B, int64_t ldb, int nthreads)
{
    if (m < 0 || n < 0) return ORC_EINVAL;
    field_tables* T = (field_tables*)malloc(sizeof *T);
    if (!T) return ORC_EINVAL;
    int rc = build_tables(e, f, T);
    if (rc != ORC_OK) { free(T); return rc; }
    const int wide = e > 8;
    const uint32_t lim = 1u << e;
    /* Check the triangle that is read, and the diagonal, first. */
    for (int64_t i = 0; i < m && rc == ORC_OK; ++i) {
        for (int64_t j = lower ? 0 : i; j < (lower ? i + 1 : m); ++j) {
            if (j == i && unit) continue;
            const uint32_t t = get_el(Tm, wide, i * ldt + j);
            if (t >= lim) { rc = ORC_ERANGE; break; }
            if (j == i && t == 0) { rc = ORC_ESINGULAR; break; }
        }
    }
    if (rc == ORC_OK && !all_in_field(B, wide, m, n, ldb, lim)) rc = ORC_ERANGE;
    if (rc != ORC_OK) { free(T); return rc; }
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    const int64_t chunk = 64;

#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
        const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
        for (int64_t step = 0; step < m; ++step) {
            const int64_t i = lower ? step : m - 1 - step;
            if (!unit) {
                /* inverse of T[i][i] = g^(q - log T[i][i]) */
                const uint32_t d = get_el(Tm, wide, i * ldt + i);
                const uint32_t dinv = T->exp[T->q - T->log[d]];
                for (int64_t j = c0; j < c1; ++j)
                    put_el(B, wide, i * ldb + j, tab_mul(T, dinv, get_el(B, wide, i * ldb + j)));
            }
            const int64_t r0 = lower ? i + 1 : 0, r1 = lower ? m : i;
            for (int64_t r = r0; r < r1; ++r) {
                const uint32_t x = get_el(Tm, wide, r * ldt + i);
                if (!x) continue;
                for (int64_t j = c0; j < c1; ++j)
                    put_el(B, wide, r * ldb + j,
                           get_el(B, wide, r * ldb + j) ^ tab_mul(T, x, get_el(B, wide, i * ldb + j)));
            }
        }
    }
    free(T);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Echelon forms (Section 4.1 elimination, Section 6).                     */
/* ---------------------------------------------------------------------- */

/* Row echelon form of A (m x n) in place, by the elimination loop of
 * Section 4.1: for each column j in turn, the first row i >= r with a
 * nonzero entry there is scaled so the entry becomes 1 and swapped into row
 * r, and its multiples are added to the rows below it (full = 0) or to every
 * other row (full = 1, the reduced form); r grows by one.  Returns the rank
 * in *rank and the pivot column of row t in pivots[t] (t < rank; pivots may
 * be NULL).  ORC_ERANGE if an entry is not below 2^e (A unchanged). */
int gf2e_oracle_echelon(int e, uint32_t f, int full, int64_t m, int64_t n, void* A, int64_t lda,
                        int64_t* rank, int64_t* pivots)
{
    if (m < 0 || n < 0 || !rank) return ORC_EINVAL;
    field_tables* T = (field_tables*)malloc(sizeof *T);
    if (!T) return ORC_EINVAL;
    int rc = build_tables(e, f, T);
    if (rc != ORC_OK) { free(T); return rc; }
    const int wide = e > 8;
    if (!all_in_field(A, wide, m, n, lda, 1u << e)) { free(T); return ORC_ERANGE; }
    int64_t r = 0;
    for (int64_t j = 0; j < n && r < m; ++j) {
        int64_t i = r;
        while (i < m && get_el(A, wide, i * lda + j) == 0) ++i;
        if (i == m) continue;
        /* scale row i so that its entry in column j is 1 */
        const uint32_t d = get_el(A, wide, i * lda + j);
        const uint32_t dinv = T->exp[T->q - T->log[d]];
        for (int64_t c = j; c < n; ++c) put_el(A, wide, i * lda + c, tab_mul(T, dinv, get_el(A, wide, i * lda + c)));
        /* swap rows i and r */
        if (i != r)
            for (int64_t c = 0; c < n; ++c) {
                const uint32_t a = get_el(A, wide, i * lda + c), b = get_el(A, wide, r * lda + c);
                put_el(A, wide, i * lda + c, b);
                put_el(A, wide, r * lda + c, a);
            }
        /* add multiples of row r to the other rows */
        for (int64_t k = full ? 0 : r + 1; k < m; ++k) {
            if (k == r) continue;
            const uint32_t x = get_el(A, wide, k * lda + j);
            if (!x) continue;
            for (int64_t c = j; c < n; ++c)
                put_el(A, wide, k * lda + c, get_el(A, wide, k * lda + c) ^ tab_mul(T, x, get_el(A, wide, r * lda + c)));
        }
        if (pivots) pivots[r] = j;
        ++r;
    }
    *rank = r;
    free(T);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* PLE decomposition (Section 4.2).                                        */
/* ---------------------------------------------------------------------- */

/* A = P * L * E for an m x n matrix A, by the elimination loop of Section
 * 4.1 modified as Section 4.2 describes: for each column j in turn, the
 * first row i >= r with a nonzero entry d there is swapped into row r (its
 * stored multipliers in L and its record in P move with it), d is recorded
 * as L[r][r] and the row is scaled to leading entry 1 (the paper's variant:
 * L is not unit, E has unit pivots); for every row k below, x = A[k][j] is
 * recorded as L[k][r] and x times row r is added to row k (no row above is
 * touched, so E is not reduced).  Columns are recorded in Q.
 * On return: A holds E (rows 0..rank-1 in row echelon form with leading 1
 * in column Q[t], rows rank..m-1 zero); L (m x min(m, n), row pitch ldl)
 * holds L[i][t] for t < rank (zero for t > i and in columns rank..);
 * P[i] is the index in the input of the row that row i of L*E equals.
 * ORC_ERANGE if an entry is not below 2^e (nothing changed). */
int gf2e_oracle_ple(int e, uint32_t f, int64_t m, int64_t n, void* A, int64_t lda, void* L, int64_t ldl,
                    int64_t* P, int64_t* Q, int64_t* rank)
{
    if (m < 0 || n < 0 || !rank || (m > 0 && !P)) return ORC_EINVAL;
    field_tables* T = (field_tables*)malloc(sizeof *T);
    if (!T) return ORC_EINVAL;
    int rc = build_tables(e, f, T);
    if (rc != ORC_OK) { free(T); return rc; }
    const int wide = e > 8;
    if (!all_in_field(A, wide, m, n, lda, 1u << e)) { free(T); return ORC_ERANGE; }
    const int64_t mn = m < n ? m : n;
    for (int64_t i = 0; i < m; ++i) {
        P[i] = i;
        for (int64_t t = 0; t < mn; ++t) put_el(L, wide, i * ldl + t, 0);
    }
    int64_t r = 0;
    for (int64_t j = 0; j < n && r < m; ++j) {
        int64_t i = r;
        while (i < m && get_el(A, wide, i * lda + j) == 0) ++i;
        if (i == m) continue;
        /* swap rows i and r of A, of the multipliers found so far, and of P */
        if (i != r) {
            for (int64_t c = 0; c < n; ++c) {
                const uint32_t a = get_el(A, wide, i * lda + c), b = get_el(A, wide, r * lda + c);
                put_el(A, wide, i * lda + c, b);
                put_el(A, wide, r * lda + c, a);
            }
            for (int64_t t = 0; t < r; ++t) {
                const uint32_t a = get_el(L, wide, i * ldl + t), b = get_el(L, wide, r * ldl + t);
                put_el(L, wide, i * ldl + t, b);
                put_el(L, wide, r * ldl + t, a);
            }
            const int64_t p = P[i];
            P[i] = P[r];
            P[r] = p;
        }
        /* the pivot goes to L, the row is scaled to leading entry 1 */
        const uint32_t d = get_el(A, wide, r * lda + j);
        put_el(L, wide, r * ldl + r, d);
        const uint32_t dinv = T->exp[T->q - T->log[d]];
        for (int64_t c = j; c < n; ++c) put_el(A, wide, r * lda + c, tab_mul(T, dinv, get_el(A, wide, r * lda + c)));
        /* rows below: record the multiplier, subtract (add) its multiple */
        for (int64_t k = r + 1; k < m; ++k) {
            const uint32_t x = get_el(A, wide, k * lda + j);
            if (!x) continue;
            put_el(L, wide, k * ldl + r, x);
            for (int64_t c = j; c < n; ++c)
                put_el(A, wide, k * lda + c, get_el(A, wide, k * lda + c) ^ tab_mul(T, x, get_el(A, wide, r * lda + c)));
        }
        if (Q) Q[r] = j;
        ++r;
    }
    *rank = r;
    free(T);
    return ORC_OK;
}
