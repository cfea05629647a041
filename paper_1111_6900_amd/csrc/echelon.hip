// Row echelon forms over F_{2^e} (M4RIE paper, Sections 4.1 and 6): the
// reduced (or plain) row echelon form of A in place, its rank and its pivot
// columns.
//
// The paper eliminates one column at a time with Newton-John tables and, for
// speed, recurses through PLE decomposition so that most of the work becomes
// matrix products.  Here the matrix is processed in column panels of 64, and
// per panel:
//   1. pivots and W = K^{-1} (K: the original entries of the pivot rows at
//      the pivot columns).  A probe workgroup eliminates the first 128 of
//      the rows r..m-1; when they give a pivot in every panel column, they
//      are the panel's pivots.  Otherwise a tournament over all the rows
//      keeps each workgroup's pivot rows until one workgroup holds them all.
//      That last workgroup (or the probe) eliminates by Gauss-Jordan and
//      carries each row along as a combination of the pivot rows, so it
//      also writes W.
//   2. the pivot rows Y are moved to rows r..r+rp-1 (only the rows that
//      must move), and on columns c0..n-1 one product on the bitsliced path
//      finishes the panel:
//          A[rows from lo] += H * Y,   H = G * W on the other rows,
//                                      H = W - I on the pivot rows,
//      (G: the other rows' original pivot-column entries, zero on the pivot
//      rows), so that the pivot rows become the reduced rows W * Y and every
//      other row adds G * (W * Y).  The other rows are those below, and
//      those above as well for the reduced form (lo = 0).  The rows below
//      become zero on the panel (they lie in the span of the pivot rows
//      there).  G * W, and the next panel's columns of the result, come from
//      tables of multiples (the Newton-John tables of Section 4), so the
//      next panel's pivot search starts on a side stream before the product
//      and runs beside it.
// The reduced row echelon form is unique, so it equals the oracle's result
// whatever rows are chosen as pivots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <utility>
#include <vector>

#include "ctx.hpp"
#include "field.hpp"
#include "gf2e.h"
#include "gf2e_internal.hpp"

namespace gf2e {

namespace {

constexpr int kPanel = 64;  // columns per panel (max pivots per panel)

// Log/antilog tables (Ctx::field_tables): exp[i] = g^i for i < 2q and 0 for
// 2q <= i <= 4q; log[a] for a != 0, and log[0] = 2q, so that
// exp[log[a] + log[b]] is the product a*b for all a, b without a branch.
struct DevField {
    const uint16_t* exp;  // 4q + 1 entries
    const uint32_t* log;  // q + 1 entries
    uint32_t q;
};
constexpr int kMaxLdsQ = 1023;  // tables staged in LDS up to e = 10
constexpr int kLdsExp = 4 * kMaxLdsQ + 1;


__device__ inline uint32_t ld_el(const void* M, int wide, int64_t i)
{
    return wide ? static_cast<const uint16_t*>(M)[i] : static_cast<const uint8_t*>(M)[i];
}
__device__ inline void st_el(void* M, int wide, int64_t i, uint32_t v)
{
    if (wide) static_cast<uint16_t*>(M)[i] = uint16_t(v);
    else static_cast<uint8_t*>(M)[i] = uint8_t(v);
}

// Sticky err |= 1 if an entry of A (m x n) is >= 2^e.
__global__ void range_check_kernel(const void* A, int64_t lda, int64_t m, int64_t n, int wide, uint32_t lim,
                                   int* err)
{
    bool bad = false;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y)
        for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < n; c += int64_t(gridDim.x) * blockDim.x)
            bad |= ld_el(A, wide, i * lda + c) >= lim;
    if (bad) atomicOr(err, 1);
}

// Panel copy: orig[i][c] = A[i][c0 + c] (uint16, row pitch kPanel, zero
// past the panel's last column).
__global__ void panel_copy_kernel(const void* A, int64_t lda, int64_t m, int64_t c0, int bc, int wide,
                                  uint16_t* orig)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * kPanel) return;
    const int64_t i = idx / kPanel;
    const int c = int(idx % kPanel);
    orig[idx] = c < bc ? uint16_t(ld_el(A, wide, i * lda + c0 + c)) : 0;
}

// State of the pivot search of one panel.
struct PanelState {
    int rows[kPanel];      // pivot t: row (relative to r) ...
    int cols[kPanel];      // ... and panel column
    int rp;                // pivots found
};

// Pivot search by tournament: each workgroup takes up to ROWS candidate
// rows of the panel (original entries, from orig), eliminates them column by
// column and keeps the rows that became pivots (at most kPanel, in
// pivot-column order).  Any maximal independent subset of the panel's rows
// spans its row space, so the rows kept by all workgroups span it too, and a
// further level over the kept rows (until one workgroup remains) yields a
// valid pivot set with the panel's pivot columns.  Candidates are row
// indices relative to r (in == nullptr: rows 0..ncand-1; -1: an empty slot).
// A workgroup writes its kept rows to out[blockIdx.x*kPanel + t] (-1 past
// its count); the final level writes the panel state and W = K^{-1} instead
// (see the Gauss-Jordan step below).
//
// Each row is held in registers by PARTS neighbouring lanes of one wave,
// lane `part` owning columns part, part + PARTS, ...  The column loop is
// unrolled, so every register index is a constant and the updates of one
// step are independent of each other; a step costs two barriers and a few
// LDS round trips (the pivot row's logarithms, the antilog lookups).
//
// Before the tournament, one workgroup runs the same elimination on the
// first rows only.  When they already hold a pivot in every column of the
// panel (the usual case for a matrix of full rank), no other row can add
// one, and their pivots are the panel's.
constexpr int kSelRows = 256;   // rows per workgroup of the tournament
constexpr int kSelParts = 4;    // lanes per row in the tournament levels
constexpr int kFinalParts = 8;  // lanes per row in the final level (128 rows, 1024 threads)
constexpr int kProbeRows = 128; // rows of the probe (2 kPanel: full rank unless the rows are special)
// Fields from 2^6 elements on: 64 random rows of a 64-column panel are of
// full rank with probability above 0.98, so the probe takes kPanel rows
// with 16 lanes per row (4 columns per lane, shorter steps).
constexpr int kShortProbeMinE = 6;

template <int ROWS, int PARTS, bool LDS_TABS, bool FINAL>
__global__ __launch_bounds__(ROWS * PARTS) void panel_select_kernel(const uint16_t* orig, int64_t r, int bc,
                                                                    const int* in, int64_t ncand, int* out,
                                                                    PanelState* st, PanelState* hst, DevField F,
                                                                    int wide, void* W)
{
    constexpr int NT = ROWS * PARTS, CPT = kPanel / PARTS;
    static_assert(kPanel % PARTS == 0 && 64 % PARTS == 0 && NT <= 1024, "rows lie within one wave");
    __shared__ uint16_t sexp[LDS_TABS ? kLdsExp : 1];
    __shared__ uint32_t slog[LDS_TABS ? kMaxLdsQ + 1 : 1];
    __shared__ int pivs[kPanel];
    __shared__ int plog[kPanel];
    __shared__ int alog[FINAL ? kPanel : 1];    // the pivot row's coefficients (logs)
    __shared__ int colpiv[FINAL ? kPanel : 1];  // pivot index of each panel column, -1 if none
    // Row and column of each pivot, written out after the last step: stores
    // to the panel state (host memory for the final level) inside the steps
    // would make every later barrier wait for them.
    __shared__ int prow_of[kPanel], pcol_of[kPanel];
    __shared__ int lead;
    const int tid = threadIdx.x, rl = tid / PARTS, part = tid % PARTS, lane = tid & 63;
    const int q = int(F.q);
    const int64_t slot = int64_t(blockIdx.x) * ROWS + rl;
    const int row = slot < ncand ? (in ? in[slot] : int(slot)) : -1;
    uint32_t v[CPT];  // v[i]: column part + PARTS * i of this row
#pragma unroll
    for (int i = 0; i < CPT; ++i) v[i] = row >= 0 ? orig[(r + row) * kPanel + part + PARTS * i] : 0u;
    // a[i]: this row as a combination of the pivot rows found so far, indexed
    // by their pivot columns (part + PARTS * i); the final level only
    uint32_t a[FINAL ? CPT : 1] = {};
    // tables in LDS when they fit (e <= 10), else read from the device copy;
    // a compile-time choice, so that the lookups are LDS (or global) loads
    if constexpr (LDS_TABS) {
        for (int k = tid; k <= 4 * q; k += NT) sexp[k] = F.exp[k];
        for (int k = tid; k <= q; k += NT) slog[k] = F.log[k];
    }
    const uint16_t* ex = LDS_TABS ? sexp : F.exp;
    const uint32_t* lg = LDS_TABS ? slog : F.log;
    if (tid < kPanel) {
        pivs[tid] = INT_MAX;
        if constexpr (FINAL) colpiv[tid] = -1;
    }
    __syncthreads();
    bool used = row < 0;
    int npiv = 0;
    int my_t = -1, my_lead = 0;  // a pivot row's index and log of 1 / its pivot
    // Offers this row as the pivot of column c (the first row with a nonzero
    // entry there wins); only the lane owning column c has a say.
    auto offer = [&](int c, bool nonzero) __attribute__((always_inline)) {
        const uint64_t bal = __ballot(c < bc && !used && part == c % PARTS && nonzero);
        if (bal && lane == __ffsll(static_cast<long long>(bal)) - 1) atomicMin(&pivs[c], rl);
    };
    offer(0, v[0] != 0);
    // Step J eliminates column J; the steps are instantiated one by one, so
    // that J is a constant in each.  The final level eliminates column J
    // from every other row, pivot rows included (Gauss-Jordan), and carries
    // the combinations along, so that each pivot row ends as its row of
    // K^{-1} times its pivot.
    auto step = [&]<int J>() __attribute__((always_inline)) {  // inlined, so v and a stay in registers
        if (J >= bc) return;  // uniform
        __syncthreads();      // pivs[J] is final; plog, alog and lead of step J - 1 are no longer read
        const int p = pivs[J];
        if (p == INT_MAX) {  // no pivot in column J: offer column J + 1 as it is
            if constexpr (J + 1 < kPanel) offer(J + 1, v[(J + 1) / PARTS] != 0);
            return;
        }
        if constexpr (FINAL)  // the pivot row's own coefficient
            a[J / PARTS] = rl == p && part == J % PARTS ? 1u : a[J / PARTS];
        if (rl == p) {  // the pivot row publishes the logarithms of its entries (2q for zeros)
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                plog[part + PARTS * i] = int(lg[v[i]]);
                if constexpr (FINAL) alog[part + PARTS * i] = int(lg[a[i]]);
            }
            if (part == J % PARTS) lead = q - int(lg[v[J / PARTS]]);
        }
        if constexpr (FINAL)
            if (tid == 0) colpiv[J] = npiv;
        __syncthreads();
        if (rl == p) {
            if (part == 0) {
                prow_of[npiv] = row;
                pcol_of[npiv] = J;
            }
            used = true;
            my_t = npiv;
            my_lead = lead;
        }
        ++npiv;  // uniform across the workgroup
        // x: this row's entry in column J, held by the lane owning column J
        const uint32_t x = __shfl(v[J / PARTS], (lane & ~(PARTS - 1)) | (J % PARTS));
        // lf: log of the multiplier x / pivot, or 2q (a zero product) for
        // rows with nothing to eliminate; no branch per row
        int lf = int(lg[x]) + lead;
        lf -= lf >= q ? q : 0;
        const bool skip = FINAL ? (rl == p || x == 0) : (used || x == 0);
        lf = skip ? 2 * q : lf;
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            if (part + PARTS * i > J) v[i] ^= ex[lf + plog[part + PARTS * i]];
            // combinations only reach the columns of pivots found so far
            if constexpr (FINAL)
                if (part + PARTS * i <= J) a[i] ^= ex[lf + alog[part + PARTS * i]];
        }
        if constexpr (J + 1 < kPanel) offer(J + 1, v[(J + 1) / PARTS] != 0);
    };
    [&]<int... J>(std::integer_sequence<int, J...>) __attribute__((always_inline)) {
        (step.template operator()<J>(), ...);
    }(std::make_integer_sequence<int, kPanel>{});
    __syncthreads();  // prow_of and pcol_of are complete
    if constexpr (FINAL) {
        if (tid < npiv) {
            st->rows[tid] = prow_of[tid];
            st->cols[tid] = pcol_of[tid];
            hst->rows[tid] = prow_of[tid];
            hst->cols[tid] = pcol_of[tid];
        }
        if (tid == 0) {
            st->rp = npiv;
            hst->rp = npiv;
        }
        // W[t][s] = coefficient of pivot row s in pivot row t, over its pivot
        if (my_t >= 0) {
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int s = colpiv[part + PARTS * i];
                if (s >= 0) st_el(W, wide, int64_t(my_t) * npiv + s, ex[int(lg[a[i]]) + my_lead]);
            }
        }
    } else {
        if (tid < kPanel) out[int64_t(blockIdx.x) * kPanel + tid] = tid < npiv ? prow_of[tid] : -1;
    }
}

// The final-level pivot search over F_4 (x^2 + x + 1) in one wave: lane l
// holds candidate rows l and l + 64, each as two 64-bit planes (bit c of lo
// / hi: the x^0 / x^1 coefficient of column c), so that a step is two
// ballots, a broadcast of the pivot row by lane reads and a dozen word
// operations per row, with no barrier.  Same results as
// panel_select_kernel<ROWS, PARTS, *, true>: the first row (in candidate
// order) with a nonzero entry in column J becomes pivot J, column J is
// eliminated from every other row (Gauss-Jordan), the combinations a (over
// pivot columns) are carried along, and W = K^{-1}.  Up to kGf4Rows = 128
// candidates.
constexpr int kGf4Rows = 128;

// m * (h x + l) over F_4 on bit-planes, m = m1 x + m0 as all-ones masks
// (x^2 = x + 1): high plane m1 (h + l) + m0 h, low plane m1 h + m0 l.
__device__ __attribute__((always_inline)) inline void gf4_axpy(uint64_t M1, uint64_t M0, uint64_t h, uint64_t l,
                                                                uint64_t& dh, uint64_t& dl)
{
    dh ^= (M1 & (h ^ l)) ^ (M0 & h);
    dl ^= (M1 & h) ^ (M0 & l);
}
// Product of two elements of F_4 (values 0..3).
__device__ __attribute__((always_inline)) inline uint32_t gf4_mul(uint32_t a, uint32_t b)
{
    const uint32_t a1 = a >> 1, a0 = a & 1, b1 = b >> 1, b0 = b & 1;
    return (((a1 & b1) ^ (a1 & b0) ^ (a0 & b1)) << 1) | ((a1 & b1) ^ (a0 & b0));
}
__device__ __attribute__((always_inline)) inline uint32_t gf4_at(uint64_t hi, uint64_t lo, int c)
{
    return uint32_t(((hi >> c) & 1) << 1 | ((lo >> c) & 1));
}
// x from lane `src` of the wave (src uniform).
__device__ __attribute__((always_inline)) inline uint64_t lane_read64(uint64_t x, int src)
{
    const uint32_t l = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x)), src));
    const uint32_t h = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x >> 32)), src));
    return uint64_t(l) | (uint64_t(h) << 32);
}

// One candidate row (slot) of the F_4 search: its planes and combination.
struct Gf4Row {
    uint64_t lo = 0, hi = 0, alo = 0, ahi = 0;
    int row = -1, t = -1;  // input row (relative to r), pivot index
    uint32_t inv = 0;      // 1 / its pivot entry
    bool used = true;
};

__global__ __launch_bounds__(64) void panel_select_gf4_kernel(const uint16_t* orig, int64_t r, int bc, const int* in,
                                                              int64_t ncand, PanelState* st, PanelState* hst,
                                                              void* W)
{
    __shared__ int colpiv[kPanel];
    __shared__ int prow_of[kPanel], pcol_of[kPanel];  // written out after the last step
    const int lane = threadIdx.x;
    Gf4Row R[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int slot = lane + 64 * h;
        R[h].row = slot < ncand ? (in ? in[slot] : slot) : -1;
        R[h].used = R[h].row < 0;
        if (R[h].row >= 0) {
            // the panel copy's rows are 64 uint16 (128 bytes): 8 loads of 16 bytes
            const uint4* src = reinterpret_cast<const uint4*>(orig + (r + R[h].row) * kPanel);
#pragma unroll
            for (int q = 0; q < kPanel / 8; ++q) {
                const uint4 v = src[q];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint64_t x = (w[k >> 1] >> (16 * (k & 1))) & 3u;
                    R[h].lo |= (x & 1) << (8 * q + k);
                    R[h].hi |= (x >> 1) << (8 * q + k);
                }
            }
            const uint64_t keep = bc >= 64 ? ~uint64_t(0) : (uint64_t(1) << bc) - 1;  // (columns past bc are zero)
            R[h].lo &= keep;
            R[h].hi &= keep;
        }
    }
    colpiv[lane] = -1;
    int npiv = 0;
    for (int J = 0; J < bc; ++J) {
        // the first candidate (slots 0..63, then 64..127) with a nonzero entry in column J
        const uint64_t b0 = __ballot(!R[0].used && (((R[0].lo | R[0].hi) >> J) & 1));
        const uint64_t b1 = __ballot(!R[1].used && (((R[1].lo | R[1].hi) >> J) & 1));
        if (!b0 && !b1) continue;  // no pivot in column J (uniform)
        const int ph = b0 ? 0 : 1;
        const int pl = __ffsll(static_cast<long long>(b0 ? b0 : b1)) - 1;
        const bool mine = lane == pl;
        // the pivot row's own coefficient, then the row to every lane
        if (mine) (ph ? R[1] : R[0]).alo |= uint64_t(1) << J;
        const Gf4Row& P = ph ? R[1] : R[0];
        const uint64_t plo = lane_read64(P.lo, pl), phi = lane_read64(P.hi, pl);
        const uint64_t palo = lane_read64(P.alo, pl), pahi = lane_read64(P.ahi, pl);
        const uint32_t x = gf4_at(phi, plo, J);
        const uint32_t pinv = x == 1 ? 1u : x ^ 1u;  // 1/x: 1 -> 1, x -> x + 1, x + 1 -> x
        if (mine) {
            Gf4Row& Q = ph ? R[1] : R[0];
            Q.used = true;
            Q.t = npiv;
            Q.inv = pinv;
            prow_of[npiv] = Q.row;
            pcol_of[npiv] = J;
            colpiv[J] = npiv;
        }
        ++npiv;  // uniform
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (mine && h == ph) continue;
            const uint32_t mlt = gf4_mul(gf4_at(R[h].hi, R[h].lo, J), pinv);  // 0: nothing to eliminate
            const uint64_t M1 = 0 - uint64_t(mlt >> 1), M0 = 0 - uint64_t(mlt & 1);
            gf4_axpy(M1, M0, phi, plo, R[h].hi, R[h].lo);
            gf4_axpy(M1, M0, pahi, palo, R[h].ahi, R[h].alo);
        }
    }
    __syncthreads();  // colpiv, prow_of and pcol_of are complete
    if (lane < npiv) {
        st->rows[lane] = prow_of[lane];
        st->cols[lane] = pcol_of[lane];
        hst->rows[lane] = prow_of[lane];
        hst->cols[lane] = pcol_of[lane];
    }
    if (lane == 0) {
        st->rp = npiv;
        hst->rp = npiv;
    }
    // W[t][s] = coefficient of pivot row s (at its column) in pivot row t, over t's pivot
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (R[h].t >= 0)
            for (int c = 0; c < bc; ++c) {
                const int s2 = colpiv[c];
                if (s2 >= 0)
                    st_el(W, 0, int64_t(R[h].t) * npiv + s2, gf4_mul(gf4_at(R[h].ahi, R[h].alo, c), R[h].inv));
            }
}

// G[i][t] = original entry of (new) row i at pivot column t, for all rows:
// rows i < r are unmoved, row r + k is old row r + perm[k] for k < plen and
// unmoved beyond, and the pivot rows r..r+rp-1 get zeros (so that one
// product can update every other row).  Pitch rp.
__global__ void gather_pivot_columns_kernel(const uint16_t* orig, int64_t r, int64_t m, const int* perm,
                                            int plen, const PanelState* st, int rp, int wide, void* G)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * rp) return;
    const int64_t i = idx / rp;
    const int t = int(idx % rp);
    if (i >= r && i < r + rp) {
        st_el(G, wide, idx, 0);
        return;
    }
    const int64_t src = i < r ? i : r + (i - r < plen ? perm[i - r] : i - r);
    st_el(G, wide, idx, orig[src * kPanel + st->cols[t]]);
}

// PLE form of a panel (Section 4.2): K = the original entries of the pivot
// rows at the pivot columns (rp x rp, pivot order), factored K = Lk Uk
// without row exchanges: the pivot search found row t's pivot in column t
// after eliminating the earlier pivots, so every step has a nonzero pivot.
// Lk is lower triangular with the pivots on its diagonal, Uk unit upper
// triangular.  Writes Lk, Lk^{-1} and Uk^{-1} (rp x rp, pitch rp): the
// panel's rows of E are Lk^{-1} times the pivot rows, and a row below with
// pivot-column entries g gets the multipliers g Uk^{-1} in L.
//
// One workgroup eliminates [K | I] forward, one barrier per step: step t
// adds (K[i][t] / K[t][t]) times row t to every row i below, on the columns
// right of t and on the right half, leaving column t (Lk's column) and row t
// unscaled.  Afterwards Lk is the left half's lower triangle, and row t of
// the right half over K[t][t] is row t of Lk^{-1} (the same row operations,
// scaled, take K to Uk).  Uk^{-1} = K^{-1} Lk, with K^{-1} = W from the
// pivot search.
template <bool LDS_TABS>
__global__ __launch_bounds__(1024) void panel_lu_kernel(const uint16_t* orig, int64_t r, const PanelState* st,
                                                        DevField F, int wide, const void* W, void* Lk, void* Linv,
                                                        void* Uinv)
{
    constexpr int NT = 1024, PX = 2 * kPanel + 1;
    __shared__ uint16_t sexp[LDS_TABS ? kLdsExp : 1];
    __shared__ uint32_t slog[LDS_TABS ? kMaxLdsQ + 1 : 1];
    __shared__ uint16_t X[kPanel * PX];         // [K | I], then [Lk, U' | M]
    __shared__ uint32_t lw[kPanel * kPanel];    // logs of Lk (for Uk^{-1})
    __shared__ uint32_t lwi[kPanel * kPanel];   // logs of W = K^{-1}
    __shared__ uint32_t lrow[2 * kPanel];       // step t: logs of row t
    __shared__ uint32_t lcol[kPanel];           // step t: logs of K[i][t] / K[t][t]
    const int tid = threadIdx.x, q = int(F.q), rp = st->rp;
    if constexpr (LDS_TABS) {
        for (int k = tid; k <= 4 * q; k += NT) sexp[k] = F.exp[k];
        for (int k = tid; k <= q; k += NT) slog[k] = F.log[k];
        __syncthreads();
    }
    const uint16_t* ex = LDS_TABS ? sexp : F.exp;
    const uint32_t* lg = LDS_TABS ? slog : F.log;
    for (int idx = tid; idx < rp * rp; idx += NT) {
        const int t = idx / rp, c = idx % rp;
        X[t * PX + c] = orig[(r + st->rows[t]) * kPanel + st->cols[c]];
        X[t * PX + kPanel + c] = t == c ? 1 : 0;
        lwi[idx] = lg[ld_el(W, wide, idx)];
    }
    __syncthreads();
    for (int t = 0; t < rp; ++t) {
        const int wl = rp - t - 1;  // left columns t+1..rp-1; right-half columns 0..t
        if (tid < wl + t + 1) {
            const int c = tid < wl ? t + 1 + tid : kPanel + (tid - wl);
            lrow[c] = lg[X[t * PX + c]];
        } else if (tid >= 128 && tid - 128 < wl) {
            const int i = t + 1 + (tid - 128);
            const uint32_t inv = uint32_t(q) - lg[X[t * PX + t]];
            lcol[i] = lg[ex[lg[X[i * PX + t]] + inv]];
        }
        __syncthreads();
        // thread (row group, column): column tc of the step's w <= kPanel
        // columns, rows t + 1 + tr, t + 17, ... (independent updates)
        const int tc = tid % kPanel, tr = tid / kPanel;
        if (tc < wl + t + 1) {
            const int c = tc < wl ? t + 1 + tc : kPanel + (tc - wl);
            const uint32_t lr = lrow[c];
#pragma unroll 4
            for (int i = t + 1 + tr; i < rp; i += NT / kPanel) X[i * PX + c] ^= ex[lcol[i] + lr];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < rp * rp; idx += NT) {
        const int t = idx / rp, c = idx % rp;
        const uint32_t inv = uint32_t(q) - lg[X[t * PX + t]];
        const uint32_t l = c <= t ? X[t * PX + c] : 0u;
        st_el(Lk, wide, idx, l);
        st_el(Linv, wide, idx, ex[lg[X[t * PX + kPanel + c]] + inv]);
        lw[idx] = lg[l];
    }
    __syncthreads();
    // Uk^{-1}[t][c] = sum_s W[t][s] Lk[s][c] (Lk[s][c] = 0 for s < c)
    for (int idx = tid; idx < rp * rp; idx += NT) {
        const int t = idx / rp, c = idx % rp;
        uint32_t u = 0;
#pragma unroll 8
        for (int sr = c; sr < rp; ++sr) u ^= ex[lwi[t * rp + sr] + lw[sr * rp + c]];
        st_el(Uinv, wide, idx, u);
    }
}

// Row moves of one panel on columns c0..c0+cols-1: position r + moves[j]
// takes old row r + perm[moves[j]].  Gathered into tmp (pitch cols) first,
// then scattered, since the moves permute the rows among themselves.
__global__ void gather_rows_kernel(const void* A, int64_t lda, int64_t r, int64_t c0, const int* perm,
                                   const int* moves, int nmoves, int64_t cols, int wide, void* tmp)
{
    for (int64_t j = blockIdx.y; j < nmoves; j += gridDim.y) {
        const int64_t src = (r + perm[moves[j]]) * lda + c0;
        for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < cols; c += int64_t(gridDim.x) * blockDim.x)
            st_el(tmp, wide, j * cols + c, ld_el(A, wide, src + c));
    }
}

__global__ void scatter_rows_kernel(void* A, int64_t lda, int64_t r, int64_t c0, const int* moves, int nmoves,
                                    int64_t cols, int wide, const void* tmp)
{
    for (int64_t j = blockIdx.y; j < nmoves; j += gridDim.y) {
        const int64_t dst = (r + moves[j]) * lda + c0;
        for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < cols; c += int64_t(gridDim.x) * blockDim.x)
            st_el(A, wide, dst + c, ld_el(tmp, wide, j * cols + c));
    }
}

// Products with a short inner dimension by tables of multiples (the
// Newton-John tables of Section 4: all multiples of a row, built once and
// then read instead of multiplying).  For a k x w block V (k <= kPanel,
// w <= kPanel; columns from w on count as zero) the table holds, for every
// row s of V, byte half h of an element (one half for e <= 8, two above)
// and byte value x,
//     T[((h * k + s) * 256 + x) * kPanel + c] = (x << 8h) * V[s][c],
// so that X[i][s] * V[s][:] is the XOR of one table row per half.  Each
// thread computes one entry by logarithms; values x << 8h outside the
// field are never looked up and hold zero.  One launch builds the tables of
// two blocks V1 (into T1) and V2 (into T2, when V2 is set) with the same k.
__global__ __launch_bounds__(256) void grease_build_kernel(const void* V1, int64_t ldv1, int w1, void* T1,
                                                           const void* V2, int64_t ldv2, int w2, void* T2, int k,
                                                           int halves, DevField F, int e, int wide)
{
    const int64_t entries = int64_t(halves) * k * 256 * kPanel;
    int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const bool second = idx >= entries;
    if (second) idx -= entries;
    if (idx >= entries || (second && !V2)) return;
    const void* V = second ? V2 : V1;
    const int64_t ldv = second ? ldv2 : ldv1;
    const int w = second ? w2 : w1;
    const int c = int(idx % kPanel);
    const int x = int((idx / kPanel) % 256);
    const int64_t hs = idx / (int64_t(kPanel) * 256);
    const int sr = int(hs % k), h = int(hs / k);
    const uint32_t xv = uint32_t(x) << (8 * h);
    const uint32_t v = c < w ? ld_el(V, wide, sr * ldv + c) : 0u;
    const uint32_t prod = (xv >> e) == 0 ? F.exp[F.log[xv] + F.log[v]] : 0u;
    st_el(second ? T2 : T1, wide, idx, prod);
}

// Applies the table of V (grease_build_kernel) to the rows of X (k columns):
// for rows i in [x_lo, m) and columns c < kPanel,
//     out[i][c] = (Cin ? Cin[i][c] : 0) + sum_{s < k} X[i][s] * V[s][c].
// Cin and Cout have w columns (entries past them count as zero), orig takes
// columns c < ow (zero beyond; uint16, pitch kPanel); either output may be
// null.  Rows below x_lo are not written to Cout and copy Cin into orig.
// With Pv set, rows pr0..pr0+k-1 take Pv - I instead (Pv: k x k, pitch k;
// written to Cout only): in the one product that finishes a panel these
// rows turn the pivot rows Y into Pv * Y = Y + (Pv - I) * Y.  Sixteen
// threads share a row, each owning four columns; they read the row of X and
// the table rows that its entries select (64 bytes of a table row per entry
// and half).
__global__ __launch_bounds__(256) void grease_apply_kernel(const void* X, int64_t ldx, int k, int64_t m, int64_t x_lo,
                                                           const void* T, int halves, int wide, const void* Cin,
                                                           int64_t ldcin, void* Cout, int64_t ldcout, int w,
                                                           uint16_t* orig, int ow, const void* Pv, int64_t pr0)
{
    // The workgroup's sixteen rows of X go through LDS first (each thread
    // loads four entries), so that every thread then issues all its table
    // loads at once instead of waiting for each entry of X.
    __shared__ uint32_t xl[16][kPanel];
    const int rl = threadIdx.x / 16, c4 = 4 * (threadIdx.x % 16);
    const int64_t i = int64_t(blockIdx.x) * 16 + rl;
    const bool pivot = Pv && i >= pr0 && i < pr0 + k;
    const bool live = i < m && i >= x_lo && !pivot;
#pragma unroll
    for (int j = 0; j < 4; ++j) xl[rl][c4 + j] = live && c4 + j < k ? ld_el(X, wide, i * ldx + c4 + j) : 0u;
    __syncthreads();
    if (i >= m) return;
    if (pivot) {
        const int t = int(i - pr0);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (c4 + j < w) st_el(Cout, wide, i * ldcout + c4 + j, ld_el(Pv, wide, t * k + c4 + j) ^ (c4 + j == t ? 1u : 0u));
        return;
    }
    uint32_t acc[4] = {0u, 0u, 0u, 0u};
    if (Cin)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (c4 + j < w) acc[j] = ld_el(Cin, wide, i * ldcin + c4 + j);
    if (live) {
        // 16 table loads in flight, then their XORs
#pragma unroll
        for (int s0 = 0; s0 < kPanel; s0 += 16) {
            if (s0 >= k) break;  // uniform
            uint2 t[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int sr = s0 + u;
                const uint32_t x = sr < k ? xl[rl][sr] : 0u;
                const int srow = sr < k ? sr : 0;  // x = 0 selects a zero row
                if (wide) {
                    const uint16_t* T16 = static_cast<const uint16_t*>(T);
                    const uint2 lo = *reinterpret_cast<const uint2*>(T16 + ((int64_t(srow) * 256 + (x & 0xFFu)) * kPanel + c4));
                    uint2 hi = make_uint2(0u, 0u);
                    if (halves > 1)
                        hi = *reinterpret_cast<const uint2*>(
                            T16 + ((int64_t(k + srow) * 256 + ((x >> 8) & 0xFFu)) * kPanel + c4));
                    t[u] = make_uint2(lo.x ^ hi.x, lo.y ^ hi.y);
                } else {
                    const uint8_t* T8 = static_cast<const uint8_t*>(T);
                    t[u] = make_uint2(*reinterpret_cast<const uint32_t*>(T8 + (int64_t(srow) * 256 + x) * kPanel + c4), 0u);
                }
            }
            uint2 sum = make_uint2(0u, 0u);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                sum.x ^= t[u].x;
                sum.y ^= t[u].y;
            }
            if (wide) {
                acc[0] ^= sum.x & 0xFFFFu;
                acc[1] ^= sum.x >> 16;
                acc[2] ^= sum.y & 0xFFFFu;
                acc[3] ^= sum.y >> 16;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j] ^= (sum.x >> (8 * j)) & 0xFFu;
            }
        }
        if (Cout)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c4 + j < w) st_el(Cout, wide, i * ldcout + c4 + j, acc[j]);
    }
    if (orig)
#pragma unroll
        for (int j = 0; j < 4; ++j) orig[i * kPanel + c4 + j] = c4 + j < ow ? uint16_t(acc[j]) : 0;
}

dim3 rows_grid(int64_t rows, int64_t cols)
{
    return dim3(unsigned(std::min<int64_t>(ceil_div(cols, 256), 64)), unsigned(std::min<int64_t>(rows, 65535)));
}

}  // namespace

DevTables Ctx::field_tables(int e, uint32_t f)
{
    const uint64_t key = (uint64_t(e) << 32) | f;
    const uint32_t q = (1u << e) - 1u;
    const size_t exp_words = round_up(4 * q + 1, 2);  // uint16 entries, padded to 4 bytes
    auto view = [&](void* d) {
        return DevTables{static_cast<const uint16_t*>(d),
                         reinterpret_cast<const uint32_t*>(static_cast<const uint16_t*>(d) + exp_words)};
    };
    auto it = ftabs.find(key);
    if (it != ftabs.end()) return view(it->second);
    std::vector<uint16_t> hexp(exp_words, 0);
    std::vector<uint32_t> hlog(q + 1, 0);
    const uint32_t g = find_generator(e, f);
    uint32_t x = 1;
    for (uint32_t i = 0; i < q; ++i) {
        hexp[i] = hexp[i + q] = uint16_t(x);
        hlog[x] = i;
        x = polymulmod(x, g, f, e);
    }
    hlog[0] = 2 * q;
    void* d = nullptr;
    const size_t eb = exp_words * sizeof(uint16_t), lb = hlog.size() * sizeof(uint32_t);
    if (hipMalloc(&d, eb + lb) != hipSuccess) {
        (void)hipGetLastError();
        return {nullptr, nullptr};
    }
    if (hipMemcpy(d, hexp.data(), eb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(static_cast<uint8_t*>(d) + eb, hlog.data(), lb, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return {nullptr, nullptr};
    }
    ftabs[key] = d;
    return view(d);
}

void* Ctx::ensure_pinned(size_t bytes)
{
    if (pinned_bytes >= bytes) return pinned;
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_bytes = 0;
    if (hipHostMalloc(&pinned, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        pinned = nullptr;
        return nullptr;
    }
    pinned_bytes = bytes;
    return pinned;
}

hipStream_t Ctx::side_stream()
{
    if (!side && hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        side = nullptr;
    }
    return side;
}

int Ctx::echelon(gf2e_mat* A, int e, uint32_t f, int full, int64_t* rank, int64_t* pivots, hipStream_t s,
                 PleOut* ple)
{
    const int64_t m = A->rows, n = A->cols;
    *rank = 0;
    if (m == 0 || n == 0) return GF2E_OK;
    const int wide = e > 8 ? 1 : 0;
    const int esz = elem_bytes(e);
    const DevTables tabs = field_tables(e, f);
    if (!tabs.exp) return GF2E_ENOMEM;
    const uint32_t q = (1u << e) - 1u;
    const DevField F{tabs.exp, tabs.log, q};

    // Entries >= 2^e: report before touching A.
    int flag = 0;
    hipLaunchKernelGGL(range_check_kernel, rows_grid(m, n), dim3(256), 0, s, A->data, A->ld, m, n, wide, 1u << e,
                       d_err);
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(&flag, d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return GF2E_EDEVICE;
    if (flag & 1) {
        const int zero = 0;
        (void)hipMemcpy(d_err, &zero, sizeof(int), hipMemcpyHostToDevice);
        return GF2E_ERANGE;
    }

    // Buffers: the panel copy, two candidate lists of the tournament, panel
    // state, permutation and row moves, W, pivot-column gather, and the
    // moved rows of one panel.
    auto al = [](int64_t b) { return round_up(b, 256); };
    const int64_t b_orig = al(m * kPanel * 2), b_cand = al(ceil_div(m, kSelRows) * kPanel * 4),
                  b_state = al(sizeof(PanelState)), b_perm = al((m + 2 * kPanel) * 4),
                  b_w = al(int64_t(kPanel) * kPanel * esz), b_g = al(m * kPanel * esz),
                  b_mv = al(2 * kPanel * n * esz), b_lu = ple ? 6 * b_w : 0,
                  b_tab = al(4 * int64_t(kPanel) * 256 * kPanel * esz), b_h = al(m * kPanel * esz);
    int rc = ensure_aux(b_orig + 2 * b_cand + b_state + b_perm + b_w + b_g + b_mv + b_lu + b_tab + b_h, s);
    if (rc) return rc;
    uint8_t* base = static_cast<uint8_t*>(aux);
    uint16_t* orig = reinterpret_cast<uint16_t*>(base);
    int* cand[2] = {reinterpret_cast<int*>(base + b_orig), reinterpret_cast<int*>(base + b_orig + b_cand)};
    PanelState* st = reinterpret_cast<PanelState*>(base + b_orig + 2 * b_cand);
    int* perm = reinterpret_cast<int*>(base + b_orig + 2 * b_cand + b_state);
    uint8_t* W = base + b_orig + 2 * b_cand + b_state + b_perm;
    uint8_t* G = W + b_w;
    uint8_t* mvbuf = G + b_g;
    // PLE: the panel's Lk, Lk^{-1} and Uk^{-1} (panel_lu_kernel), two sets:
    // the next panel's are computed on the side stream while this panel's
    // are still read.
    uint8_t* lu_sets = mvbuf + b_mv;
    auto lu_set = [&](int64_t c0p, int which) { return lu_sets + (((c0p / kPanel) & 1) * 3 + which) * b_w; };
    // Tables of multiples and the coefficient matrix H of each panel's product
    uint8_t* Tab = mvbuf + b_mv + b_lu;
    uint8_t* H = Tab + b_tab;
    const int halves = e > 8 ? 2 : 1;
    std::vector<int64_t> rowid, moved;  // PLE: input index of each current row
    if (ple) {
        rowid.resize(size_t(m));
        for (int64_t i = 0; i < m; ++i) rowid[size_t(i)] = i;
        const int64_t mn = std::min(m, n);
        if (launch_zero(ple->L->data, m, mn, ple->L->ld, esz, s) != hipSuccess) return GF2E_EDEVICE;
    }

    // The final pivot-search level writes the panel state to device memory
    // (read by later kernels) and to this mapped host copy (read by the host
    // once the launch has completed), so no copy runs between them.  The
    // row permutation is staged after it in the same pinned buffer.
    constexpr size_t kPermAt = (sizeof(PanelState) + 255) / 256 * 256;
    uint8_t* pin = static_cast<uint8_t*>(ensure_pinned(kPermAt + size_t(m + 2 * kPanel) * 4));
    if (!pin) return GF2E_ENOMEM;
    PanelState* hsp = reinterpret_cast<PanelState*>(pin);
    int* hperm = reinterpret_cast<int*>(pin + kPermAt);
    PanelState* hst_dev = nullptr;
    if (hipHostGetDevicePointer(reinterpret_cast<void**>(&hst_dev), hsp, 0) != hipSuccess || !hst_dev)
        return GF2E_EDEVICE;
    // The pivot search of the next panel runs on a side stream, beside the
    // trailing update of the current one (one panel of lookahead): the update
    // first brings the next panel's columns up to date (event ahead on s),
    // the search waits for that, and the rest of the update follows on s.
    hipStream_t s2 = side_stream();
    // (PLE: the panel's LU factors follow the search on the side stream;
    // the host waits only for the search, s for the factors, event lu_done.)
    hipEvent_t sel_done = get_event(), ahead = get_event(), lu_done = get_event();
    if (!s2 || !sel_done || !ahead || !lu_done) return GF2E_EDEVICE;
    struct EventBack {  // back to the pool on every return, the side stream drained
        Ctx* c;
        hipStream_t side;
        hipEvent_t ev[3];
        ~EventBack()
        {
            (void)hipStreamSynchronize(side);
            for (hipEvent_t e : ev) c->event_pool.push_back(e);
        }
    } event_back{this, s2, {sel_done, ahead, lu_done}};
    const PanelState& hs = *hsp;
    std::vector<char> is_piv;
    uint8_t* Ad = static_cast<uint8_t*>(A->data);
    const int64_t lda = A->ld;
    int64_t r = 0;
    const bool lds_tabs = q <= kMaxLdsQ;
    // A pivot-search launch on the side stream for the panel of bc columns
    // whose rows start at r0; the final level (one workgroup) also writes the
    // panel state and W = K^{-1}.
    auto launch_select = [&]<int ROWS, bool FIN, int PARTS = (FIN ? kFinalParts : kSelParts)>(
                             int64_t r0, int bc, int64_t nb, int64_t ncand, const int* in, int* out) {
        const dim3 grid{unsigned(nb)}, block{unsigned(ROWS * PARTS)};
        if (lds_tabs)
            hipLaunchKernelGGL((panel_select_kernel<ROWS, PARTS, true, FIN>), grid, block, 0, s2, orig, r0, bc, in,
                               ncand, out, st, hst_dev, F, wide, static_cast<void*>(W));
        else
            hipLaunchKernelGGL((panel_select_kernel<ROWS, PARTS, false, FIN>), grid, block, 0, s2, orig, r0, bc, in,
                               ncand, out, st, hst_dev, F, wide, static_cast<void*>(W));
    };
    // PLE: the LU factors of the pivot block of the panel at column c0n (rows
    // from r0) on the side stream, after its pivot search.
    auto launch_lu = [&](int64_t c0n, int64_t r0) {
        void *lk = lu_set(c0n, 0), *li = lu_set(c0n, 1), *ui = lu_set(c0n, 2);
        const void* w = W;
        if (lds_tabs)
            hipLaunchKernelGGL(panel_lu_kernel<true>, dim3(1), dim3(1024), 0, s2, orig, r0, st, F, wide, w, lk, li,
                               ui);
        else
            hipLaunchKernelGGL(panel_lu_kernel<false>, dim3(1), dim3(1024), 0, s2, orig, r0, st, F, wide, w, lk, li,
                               ui);
    };
    // Probes the first rows from row r0 of the panel at column c0n, on the
    // side stream after everything enqueued on s so far; copy: copy the panel
    // first (else the update that precedes has written the copy).
    auto start_search = [&](int64_t c0n, int64_t r0, bool copy) -> int {
        const int bcn = int(std::min<int64_t>(kPanel, n - c0n));
        if (hipEventRecord(ahead, s) != hipSuccess || hipStreamWaitEvent(s2, ahead, 0) != hipSuccess)
            return GF2E_EDEVICE;
        if (copy)
            hipLaunchKernelGGL(panel_copy_kernel, dim3(unsigned(ceil_div(m * kPanel, 256))), dim3(256), 0, s2,
                               A->data, lda, m, c0n, bcn, wide, orig);
        if (e == 2)
            hipLaunchKernelGGL(panel_select_gf4_kernel, dim3(1), dim3(64), 0, s2, orig, r0, bcn,
                               static_cast<const int*>(nullptr), std::min<int64_t>(m - r0, kGf4Rows), st, hst_dev,
                               static_cast<void*>(W));
        else if (e >= kShortProbeMinE)
            launch_select.template operator()<kPanel, true, 16>(r0, bcn, 1, std::min<int64_t>(m - r0, kPanel),
                                                                static_cast<const int*>(nullptr), cand[0]);
        else
            launch_select.template operator()<kProbeRows, true>(r0, bcn, 1, std::min<int64_t>(m - r0, kProbeRows),
                                                                static_cast<const int*>(nullptr), cand[0]);
        if (hipGetLastError() != hipSuccess || hipEventRecord(sel_done, s2) != hipSuccess) return GF2E_EDEVICE;
        if (ple) {
            launch_lu(c0n, r0);
            if (hipGetLastError() != hipSuccess || hipEventRecord(lu_done, s2) != hipSuccess) return GF2E_EDEVICE;
        }
        return GF2E_OK;
    };
    // Products with a short inner dimension k <= kPanel on s by tables of
    // multiples: build() writes the tables of V1 (to Tab) and of V2 (to Tab2,
    // when set) in one launch; apply() forms out = (Cin) + X * V from a table
    // (X, Cin and Cout indexed by absolute row, rows below x_lo left alone;
    // with Pv set, rows r..r+k-1 of Cout take Pv - I).
    uint8_t* Tab2 = Tab + b_tab / 2;
    auto build = [&](int k, const void* V1, int64_t ldv1, int w1, const void* V2, int64_t ldv2, int w2) -> int {
        const int64_t entries = int64_t(halves) * k * 256 * kPanel * (V2 ? 2 : 1);
        hipLaunchKernelGGL(grease_build_kernel, dim3(unsigned(ceil_div(entries, 256))), dim3(256), 0, s, V1, ldv1, w1,
                           static_cast<void*>(Tab), V2, ldv2, w2, static_cast<void*>(Tab2), k, halves, F, e, wide);
        return hipGetLastError() == hipSuccess ? GF2E_OK : GF2E_EDEVICE;
    };
    auto apply = [&](const uint8_t* T, int k, const void* X, int64_t ldx, int64_t x_lo, const void* Cin, int64_t ldcin,
                     void* Cout, int64_t ldcout, int w, uint16_t* o, int ow, const void* Pv) -> int {
        hipLaunchKernelGGL(grease_apply_kernel, dim3(unsigned(ceil_div(m, 16))), dim3(256), 0, s, X, ldx, k, m, x_lo,
                           static_cast<const void*>(T), halves, wide, Cin, ldcin, Cout, ldcout, w, o, ow, Pv, r);
        return hipGetLastError() == hipSuccess ? GF2E_OK : GF2E_EDEVICE;
    };
    if (n > 0 && (rc = start_search(0, 0, true))) return rc;
    for (int64_t c0 = 0; c0 < n && r < m; c0 += kPanel) {
        const int bc = int(std::min<int64_t>(kPanel, n - c0));
        const int64_t mr = m - r;
        // The probe on the first rows was started by the previous panel; the
        // whole tournament runs only when they lack a pivot in some column
        // and further rows exist.
        if (hipEventSynchronize(sel_done) != hipSuccess) return GF2E_EDEVICE;
        const int64_t probe = std::min<int64_t>(mr, e >= kShortProbeMinE ? kPanel : kProbeRows);
        if (hs.rp < bc && mr > probe) {
            // Tournament levels of kSelRows-row workgroups until at most
            // kProbeRows candidates remain, then the final level on those.
            const int* in = nullptr;
            int64_t ncand = mr;
            for (int level = 0; ncand > kProbeRows; ++level) {
                const int64_t nb = ceil_div(ncand, kSelRows);
                int* out = cand[level & 1];
                launch_select.template operator()<kSelRows, false>(r, bc, nb, ncand, in, out);
                in = out;
                ncand = nb * kPanel;
            }
            launch_select.template operator()<kProbeRows, true>(r, bc, 1, ncand, in, cand[0]);
            if (hipGetLastError() != hipSuccess || hipEventRecord(sel_done, s2) != hipSuccess) return GF2E_EDEVICE;
            if (ple) {
                launch_lu(c0, r);  // again, on the final pivots
                if (hipGetLastError() != hipSuccess || hipEventRecord(lu_done, s2) != hipSuccess)
                    return GF2E_EDEVICE;
            }
            if (hipEventSynchronize(sel_done) != hipSuccess) return GF2E_EDEVICE;
        }
        // (The host has seen the search complete, so the kernels enqueued on s
        // from here on read its panel state, W and panel copy.)
        const int rp = hs.rp;
        const bool next = c0 + kPanel < n && r + rp < m;  // a panel follows
        if (rp == 0) {
            if (next && (rc = start_search(c0 + kPanel, r, true))) return rc;
            continue;
        }
        for (int t = 0; t < rp; ++t)
            if (pivots) pivots[r + t] = c0 + hs.cols[t];

        // Rows r..r+rp-1 receive the pivot rows; a non-pivot row found there
        // moves to the place left by a pivot row from further down.  The
        // order of the non-pivot rows does not matter: they are reduced by
        // later panels, and the reduced form is unique.  Rows from plen on
        // (past every pivot row) stay where they are, so only the first plen
        // entries of the permutation and the list of moved rows are sent.
        int plen = rp;
        for (int t = 0; t < rp; ++t) plen = std::max(plen, hs.rows[t] + 1);
        for (int i = 0; i < plen; ++i) hperm[i] = i;
        is_piv.assign(size_t(std::min<int64_t>(mr, kPanel)), 0);
        for (int t = 0; t < rp; ++t)
            if (hs.rows[t] < rp) is_piv[hs.rows[t]] = 1;
        int disp[kPanel], nd = 0;
        for (int k = 0; k < rp; ++k)
            if (!is_piv[k]) disp[nd++] = k;
        int* moves = hperm + plen;
        int nm = 0;
        for (int t = 0, j = 0; t < rp; ++t) {
            if (hs.rows[t] != t) moves[nm++] = t;
            if (hs.rows[t] >= rp) {
                hperm[hs.rows[t]] = disp[j++];
                moves[nm++] = hs.rows[t];
            }
        }
        for (int t = 0; t < rp; ++t) hperm[t] = hs.rows[t];
        // from pinned memory: a direct copy; the host writes the buffer again
        // only after the next panel's pivot search, which follows this copy
        if (hipMemcpyAsync(perm, hperm, size_t(plen + nm) * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            return GF2E_EDEVICE;

        hipLaunchKernelGGL(gather_pivot_columns_kernel, dim3(unsigned(ceil_div(m * rp, 256))), dim3(256), 0, s, orig,
                           r, m, perm, plen, st, rp, wide, G);
        const int64_t nc = n - c0;
        if (nm > 0) {
            hipLaunchKernelGGL(gather_rows_kernel, rows_grid(nm, nc), dim3(256), 0, s, A->data, lda, r, c0, perm,
                               perm + plen, nm, nc, wide, mvbuf);
            hipLaunchKernelGGL(scatter_rows_kernel, rows_grid(nm, nc), dim3(256), 0, s, A->data, lda, r, c0,
                               perm + plen, nm, nc, wide, mvbuf);
            if (ple) {
                // the moved rows take their multipliers of the earlier panels
                // (columns 0..r-1 of L) and their input indices along
                if (r > 0) {
                    hipLaunchKernelGGL(gather_rows_kernel, rows_grid(nm, r), dim3(256), 0, s, ple->L->data,
                                       ple->L->ld, r, int64_t(0), perm, perm + plen, nm, r, wide, mvbuf);
                    hipLaunchKernelGGL(scatter_rows_kernel, rows_grid(nm, r), dim3(256), 0, s, ple->L->data,
                                       ple->L->ld, r, int64_t(0), perm + plen, nm, r, wide, mvbuf);
                }
                moved.resize(size_t(nm));
                for (int j = 0; j < nm; ++j) moved[size_t(j)] = rowid[size_t(r + hperm[moves[j]])];
                for (int j = 0; j < nm; ++j) rowid[size_t(r + moves[j])] = moved[size_t(j)];
            }
        }
        if (hipGetLastError() != hipSuccess) return GF2E_EDEVICE;

        // The product that finishes the panel: A[i][c0..n) += H[i] * Y for
        // rows i >= lo, where Y is the rp pivot rows (at row r, as they are
        // now) and H (pitch rp) was set up by the caller: its pivot rows are
        // V - I, so that the pivot rows become V * Y, and the other rows add
        // their multiples of V * Y.  Before it, the next panel's copy is
        // computed from the same H and Y by a table (orig = A + H * Y on the
        // next panel's columns, from Tab2, which the caller built from the
        // next panel's columns of Y) and the next pivot search starts on the
        // side stream (its rows begin at rn).
        uint8_t* Y = Ad + (r * lda + c0) * esz;
        const int bcn = next ? int(std::min<int64_t>(kPanel, n - c0 - kPanel)) : 0;
        const void* Ynext = next ? static_cast<const void*>(Y + kPanel * esz) : nullptr;
        auto finish = [&](int64_t lo, int64_t rn) -> int {
            int rc2;
            if (next) {
                if ((rc2 = apply(Tab2, rp, H, rp, lo, Ad + (c0 + kPanel) * esz, lda, nullptr, 0, bcn, orig, bcn,
                                 nullptr)))
                    return rc2;
                if ((rc2 = start_search(c0 + kPanel, rn, false))) return rc2;
            }
            const gf2e_mat Hm{H + lo * rp * esz, m - lo, rp, rp};
            const gf2e_mat Ym{Y, rp, nc, lda};
            gf2e_mat Cm{Ad + (lo * lda + c0) * esz, m - lo, nc, lda};
            return mul(e, f, &Hm, &Ym, &Cm, s, true);
        };

        if (ple) {
            // PLE (Section 4.2): E's rows of this panel are Lk^{-1} times the
            // pivot rows (row echelon form, leading ones), the rows below get
            // the multipliers G Uk^{-1} in L and lose their multiples of E's
            // rows; the rows above keep their entries (E is not reduced).
            // (Lk, Lk^{-1} and Uk^{-1} came with the pivot search.)
            uint8_t *Lk = lu_set(c0, 0), *Lkinv = lu_set(c0, 1), *Ukinv = lu_set(c0, 2);
            // E_p = Lk^{-1} * (pivot rows), L below = G * Uk^{-1}, and the rows
            // below lose (L below) * E_p: as one product with H = [Lk^{-1} - I;
            // (L below) * Lk^{-1}] on rows r..m-1.
            uint8_t* Ld = static_cast<uint8_t*>(ple->L->data);
            const int64_t ldl = ple->L->ld;
            if (hipStreamWaitEvent(s, lu_done, 0) != hipSuccess) return GF2E_EDEVICE;
            if (hipMemcpy2DAsync(Ld + (r * ldl + r) * esz, size_t(ldl * esz), Lk, size_t(rp * esz),
                                 size_t(rp * esz), size_t(rp), hipMemcpyDeviceToDevice, s) != hipSuccess)
                return GF2E_EDEVICE;
            // L below (rows r + rp on) from Uk^{-1}'s table, then H: Lk^{-1}'s
            // table on L below, Lk^{-1} - I on the pivot rows.  (The last
            // panel has no rows below: only the pivot rows of H are written.)
            if ((rc = build(rp, Ukinv, rp, rp, Ynext, lda, bcn)) ||
                (rc = apply(Tab, rp, G, rp, r + rp, nullptr, 0, Ld + r * esz, ldl, rp, nullptr, 0, nullptr)) ||
                (rc = build(rp, Lkinv, rp, rp, nullptr, 0, 0)) ||
                (rc = apply(Tab, rp, Ld + r * esz, ldl, r + rp, nullptr, 0, H, rp, rp, nullptr, 0, Lkinv)) ||
                (rc = finish(r, r + rp)))
                return rc;
            r += rp;
            continue;
        }
        // H = G * W on the other rows (from lo on), W - I on the pivot rows:
        // the pivot rows become X1 = W * (pivot rows), every other row adds
        // G * X1 (G is zero on the pivot rows).
        const int64_t lo = full ? 0 : r;
        if ((rc = build(rp, W, rp, rp, Ynext, lda, bcn)) ||
            (rc = apply(Tab, rp, G, rp, lo, nullptr, 0, H, rp, rp, nullptr, 0, W)) || (rc = finish(lo, r + rp)))
            return rc;
        r += rp;
    }
    *rank = r;
    if (ple)
        for (int64_t i = 0; i < m; ++i) ple->P[i] = rowid[size_t(i)];
    return GF2E_OK;
}

}  // namespace gf2e

using namespace gf2e;

extern "C" {

int gf2e_echelonize(gf2e_ctx* handle, gf2e_mat* A, int e, uint32_t f, int full, int64_t* rank, int64_t* pivots)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || !rank) return GF2E_EINVAL;
    int rc = check_mat(A);
    if (rc) return rc;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    DeviceGuard guard(c->device);
    hipStream_t s = nullptr;
    c->order_stream(s);
    rc = c->echelon(A, e, f, full != 0, rank, pivots, s);
    c->mark_used(s);
    if (rc) return rc;
    return gf2e_sync(handle, nullptr);
}

int gf2e_ple(gf2e_ctx* handle, gf2e_mat* A, gf2e_mat* L, int e, uint32_t f, int64_t* rank, int64_t* P,
             int64_t* Q)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || !rank || !L) return GF2E_EINVAL;
    int rc = check_mat(A);
    if (rc || (rc = check_mat(L))) return rc;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    const int64_t m = A->rows, n = A->cols;
    if (L->rows != m || L->cols != std::min(m, n)) return GF2E_ESHAPE;
    if (m > 0 && !P) return GF2E_EINVAL;
    if (overlaps(A, L, elem_bytes(e))) return GF2E_EALIAS;
    *rank = 0;
    if (m == 0) return GF2E_OK;
    if (n == 0) {
        for (int64_t i = 0; i < m; ++i) P[i] = i;
        return GF2E_OK;
    }
    DeviceGuard guard(c->device);
    hipStream_t s = nullptr;
    c->order_stream(s);
    Ctx::PleOut out{L, P};
    rc = c->echelon(A, e, f, 0, rank, Q, s, &out);
    c->mark_used(s);
    if (rc) return rc;
    return gf2e_sync(handle, nullptr);
}

}  // extern "C"
