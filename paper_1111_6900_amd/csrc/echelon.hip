// Row echelon forms over F_{2^e} (M4RIE paper, Sections 4.1 and 6): the
// reduced (or plain) row echelon form of A in place, its rank and its pivot
// columns.
//
// The paper eliminates one column at a time with Newton-John tables and, for
// speed, recurses through PLE decomposition so that most of the work becomes
// matrix products.  Here the matrix is processed in column panels of 64, and
// per panel:
//   1. pivots: the panel (rows r..m-1) is copied and eliminated column by
//      column, one small kernel per column over all rows; each launch picks
//      the pivot of its column (the first unused row with a nonzero there,
//      found by atomicMin in the previous launch) and eliminates it from the
//      other unused rows of the copy.  rp pivots result.
//   2. W = K^{-1}, where K holds the original entries of the pivot rows at
//      the pivot columns (one workgroup, Gauss-Jordan in LDS).
//   3. the pivot rows are moved to rows r..r+rp-1, and on columns c0..n-1:
//          X1 = W * A[pivot rows]                 (rows r..r+rp-1)
//          A[rows below] += Z * X1                (Z: their original pivot-column entries)
//          A[rows above] += Y * X1                (reduced form only)
//      three products on the bitsliced path.  The rows below become zero on
//      the panel (they lie in the span of the pivot rows there), and the
//      pivot rows become the reduced rows.
// The reduced row echelon form is unique, so it equals the oracle's result
// whatever rows are chosen as pivots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <vector>

#include "ctx.hpp"
#include "field.hpp"
#include "gf2e.h"
#include "gf2e_internal.hpp"

namespace gf2e {

namespace {

constexpr int kPanel = 64;  // columns per panel (max pivots per panel)
constexpr int kStepThreads = 256;

struct DevField {
    const uint16_t* exp;  // exp[i] = g^i for i < 2q
    const uint16_t* log;  // log[a] for a != 0
    uint32_t q;
};

__device__ inline uint32_t fmul(const DevField& F, uint32_t a, uint32_t b)
{
    return (a && b) ? F.exp[F.log[a] + F.log[b]] : 0u;
}
__device__ inline uint32_t finv(const DevField& F, uint32_t a) { return F.exp[F.q - F.log[a]]; }

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

// Panel copies: orig[i][c] = work[i][c] = A[i][c0 + c] for i < m, c < bc
// (uint16 entries, row pitch kPanel).
__global__ void panel_copy_kernel(const void* A, int64_t lda, int64_t m, int64_t c0, int bc, int wide,
                                  uint16_t* orig, uint16_t* work)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * kPanel) return;
    const int64_t i = idx / kPanel;
    const int c = int(idx % kPanel);
    const uint16_t v = c < bc ? uint16_t(ld_el(A, wide, i * lda + c0 + c)) : 0;
    orig[idx] = v;
    work[idx] = v;
}

// State of the pivot search of one panel.
struct PanelState {
    int next[kPanel + 1];  // candidate pivot row (relative to r) of column j, INT_MAX = none
    int rows[kPanel];      // pivot t: row (relative to r) ...
    int cols[kPanel];      // ... and panel column
    int rp;                // pivots found
};

__global__ void panel_reset_kernel(PanelState* st)
{
    for (int j = threadIdx.x; j <= kPanel; j += blockDim.x) st->next[j] = INT_MAX;
    if (threadIdx.x == 0) st->rp = 0;
}

// Rows r..m-1 of the work copy: clear the used flags and offer the rows with
// a nonzero in column 0 as its pivot.
__global__ void panel_start_kernel(const uint16_t* work, int64_t r, int64_t m, uint8_t* used, PanelState* st)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r + i >= m) return;
    used[i] = 0;
    if (work[(r + i) * kPanel] != 0) atomicMin(&st->next[0], int(i));
}

// Column j of the panel: take its candidate pivot row p (if any), eliminate
// column j from every other unused row of the work copy, and offer the rows
// with a nonzero in column j + 1 as that column's pivot.
__global__ void panel_step_kernel(uint16_t* work, int64_t r, int64_t m, int j, int bc, uint8_t* used,
                                  PanelState* st, DevField F)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r + i >= m) return;
    const int p = st->next[j];
    uint16_t* row = work + (r + i) * kPanel;
    if (p != INT_MAX && i == p) {
        used[i] = 1;
        const int t = st->rp;  // only this thread writes the pivot list in this launch
        st->rows[t] = p;
        st->cols[t] = j;
        st->rp = t + 1;
        return;
    }
    if (used[i]) return;
    if (p != INT_MAX) {
        const uint32_t x = row[j];
        if (x) {
            const uint16_t* prow = work + (r + p) * kPanel;
            const uint32_t factor = fmul(F, x, finv(F, prow[j]));
            for (int c = j + 1; c < bc; ++c) row[c] ^= uint16_t(fmul(F, factor, prow[c]));
        }
    }
    if (j + 1 < bc && row[j + 1] != 0) atomicMin(&st->next[j + 1], int(i));
}

// W = K^{-1}, K[s][t] = orig[r + rows[s]][cols[t]] (rp x rp), by Gauss-Jordan
// on [K | I] in LDS; W is written as elements, row pitch rp.
__global__ __launch_bounds__(1024) void pivot_inverse_kernel(const uint16_t* orig, int64_t r, const PanelState* st,
                                                             int wide, void* W, DevField F)
{
    __shared__ uint16_t M[kPanel][2 * kPanel + 1];
    __shared__ int prow;
    const int rp = st->rp;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < rp * 2 * rp; idx += nt) {
        const int s = idx / (2 * rp), c = idx % (2 * rp);
        M[s][c] = c < rp ? orig[(r + st->rows[s]) * kPanel + st->cols[c]] : uint16_t(c - rp == s ? 1 : 0);
    }
    __syncthreads();
    for (int t = 0; t < rp; ++t) {
        if (tid == 0) {
            int p = t;
            while (p < rp && M[p][t] == 0) ++p;  // K is invertible: a pivot exists
            prow = p < rp ? p : t;
        }
        __syncthreads();
        const int p = prow;
        if (p != t)
            for (int c = tid; c < 2 * rp; c += nt) {
                const uint16_t a = M[p][c];
                M[p][c] = M[t][c];
                M[t][c] = a;
            }
        __syncthreads();
        const uint32_t dinv = M[t][t] ? finv(F, M[t][t]) : 0u;
        __syncthreads();
        for (int c = tid; c < 2 * rp; c += nt) M[t][c] = uint16_t(fmul(F, dinv, M[t][c]));
        __syncthreads();
        for (int idx = tid; idx < rp * 2 * rp; idx += nt) {
            const int s = idx / (2 * rp), c = idx % (2 * rp);
            if (s == t) continue;
            const uint32_t x = M[s][t];
            if (x && c != t) M[s][c] ^= uint16_t(fmul(F, x, M[t][c]));
        }
        __syncthreads();
        for (int s = tid; s < rp; s += nt)
            if (s != t) M[s][t] = 0;
        __syncthreads();
    }
    for (int idx = tid; idx < rp * rp; idx += nt) {
        const int s = idx / rp, c = idx % rp;
        st_el(W, wide, idx, M[s][rp + c]);
    }
}

// G[i][t] = original entry of (new) row i at pivot column t, for all rows:
// rows i < r are unmoved, row r + k is old row r + perm[k].  Pitch rp.
__global__ void gather_pivot_columns_kernel(const uint16_t* orig, int64_t r, int64_t m, const int* perm,
                                            const PanelState* st, int rp, int wide, void* G)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * rp) return;
    const int64_t i = idx / rp;
    const int t = int(idx % rp);
    const int64_t src = i < r ? i : r + perm[i - r];
    st_el(G, wide, idx, orig[src * kPanel + st->cols[t]]);
}

// tmp[k][c] = A[r + perm[k]][c0 + c] for k < rows, c < cols (pitch cols).
__global__ void gather_rows_kernel(const void* A, int64_t lda, int64_t r, int64_t c0, const int* perm, int64_t rows,
                                   int64_t cols, int wide, void* tmp)
{
    for (int64_t k = blockIdx.y; k < rows; k += gridDim.y) {
        const int64_t src = (r + perm[k]) * lda + c0;
        for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < cols; c += int64_t(gridDim.x) * blockDim.x)
            st_el(tmp, wide, k * cols + c, ld_el(A, wide, src + c));
    }
}

dim3 rows_grid(int64_t rows, int64_t cols)
{
    return dim3(unsigned(std::min<int64_t>(ceil_div(cols, 256), 64)), unsigned(std::min<int64_t>(rows, 65535)));
}

}  // namespace

const uint16_t* Ctx::field_tables(int e, uint32_t f)
{
    const uint64_t key = (uint64_t(e) << 32) | f;
    auto it = ftabs.find(key);
    if (it != ftabs.end()) return it->second;
    const uint32_t q = (1u << e) - 1u;
    std::vector<uint16_t> h(2 * q + (q + 1), 0);  // exp[2q] then log[q + 1]
    const uint32_t g = find_generator(e, f);
    uint32_t x = 1;
    for (uint32_t i = 0; i < q; ++i) {
        h[i] = h[i + q] = uint16_t(x);
        h[2 * q + x] = uint16_t(i);
        x = polymulmod(x, g, f, e);
    }
    void* d = nullptr;
    if (hipMalloc(&d, h.size() * sizeof(uint16_t)) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipMemcpy(d, h.data(), h.size() * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return nullptr;
    }
    ftabs[key] = static_cast<uint16_t*>(d);
    return static_cast<uint16_t*>(d);
}

int Ctx::echelon(gf2e_mat* A, int e, uint32_t f, int full, int64_t* rank, int64_t* pivots, hipStream_t s)
{
    const int64_t m = A->rows, n = A->cols;
    *rank = 0;
    if (m == 0 || n == 0) return GF2E_OK;
    const int wide = e > 8 ? 1 : 0;
    const int esz = elem_bytes(e);
    const uint16_t* tabs = field_tables(e, f);
    if (!tabs) return GF2E_ENOMEM;
    const uint32_t q = (1u << e) - 1u;
    const DevField F{tabs, tabs + 2 * q, q};

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

    // Buffers: two panel copies, used flags, panel state, permutation, W,
    // pivot-column gather, and room for rows r..m-1 of columns c0..n-1.
    auto al = [](int64_t b) { return round_up(b, 256); };
    const int64_t b_orig = al(m * kPanel * 2), b_used = al(m), b_state = al(sizeof(PanelState)),
                  b_perm = al(m * 4), b_w = al(int64_t(kPanel) * kPanel * esz), b_g = al(m * kPanel * esz),
                  b_tmp = al(m * n * esz);
    int rc = ensure_aux(2 * b_orig + b_used + b_state + b_perm + b_w + b_g + b_tmp, s);
    if (rc) return rc;
    uint8_t* base = static_cast<uint8_t*>(aux);
    uint16_t* orig = reinterpret_cast<uint16_t*>(base);
    uint16_t* work = reinterpret_cast<uint16_t*>(base + b_orig);
    uint8_t* used = base + 2 * b_orig;
    PanelState* st = reinterpret_cast<PanelState*>(base + 2 * b_orig + b_used);
    int* perm = reinterpret_cast<int*>(base + 2 * b_orig + b_used + b_state);
    uint8_t* W = base + 2 * b_orig + b_used + b_state + b_perm;
    uint8_t* G = W + b_w;
    uint8_t* tmp = G + b_g;

    PanelState hs;
    std::vector<int> hperm;
    uint8_t* Ad = static_cast<uint8_t*>(A->data);
    const int64_t lda = A->ld;
    int64_t r = 0;
    for (int64_t c0 = 0; c0 < n && r < m; c0 += kPanel) {
        const int bc = int(std::min<int64_t>(kPanel, n - c0));
        const int64_t mr = m - r;
        hipLaunchKernelGGL(panel_copy_kernel, dim3(unsigned(ceil_div(m * kPanel, 256))), dim3(256), 0, s, A->data, lda,
                           m, c0, bc, wide, orig, work);
        hipLaunchKernelGGL(panel_reset_kernel, dim3(1), dim3(128), 0, s, st);
        const dim3 g_rows(unsigned(ceil_div(mr, kStepThreads)));
        hipLaunchKernelGGL(panel_start_kernel, g_rows, dim3(kStepThreads), 0, s, work, r, m, used, st);
        for (int j = 0; j < bc; ++j)
            hipLaunchKernelGGL(panel_step_kernel, g_rows, dim3(kStepThreads), 0, s, work, r, m, j, bc, used, st, F);
        if (hipGetLastError() != hipSuccess) return GF2E_EDEVICE;
        if (hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return GF2E_EDEVICE;
        const int rp = hs.rp;
        if (rp == 0) continue;
        for (int t = 0; t < rp; ++t)
            if (pivots) pivots[r + t] = c0 + hs.cols[t];

        // New order of rows r..m-1: the pivot rows, then the others in order.
        hperm.assign(size_t(mr), 0);
        std::vector<char> is_piv(size_t(mr), 0);
        for (int t = 0; t < rp; ++t) {
            hperm[t] = hs.rows[t];
            is_piv[hs.rows[t]] = 1;
        }
        int64_t k = rp;
        for (int64_t i = 0; i < mr; ++i)
            if (!is_piv[i]) hperm[k++] = int(i);
        if (hipMemcpyAsync(perm, hperm.data(), size_t(mr) * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            return GF2E_EDEVICE;

        hipLaunchKernelGGL(pivot_inverse_kernel, dim3(1), dim3(1024), 0, s, orig, r, st, wide, W, F);
        hipLaunchKernelGGL(gather_pivot_columns_kernel, dim3(unsigned(ceil_div(m * rp, 256))), dim3(256), 0, s, orig,
                           r, m, perm, st, rp, wide, G);
        const int64_t nc = n - c0;
        hipLaunchKernelGGL(gather_rows_kernel, rows_grid(mr, nc), dim3(256), 0, s, A->data, lda, r, c0, perm, mr, nc,
                           wide, tmp);
        if (hipGetLastError() != hipSuccess) return GF2E_EDEVICE;
        if (hipMemcpy2DAsync(Ad + (r * lda + c0) * esz, size_t(lda * esz), tmp, size_t(nc * esz), size_t(nc * esz),
                             size_t(mr), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return GF2E_EDEVICE;

        // X1 = W * (pivot rows), written back over them.
        const gf2e_mat Wm{W, rp, rp, rp};
        const gf2e_mat P1{Ad + (r * lda + c0) * esz, rp, nc, lda};
        gf2e_mat X1{tmp, rp, nc, nc};
        if ((rc = mul(e, f, &Wm, &P1, &X1, s))) return rc;
        if (hipMemcpy2DAsync(Ad + (r * lda + c0) * esz, size_t(lda * esz), tmp, size_t(nc * esz), size_t(nc * esz),
                             size_t(rp), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return GF2E_EDEVICE;
        // Rows below: += Z * X1; rows above (reduced form): += Y * X1.
        if (mr > rp) {
            const gf2e_mat Z{G + (r + rp) * rp * esz, mr - rp, rp, rp};
            gf2e_mat Cb{Ad + ((r + rp) * lda + c0) * esz, mr - rp, nc, lda};
            if ((rc = mul(e, f, &Z, &P1, &Cb, s, true))) return rc;
        }
        if (full && r > 0) {
            const gf2e_mat Y{G, r, rp, rp};
            gf2e_mat Ca{Ad + c0 * esz, r, nc, lda};
            if ((rc = mul(e, f, &Y, &P1, &Ca, s, true))) return rc;
        }
        r += rp;
    }
    *rank = r;
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

}  // extern "C"
