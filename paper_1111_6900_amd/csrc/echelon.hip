// Row echelon forms over F_{2^e} (M4RIE paper, Sections 4.1 and 6): the
// reduced (or plain) row echelon form of A in place, its rank and its pivot
// columns.
//
// The paper eliminates one column at a time with Newton-John tables and, for
// speed, recurses through PLE decomposition so that most of the work becomes
// matrix products.  Here the matrix is processed in column panels of 64, and
// per panel:
//   1. pivots: a tournament over the rows r..m-1 of the panel.  Workgroups
//      of 1024 rows eliminate their rows column by column in LDS and keep
//      the rows that became pivots; the kept rows of all workgroups go
//      through the same step again until one workgroup remains, whose pivots
//      (rp of them, with their columns) are the panel's.
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
    int next[kPanel + 1];  // candidate pivot row (relative to r) of column j, INT_MAX = none
    int rows[kPanel];      // pivot t: row (relative to r) ...
    int cols[kPanel];      // ... and panel column
    int rp;                // pivots found
};

// Pivot search by tournament: each workgroup takes up to kSelRows candidate
// rows of the panel (original entries, from orig), eliminates them column by
// column in LDS and keeps the rows that became pivots (at most kPanel, in
// pivot-column order).  Any maximal independent subset of the panel's rows
// spans its row space, so the rows kept by all workgroups span it too, and a
// further level over the kept rows (until one workgroup remains) yields a
// valid pivot set with the panel's pivot columns.  Candidates are row
// indices relative to r (in == nullptr: rows 0..ncand-1; -1: an empty slot).
// A workgroup writes its kept rows to out[blockIdx.x*kPanel + t] (-1 past
// its count); the last level (final) writes the panel state instead.  The
// kernel is bound by LDS traffic (each step rewrites the remaining columns
// of every unused row).
constexpr int kSelRows = 1024;
constexpr int kSelPitch = kPanel + 2;  // halfwords per LDS row: 33 words, distinct banks

__global__ __launch_bounds__(kSelRows) void panel_select_kernel(const uint16_t* orig, int64_t r, int bc,
                                                               const int* in, int64_t ncand, int* out, int final,
                                                               PanelState* st, DevField F)
{
    __shared__ uint16_t T[kSelRows * kSelPitch];
    __shared__ uint16_t sexp[2 * 1023];
    __shared__ uint16_t slog[1024];
    __shared__ int pivs[kPanel];
    __shared__ int plog[kPanel];
    __shared__ int lead;
    const int tid = threadIdx.x;
    const int q = int(F.q);
    const int64_t slot = int64_t(blockIdx.x) * kSelRows + tid;
    const int row = slot < ncand ? (in ? in[slot] : int(slot)) : -1;
    uint16_t* mine = T + tid * kSelPitch;
    if (row >= 0) {
        const uint4* src = reinterpret_cast<const uint4*>(orig + (r + row) * kPanel);
#pragma unroll
        for (int u = 0; u < kPanel / 8; ++u) {
            const uint4 x = src[u];
            const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                mine[8 * u + 2 * h] = uint16_t(w[h]);
                mine[8 * u + 2 * h + 1] = uint16_t(w[h] >> 16);
            }
        }
    } else {
        for (int c = 0; c < kPanel; ++c) mine[c] = 0;
    }
    // tables in LDS when they fit (e <= 10), else read from the device copy
    const bool lds_tabs = q <= 1023;
    if (lds_tabs) {
        for (int k = tid; k < 2 * q; k += kSelRows) sexp[k] = F.exp[k];
        for (int k = tid; k <= q; k += kSelRows) slog[k] = F.log[k];
    }
    const uint16_t* ex = lds_tabs ? sexp : F.exp;
    const uint16_t* lg = lds_tabs ? slog : F.log;
    if (tid < kPanel) pivs[tid] = INT_MAX;
    __syncthreads();
    bool used = row < 0;
    int npiv = 0;
    {
        const uint64_t bal = __ballot(!used && mine[0] != 0);
        if (bal && tid % 64 == __ffsll(static_cast<long long>(bal)) - 1) atomicMin(&pivs[0], tid);
    }
    for (int j = 0; j < bc; ++j) {
        __syncthreads();  // pivs[j] is final, rows of step j - 1 are written
        const int p = pivs[j];
        if (p == INT_MAX) {  // no pivot in column j: offer column j + 1 as it is
            const uint64_t bal = __ballot(j + 1 < bc && !used && mine[j + 1] != 0);
            if (bal && tid % 64 == __ffsll(static_cast<long long>(bal)) - 1) atomicMin(&pivs[j + 1], tid);
            continue;
        }
        if (tid < bc) {
            const uint32_t pv = T[p * kSelPitch + tid];
            plog[tid] = pv ? int(lg[pv]) : -1;
        }
        if (tid == 0) lead = q - int(lg[T[p * kSelPitch + j]]);
        __syncthreads();
        if (tid == p) {
            used = true;
            if (final) {
                st->rows[npiv] = row;
                st->cols[npiv] = j;
            } else {
                out[int64_t(blockIdx.x) * kPanel + npiv] = row;
            }
        }
        ++npiv;  // uniform across the workgroup
        bool cand = false;
        if (!used) {
            const uint32_t x = mine[j];
            if (x) {
                int lf = int(lg[x]) + lead;
                if (lf >= q) lf -= q;
                for (int c = j + 1; c < bc; ++c) {
                    const int pl = plog[c];
                    if (pl >= 0) mine[c] ^= ex[lf + pl];
                }
            }
            cand = j + 1 < bc && mine[j + 1] != 0;
        }
        const uint64_t bal = __ballot(cand);
        if (j + 1 < bc && bal && tid % 64 == __ffsll(static_cast<long long>(bal)) - 1) atomicMin(&pivs[j + 1], tid);
    }
    if (tid == 0) {
        if (final) st->rp = npiv;
        else
            for (int t = npiv; t < kPanel; ++t) out[int64_t(blockIdx.x) * kPanel + t] = -1;
    }
}

// W = K^{-1}, K[s][t] = orig[r + rows[s]][cols[t]] (rp x rp), by Gauss-Jordan
// on [K | I] in LDS; W is written as elements, row pitch rp.  Thread (ty, tx)
// of the 8 x 128 block handles column tx of rows ty, ty + 8, ...
__global__ __launch_bounds__(1024) void pivot_inverse_kernel(const uint16_t* orig, int64_t r, const PanelState* st,
                                                             int wide, void* W, DevField Fg)
{
    constexpr int kCols = 2 * kPanel, kRowGroups = 1024 / kCols;
    __shared__ uint16_t M[kPanel][kCols + 1];
    __shared__ uint16_t sexp[2 * 1023];
    __shared__ uint16_t slog[1024];
    __shared__ int prow;
    __shared__ uint32_t pinv;
    const int rp = st->rp;
    const int tid = threadIdx.x, tx = tid % kCols, ty = tid / kCols;
    const bool lds_tabs = Fg.q <= 1023;  // tables in LDS when they fit (e <= 10)
    if (lds_tabs) {
        for (int k = tid; k < int(2 * Fg.q); k += 1024) sexp[k] = Fg.exp[k];
        for (int k = tid; k <= int(Fg.q); k += 1024) slog[k] = Fg.log[k];
    }
    const DevField F = lds_tabs ? DevField{sexp, slog, Fg.q} : Fg;
    if (tx < 2 * rp)
        for (int s = ty; s < rp; s += kRowGroups)
            M[s][tx] = tx < rp ? orig[(r + st->rows[s]) * kPanel + st->cols[tx]] : uint16_t(tx - rp == s ? 1 : 0);
    __syncthreads();
    for (int t = 0; t < rp; ++t) {
        if (tid == 0) {
            int p = t;
            while (p < rp && M[p][t] == 0) ++p;  // K is invertible: a pivot exists
            prow = p < rp ? p : t;
            pinv = p < rp ? finv(F, M[p][t]) : 0u;
        }
        __syncthreads();
        const int p = prow;
        // swap rows p and t, then scale row t so that its entry t is 1
        if (ty == 0 && tx < 2 * rp) {
            const uint16_t a = M[p][tx], b = M[t][tx];
            M[p][tx] = b;
            M[t][tx] = uint16_t(fmul(F, pinv, a));
        }
        __syncthreads();
        // eliminate column t from the other rows (column t itself last)
        uint16_t xs[kPanel / kRowGroups];
#pragma unroll
        for (int k = 0; k < kPanel / kRowGroups; ++k) {
            const int s = ty + k * kRowGroups;
            xs[k] = s < rp ? M[s][t] : 0;
        }
        __syncthreads();
        if (tx < 2 * rp) {
            const uint32_t pv = M[t][tx];
#pragma unroll
            for (int k = 0; k < kPanel / kRowGroups; ++k) {
                const int s = ty + k * kRowGroups;
                if (s < rp && s != t && xs[k]) M[s][tx] ^= uint16_t(fmul(F, xs[k], pv));
            }
        }
        __syncthreads();
    }
    if (tx < rp)
        for (int s = ty; s < rp; s += kRowGroups) st_el(W, wide, int64_t(s) * rp + tx, M[s][rp + tx]);
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

    // Buffers: the panel copy, two candidate lists of the tournament, panel
    // state, permutation, W, pivot-column gather, and room for rows r..m-1
    // of columns c0..n-1.
    auto al = [](int64_t b) { return round_up(b, 256); };
    const int64_t b_orig = al(m * kPanel * 2), b_cand = al(ceil_div(m, kSelRows) * kPanel * 4),
                  b_state = al(sizeof(PanelState)), b_perm = al(m * 4), b_w = al(int64_t(kPanel) * kPanel * esz),
                  b_g = al(m * kPanel * esz), b_tmp = al(m * n * esz);
    int rc = ensure_aux(b_orig + 2 * b_cand + b_state + b_perm + b_w + b_g + b_tmp, s);
    if (rc) return rc;
    uint8_t* base = static_cast<uint8_t*>(aux);
    uint16_t* orig = reinterpret_cast<uint16_t*>(base);
    int* cand[2] = {reinterpret_cast<int*>(base + b_orig), reinterpret_cast<int*>(base + b_orig + b_cand)};
    PanelState* st = reinterpret_cast<PanelState*>(base + b_orig + 2 * b_cand);
    int* perm = reinterpret_cast<int*>(base + b_orig + 2 * b_cand + b_state);
    uint8_t* W = base + b_orig + 2 * b_cand + b_state + b_perm;
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
                           m, c0, bc, wide, orig);
        // Tournament levels until one workgroup holds all candidates.
        const int* in = nullptr;
        int64_t ncand = mr;
        for (int level = 0;; ++level) {
            const int64_t nb = ceil_div(ncand, kSelRows);
            int* out = cand[level & 1];
            hipLaunchKernelGGL(panel_select_kernel, dim3(unsigned(nb)), dim3(kSelRows), 0, s, orig, r, bc, in, ncand,
                               out, nb == 1 ? 1 : 0, st, F);
            if (nb == 1) break;
            in = out;
            ncand = nb * kPanel;
        }
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
