// Triangular solving with matrices over F_{2^e} (M4RIE paper, Section 4.3):
// X = T^{-1} B for a triangular m x m matrix T, B overwritten by X.
//
// The paper's algorithm walks the rows one by one and updates the rows above
// with Newton-John tables.  Here the solve is blocked for the GPU:
//   1. one kernel inverts all 128 x 128 diagonal blocks of T at once (one
//      workgroup of 1024 threads per block, right-looking substitution with
//      the block in registers, field products by log/antilog tables, in LDS
//      for e <= 10);
//   2. a recursion over block ranges turns the rest into products on the
//      bitsliced path: for upper T,
//          X2 = solve(T22, B2);  B1 += T12 * X2;  X1 = solve(T11, B1),
//      and a single block row is X_q = inv(T_qq) * B_q.
// Every update is a gf2e product (C += A*B), so almost all of the work runs
// on the matrix cores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "ctx.hpp"
#include "field.hpp"
#include "gf2e.h"
#include "gf2e_internal.hpp"

namespace gf2e {

namespace {

constexpr int kTrsmBlock = 128;  // diagonal block size = threads per workgroup

// Inverse of diagonal block q of T (rows and columns [128q, 128q + bs)),
// written row-major with leading dimension 128 at Tinv + 128q*128 (columns
// < bs).  Right-looking substitution on T_qq X = I: step i (i ascending for
// lower T, descending for upper) finishes row i of X as R_i / T_ii, then
// every row j still to come takes R_j -= T_ji X_i.  Thread (ty, c) of the
// 8 x 128 block keeps column c of R for rows ty, ty + 8, ... in registers;
// per step the new row of X passes through LDS (as logarithms, double-
// buffered), so a step costs one barrier and 16 independent table lookups per
// thread.  The triangle of T is staged once as logarithms.  Field products
// use the device tables (exp with a zero tail, log 0 = 2q), in LDS for
// e <= 10.  Only the triangle of T is read; unit = 1 takes the diagonal as
// ones.  Flags: err |= 1 for an entry >= 2^E, err |= 2 for a zero on the
// diagonal.
constexpr int kInvGroups = 8;  // threads per column
constexpr int kInvThreads = kTrsmBlock * kInvGroups;

template <int E>
__global__ __launch_bounds__(kInvThreads) void trsm_invert_kernel(const void* __restrict__ Tm, int64_t ldt,
                                                                  int64_t m, int lower, int unit,
                                                                  const uint16_t* __restrict__ dexp,
                                                                  const uint32_t* __restrict__ dlog,
                                                                  void* __restrict__ Tinv, int* __restrict__ err)
{
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
    constexpr int Q = (1 << E) - 1, RPT = kTrsmBlock / kInvGroups;
    constexpr bool kLds = E <= 10;
    __shared__ uint16_t sexp[kLds ? 4 * Q + 1 : 1];
    __shared__ uint32_t slog[kLds ? Q + 1 : 1];
    __shared__ uint32_t LT[kTrsmBlock][kTrsmBlock + 1];  // log T[i][l] (2q for zeros and outside)
    __shared__ uint32_t dlinv[kTrsmBlock];               // log of 1 / T[i][i] (0 for a unit diagonal)
    __shared__ uint32_t xlog[2][kTrsmBlock];             // log X[i][c] of the newest row
    const int tid = threadIdx.x, c = tid % kTrsmBlock, ty = tid / kTrsmBlock;
    if constexpr (kLds) {
        for (int k = tid; k <= 4 * Q; k += kInvThreads) sexp[k] = dexp[k];
        for (int k = tid; k <= Q; k += kInvThreads) slog[k] = dlog[k];
        __syncthreads();
    }
    const uint16_t* ex = kLds ? sexp : dexp;
    const uint32_t* lg = kLds ? slog : dlog;

    const int64_t r0 = int64_t(blockIdx.x) * kTrsmBlock;
    const int bs = int(m - r0 < kTrsmBlock ? m - r0 : kTrsmBlock);
    const elem_t* T = static_cast<const elem_t*>(Tm);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int i = ty + kInvGroups * k;
        uint32_t v = 0;
        if (i < bs && c < bs && (lower ? c < i : c > i)) {  // the strict triangle
            v = T[(r0 + i) * ldt + r0 + c];
            bad |= (v >> E) != 0;
            v &= uint32_t(Q);
        }
        LT[i][c] = lg[v];
    }
    if (ty == 0) {
        uint32_t d = 1;
        if (!unit && c < bs) {
            d = T[(r0 + c) * ldt + r0 + c];
            bad |= (d >> E) != 0;
            d &= uint32_t(Q);
            if (d == 0) atomicOr(err, 2);
        }
        const uint32_t ld = lg[d];
        dlinv[c] = d ? (uint32_t(Q) - ld) % uint32_t(Q) : uint32_t(2 * Q);
    }
    if (bad) atomicOr(err, 1);
    __syncthreads();

    uint32_t R[RPT];  // R[k]: column c of row ty + 8k, initially the identity
#pragma unroll
    for (int k = 0; k < RPT; ++k) R[k] = ty + kInvGroups * k == c ? 1u : 0u;
    elem_t* out = static_cast<elem_t*>(Tinv) + r0 * kTrsmBlock;
    for (int step = 0; step < bs; ++step) {
        const int i = lower ? step : bs - 1 - step;
        const int b = step & 1;
        if (ty == i % kInvGroups) {  // row i is final: X[i][c] = R_i / T_ii
            const int ki = i / kInvGroups;
            uint32_t r = 0;
#pragma unroll
            for (int k = 0; k < RPT; ++k) r = k == ki ? R[k] : r;
            const uint32_t x = ex[lg[r] + dlinv[i]];
            if (c < bs) out[int64_t(i) * kTrsmBlock + c] = elem_t(x);
            xlog[b][c] = lg[x];
        }
        __syncthreads();
        const uint32_t lx = xlog[b][c];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int j = ty + kInvGroups * k;
            const uint32_t d = ex[LT[j][i] + lx];
            R[k] = (lower ? j > i : j < i) ? R[k] ^ d : R[k];
        }
    }
}

template <int E, class Fn>
bool with_e_host(int e, Fn& fn)
{
    if constexpr (E > kMaxE) {
        return false;
    } else {
        if (e == E) {
            fn.template operator()<E>();
            return true;
        }
        return with_e_host<E + 1>(e, fn);
    }
}

hipError_t launch_trsm_invert(int e, DevTables tabs, int lower, int unit, const void* T, int64_t ldt,
                              int64_t m, void* Tinv, int* err, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    const dim3 grid(unsigned(ceil_div(m, kTrsmBlock)));
    auto go = [&]<int E>() {
        hipLaunchKernelGGL((trsm_invert_kernel<E>), grid, dim3(kInvThreads), 0, s, T, ldt, m, lower, unit, tabs.exp,
                           tabs.log, Tinv, err);
    };
    if (!with_e_host<2>(e, go)) return hipErrorInvalidValue;
    return hipGetLastError();
}

gf2e_mat sub(const gf2e_mat* M, int esz, int64_t r, int64_t c, int64_t rows, int64_t cols)
{
    gf2e_mat s;
    s.data = static_cast<uint8_t*>(M->data) + (r * M->ld + c) * esz;
    s.rows = rows;
    s.cols = cols;
    s.ld = M->ld;
    return s;
}

}  // namespace

int Ctx::ensure_aux(int64_t bytes, hipStream_t s)
{
    if (bytes <= aux_bytes) return GF2E_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cs);
    if (cs != hipStreamCaptureStatusNone) return GF2E_ENOMEM;
    if (aux) {
        if (hipDeviceSynchronize() != hipSuccess) return GF2E_EDEVICE;
        (void)hipFree(aux);
        aux = nullptr;
        aux_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, size_t(bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return GF2E_ENOMEM;
    }
    aux = p;
    aux_bytes = bytes;
    return GF2E_OK;
}

int Ctx::trsm(int lower, int unit, const gf2e_mat* T, gf2e_mat* B, int e, uint32_t f, hipStream_t s)
{
    const int64_t m = T->rows, n = B->cols;
    if (m == 0 || n == 0) return GF2E_OK;
    const int esz = elem_bytes(e);
    const int64_t nb = ceil_div(m, kTrsmBlock);
    const int64_t inv_bytes = round_up(nb * kTrsmBlock * kTrsmBlock * esz, 256);
    int rc = ensure_aux(inv_bytes, s);
    if (rc) return rc;
    uint8_t* Tinv = static_cast<uint8_t*>(aux);
    const DevTables tabs = field_tables(e, f);
    if (!tabs.exp) return GF2E_ENOMEM;
    if (launch_trsm_invert(e, tabs, lower, unit, T->data, T->ld, m, Tinv, d_err, s) != hipSuccess) return GF2E_EDEVICE;

    const gf2e_mat inv_all{Tinv, nb * kTrsmBlock, kTrsmBlock, kTrsmBlock};
    // Solve block rows [q0, q1).
    auto solve = [&](auto&& self, int64_t q0, int64_t q1) -> int {
        const int64_t R0 = q0 * kTrsmBlock, R1 = std::min(m, q1 * kTrsmBlock);
        if (q1 - q0 == 1) {
            // X_q = inv(T_qq) * B_q in place: the product slices B_q into its
            // planes before its last kernel writes C, all in stream order.
            const int64_t bs = R1 - R0;
            const gf2e_mat Ti = sub(&inv_all, esz, R0, 0, bs, bs);
            const gf2e_mat Bq = sub(B, esz, R0, 0, bs, n);
            gf2e_mat Xq = Bq;
            return mul(e, f, &Ti, &Bq, &Xq, s);
        }
        const int64_t mid = (q0 + q1) / 2, Rm = mid * kTrsmBlock;
        int r;
        if (!lower) {
            if ((r = self(self, mid, q1))) return r;
            const gf2e_mat A = sub(T, esz, R0, Rm, Rm - R0, R1 - Rm);
            const gf2e_mat X2 = sub(B, esz, Rm, 0, R1 - Rm, n);
            gf2e_mat B1 = sub(B, esz, R0, 0, Rm - R0, n);
            if ((r = mul(e, f, &A, &X2, &B1, s, true))) return r;
            return self(self, q0, mid);
        }
        if ((r = self(self, q0, mid))) return r;
        const gf2e_mat A = sub(T, esz, Rm, R0, R1 - Rm, Rm - R0);
        const gf2e_mat X1 = sub(B, esz, R0, 0, Rm - R0, n);
        gf2e_mat B2 = sub(B, esz, Rm, 0, R1 - Rm, n);
        if ((r = mul(e, f, &A, &X1, &B2, s, true))) return r;
        return self(self, mid, q1);
    };
    return solve(solve, 0, nb);
}

}  // namespace gf2e

using namespace gf2e;

extern "C" {

int gf2e_mul_add_async(gf2e_ctx* handle, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e, uint32_t f,
                       void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    int rc = validate_mul(A, B, C, e, f);
    if (rc) return rc;
    if (A->rows == 0 || B->cols == 0 || A->cols == 0) return GF2E_OK;  // C += 0
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    c->order_stream(s);
    rc = c->mul(e, f, A, B, C, s, true);
    c->mark_used(s);
    return rc;
}

int gf2e_mul_add(gf2e_ctx* handle, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e, uint32_t f)
{
    int rc = gf2e_mul_add_async(handle, A, B, C, e, f, nullptr);
    if (rc) return rc;
    return gf2e_sync(handle, nullptr);
}

int gf2e_trsm_async(gf2e_ctx* handle, int lower, int unit, const gf2e_mat* T, gf2e_mat* B, int e, uint32_t f,
                    void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    int rc;
    if ((rc = check_mat(T)) || (rc = check_mat(B))) return rc;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    if (T->rows != T->cols || B->rows != T->rows) return GF2E_ESHAPE;
    if (overlaps(B, T, elem_bytes(e))) return GF2E_EALIAS;
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    c->order_stream(s);
    rc = c->trsm(lower != 0, unit != 0, T, B, e, f, s);
    c->mark_used(s);
    return rc;
}

int gf2e_trsm(gf2e_ctx* handle, int lower, int unit, const gf2e_mat* T, gf2e_mat* B, int e, uint32_t f)
{
    int rc = gf2e_trsm_async(handle, lower, unit, T, B, e, f, nullptr);
    if (rc) return rc;
    return gf2e_sync(handle, nullptr);
}

}  // extern "C"
