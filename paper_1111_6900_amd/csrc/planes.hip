// Bandwidth-bound kernels of the product pipeline (gfx950):
//   * slicing: elements -> Karatsuba operand bit-planes (Section 3.2 slicing,
//     fused with the operand sums of the Section 5 schedule),
//   * combining: plane products -> coefficient planes -> reduction mod f ->
//     elements (the recombination and reduction of Section 5, fused with
//     clinging, the inverse of slicing).
// One thread owns one 64-bit plane word: 64 consecutive elements of a row of
// A (or of a column of B, or of a row of C).  Bits are moved between element
// bytes and plane words with 8x8 bit-matrix transposes.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gf2e_device.hpp"
#include "gf2e_internal.hpp"
#include "gf2e_schedule.hpp"

namespace gf2e {

namespace {

constexpr int kThreads = 256;

// planes[p] (p < e) of 64 elements held as bytes lo[g] / hi[g] (g < 8: eight
// elements per 64-bit group, element 8g+b in byte b).  lo holds bits 0..7 of
// each element, hi bits 8..15 (wide fields only).
template <int E>
__device__ inline void bytes_to_planes(const uint64_t (&lo)[8], const uint64_t (&hi)[8],
                                       uint64_t (&planes)[E])
{
#pragma unroll
    for (int p = 0; p < E; ++p) planes[p] = 0;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        const uint64_t y = transpose8x8(lo[g]);  // byte p = bit p of the 8 elements
#pragma unroll
        for (int p = 0; p < (E < 8 ? E : 8); ++p)
            planes[p] |= uint64_t(byte_of(y, p)) << (8 * g);
        if constexpr (E > 8) {
            const uint64_t yh = transpose8x8(hi[g]);
#pragma unroll
            for (int p = 8; p < E; ++p) planes[p] |= uint64_t(byte_of(yh, p - 8)) << (8 * g);
        }
    }
}

// Karatsuba operand planes: out[s] = XOR of planes[i] for i in u[s].
template <int E>
__device__ inline void store_operands(const uint64_t (&planes)[E], uint64_t* dst,
                                      int64_t plane_stride)
{
    constexpr Schedule S = build_schedule(E);
#pragma unroll
    for (int s = 0; s < S.t; ++s) {
        uint64_t w = 0;
#pragma unroll
        for (int i = 0; i < E; ++i)
            if ((S.u[s] >> i) & 1u) w ^= planes[i];
        dst[s * plane_stride] = w;
    }
}

// Row slicing of one plane word: row r of A, k-bits [64kw, 64kw+64).
template <int E>
__device__ __attribute__((always_inline)) inline void slice_row_word(const void* __restrict__ A, int64_t lda, int64_t m, int64_t k,
                                      uint64_t* __restrict__ planes, int64_t Mp, int64_t K64p,
                                      int* __restrict__ err, int64_t r, int64_t kw)
{
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
    uint64_t lo[8] = {}, hi[8] = {};
    bool bad = false;
    const int64_t c0 = kw * 64;
    if (r < m && c0 < k) {
        const elem_t* row = reinterpret_cast<const elem_t*>(A) + r * lda + c0;
        const int64_t valid = (k - c0) < 64 ? (k - c0) : 64;
        if constexpr (E <= 8) {
            if (valid == 64 && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
                const uint4* v = reinterpret_cast<const uint4*>(row);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint4 x = v[q];
                    lo[2 * q] = uint64_t(x.x) | (uint64_t(x.y) << 32);
                    lo[2 * q + 1] = uint64_t(x.z) | (uint64_t(x.w) << 32);
                }
            } else {
#pragma unroll
                for (int c = 0; c < 64; ++c)
                    if (c < valid) lo[c >> 3] |= uint64_t(row[c]) << (8 * (c & 7));
            }
#pragma unroll
            for (int g = 0; g < 8; ++g) bad |= bytes_out_of_field(lo[g], E);
        } else {
#pragma unroll
            for (int c = 0; c < 64; ++c) {
                if (c < valid) {
                    const uint32_t x = row[c];
                    bad |= (x >> E) != 0;
                    lo[c >> 3] |= uint64_t(x & 0xFFu) << (8 * (c & 7));
                    hi[c >> 3] |= uint64_t(x >> 8) << (8 * (c & 7));
                }
            }
        }
    }
    if (bad) atomicOr(err, 1);
    uint64_t pl[E];
    bytes_to_planes<E>(lo, hi, pl);
    store_operands<E>(pl, planes + kw * Mp + r, K64p * Mp);
}

// Column slicing of one plane word: column j of B, k-bits [64kw, 64kw+64).
// Consecutive threads take consecutive columns, so every load is coalesced.
template <int E>
__device__ __attribute__((always_inline)) inline void slice_col_word(const void* __restrict__ B, int64_t ldb, int64_t k, int64_t n,
                                      uint64_t* __restrict__ planes, int64_t Np, int64_t K64p,
                                      int* __restrict__ err, int64_t j, int64_t kw)
{
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
    uint64_t lo[8] = {}, hi[8] = {};
    bool bad = false;
    const int64_t r0 = kw * 64;
    if (j < n && r0 < k) {
        const elem_t* col = reinterpret_cast<const elem_t*>(B) + r0 * ldb + j;
        const int64_t valid = (k - r0) < 64 ? (k - r0) : 64;
#pragma unroll
        for (int c = 0; c < 64; ++c) {
            if (c < valid) {
                const uint32_t x = col[c * ldb];
                bad |= (x >> E) != 0;
                lo[c >> 3] |= uint64_t(x & 0xFFu) << (8 * (c & 7));
                if constexpr (E > 8) hi[c >> 3] |= uint64_t(x >> 8) << (8 * (c & 7));
            }
        }
    }
    if (bad) atomicOr(err, 1);
    uint64_t pl[E];
    bytes_to_planes<E>(lo, hi, pl);
    store_operands<E>(pl, planes + kw * Np + j, K64p * Np);
}

// Combine of one word: word w of row i of every product plane becomes 64
// elements of C.  k0 set: the product has an empty inner dimension, C = 0.
template <int E>
__device__ __attribute__((always_inline)) inline void combine_word(const uint64_t* __restrict__ P, int64_t Mp, int64_t ldp,
                                    int64_t n, uint32_t f, void* __restrict__ C, int64_t ldc,
                                    int64_t i, int64_t w, bool k0)
{
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
    constexpr Schedule S = build_schedule(E);
    constexpr int D = 2 * E - 1;
    uint64_t p[S.t];
#pragma unroll
    for (int s = 0; s < S.t; ++s) p[s] = k0 ? 0ull : P[s * Mp * ldp + i * ldp + w];

    // Coefficient planes of the polynomial product: C~_d = XOR_{s in w[d]} P_s.
    uint64_t c[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        uint64_t x = 0;
#pragma unroll
        for (int s = 0; s < S.t; ++s)
            if ((S.w[d] >> s) & 1u) x ^= p[s];
        c[d] = x;
    }
    // Reduction modulo f: x^d = x^(d-E) * (f - x^E) for d >= E, highest first.
    uint64_t fm[E];
#pragma unroll
    for (int b = 0; b < E; ++b) fm[b] = 0ull - uint64_t((f >> b) & 1u);
#pragma unroll
    for (int d = D - 1; d >= E; --d)
#pragma unroll
        for (int b = 0; b < E; ++b) c[d - E + b] ^= c[d] & fm[b];

    // Cling: element 64w + 8g + b takes bit (8g + b) of planes 0..E-1.
    elem_t out[64];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        uint64_t y = 0;
#pragma unroll
        for (int q = 0; q < (E < 8 ? E : 8); ++q) y |= uint64_t(byte_of(c[q], g)) << (8 * q);
        const uint64_t x = transpose8x8(y);
        uint64_t xh = 0;
        if constexpr (E > 8) {
            uint64_t yh = 0;
#pragma unroll
            for (int q = 8; q < E; ++q) yh |= uint64_t(byte_of(c[q], g)) << (8 * (q - 8));
            xh = transpose8x8(yh);
        }
#pragma unroll
        for (int b = 0; b < 8; ++b)
            out[8 * g + b] = elem_t(byte_of(x, b) | (E > 8 ? byte_of(xh, b) << 8 : 0u));
    }
    elem_t* dst = reinterpret_cast<elem_t*>(C) + i * ldc + w * 64;
    const int64_t valid = (n - w * 64) < 64 ? (n - w * 64) : 64;
    if constexpr (E <= 8) {
        if (valid == 64 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
            uint4* v = reinterpret_cast<uint4*>(dst);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t wd[4];
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    wd[h] = uint32_t(out[16 * q + 4 * h]) | (uint32_t(out[16 * q + 4 * h + 1]) << 8) |
                            (uint32_t(out[16 * q + 4 * h + 2]) << 16) |
                            (uint32_t(out[16 * q + 4 * h + 3]) << 24);
                v[q] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
            }
            return;
        }
    }
#pragma unroll
    for (int b = 0; b < 64; ++b)
        if (b < valid) dst[b] = out[b];
}

template <int E>
__global__ __launch_bounds__(kThreads) void slice_rows_kernel(
    const void* __restrict__ A, int64_t lda, int64_t m, int64_t k, uint64_t* __restrict__ planes,
    int64_t Mp, int64_t K64p, int* __restrict__ err)
{
    const int64_t r = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (r >= Mp) return;
    slice_row_word<E>(A, lda, m, k, planes, Mp, K64p, err, r, blockIdx.y);
}

template <int E>
__global__ __launch_bounds__(kThreads) void slice_cols_kernel(
    const void* __restrict__ B, int64_t ldb, int64_t k, int64_t n, uint64_t* __restrict__ planes,
    int64_t Np, int64_t K64p, int* __restrict__ err)
{
    const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (j >= Np) return;
    slice_col_word<E>(B, ldb, k, n, planes, Np, K64p, err, j, blockIdx.y);
}

template <int E>
__global__ __launch_bounds__(kThreads) void combine_kernel(
    const uint64_t* __restrict__ P, int64_t Mp, int64_t ldp, int64_t m, int64_t n, uint32_t f,
    void* __restrict__ C, int64_t ldc)
{
    const int64_t nw = (n + 63) / 64;
    const int64_t w = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (w >= nw) return;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y)
        combine_word<E>(P, Mp, ldp, n, f, C, ldc, i, w, false);
}

// ---------------------------------------------------------------------------
// Batched forms: blockIdx.y selects the product, blockIdx.x a 256-thread job
// of that product (blocks past the product's job count return at once).
// ---------------------------------------------------------------------------
#define GF2E_SWITCH_E(e, CALL) \
    switch (e) {               \
        case 2: CALL(2); break;  \
        case 3: CALL(3); break;  \
        case 4: CALL(4); break;  \
        case 5: CALL(5); break;  \
        case 6: CALL(6); break;  \
        case 7: CALL(7); break;  \
        case 8: CALL(8); break;  \
        case 9: CALL(9); break;  \
        case 10: CALL(10); break; \
        default: break;          \
    }

__global__ __launch_bounds__(kThreads) void batched_slice_kernel(const BatchProduct* __restrict__ prods,
                                                                 int* __restrict__ err)
{
    const BatchProduct& P = prods[blockIdx.y];
    int64_t job = blockIdx.x;
    if (job < P.slice_a_blocks) {
        const int64_t rb_count = P.Mp / kThreads;
        const int64_t r = (job % rb_count) * kThreads + threadIdx.x, kw = job / rb_count;
#define S_(E) slice_row_word<E>(P.A, P.lda, P.m, P.k, P.Apl, P.Mp, P.K64p, err, r, kw)
        GF2E_SWITCH_E(P.e, S_)
#undef S_
        return;
    }
    job -= P.slice_a_blocks;
    if (job < P.slice_b_blocks) {
        const int64_t cb_count = P.Np / kThreads;
        const int64_t j = (job % cb_count) * kThreads + threadIdx.x, kw = job / cb_count;
#define S_(E) slice_col_word<E>(P.B, P.ldb, P.k, P.n, P.Bpl, P.Np, P.K64p, err, j, kw)
        GF2E_SWITCH_E(P.e, S_)
#undef S_
    }
}

__global__ __launch_bounds__(kThreads) void batched_combine_kernel(const BatchProduct* __restrict__ prods)
{
    const BatchProduct& P = prods[blockIdx.y];
    if (int64_t(blockIdx.x) >= P.combine_blocks) return;
    const int64_t nw = (P.n + 63) / 64;
    const int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (idx >= P.m * nw) return;
    const int64_t i = idx / nw, w = idx % nw;
#define C_(E) combine_word<E>(P.P, P.Mp, P.Np / 64, P.n, P.f, P.C, P.ldc, i, w, P.k == 0)
    GF2E_SWITCH_E(P.e, C_)
#undef C_
}

__global__ void zero_kernel(uint8_t* C, int64_t rows, int64_t row_bytes, int64_t ld_bytes)
{
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y)
        for (int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < row_bytes;
             b += int64_t(gridDim.x) * blockDim.x)
            C[i * ld_bytes + b] = 0;
}

}  // namespace

#define GF2E_DISPATCH_E(e, CALL)         \
    switch (e) {                         \
        case 2: CALL(2); break;          \
        case 3: CALL(3); break;          \
        case 4: CALL(4); break;          \
        case 5: CALL(5); break;          \
        case 6: CALL(6); break;          \
        case 7: CALL(7); break;          \
        case 8: CALL(8); break;          \
        case 9: CALL(9); break;          \
        case 10: CALL(10); break;        \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_slice_rows(int e, const void* A, int64_t lda, int64_t m, int64_t k,
                             uint64_t* planes, int64_t Mp, int64_t K64p, int* err, hipStream_t s)
{
    if (Mp <= 0 || K64p <= 0) return hipSuccess;
    dim3 grid(unsigned(ceil_div(Mp, kThreads)), unsigned(K64p));
#define L_(E) hipLaunchKernelGGL(slice_rows_kernel<E>, grid, dim3(kThreads), 0, s, A, lda, m, k, \
                                 planes, Mp, K64p, err)
    GF2E_DISPATCH_E(e, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_slice_cols(int e, const void* B, int64_t ldb, int64_t k, int64_t n,
                             uint64_t* planes, int64_t Np, int64_t K64p, int* err, hipStream_t s)
{
    if (Np <= 0 || K64p <= 0) return hipSuccess;
    dim3 grid(unsigned(ceil_div(Np, kThreads)), unsigned(K64p));
#define L_(E) hipLaunchKernelGGL(slice_cols_kernel<E>, grid, dim3(kThreads), 0, s, B, ldb, k, n, \
                                 planes, Np, K64p, err)
    GF2E_DISPATCH_E(e, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_combine(int e, uint32_t f, const uint64_t* P, int64_t Mp, int64_t ldp, int64_t m,
                          int64_t n, void* C, int64_t ldc, hipStream_t s)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid(unsigned(ceil_div(ceil_div(n, 64), kThreads)), unsigned(m < 65535 ? m : 65535));
#define L_(E) hipLaunchKernelGGL(combine_kernel<E>, grid, dim3(kThreads), 0, s, P, Mp, ldp, m, n, \
                                 f, C, ldc)
    GF2E_DISPATCH_E(e, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_zero(void* C, int64_t rows, int64_t cols, int64_t ld, int elem_bytes,
                       hipStream_t s)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int64_t row_bytes = cols * elem_bytes;
    dim3 grid(unsigned(ceil_div(row_bytes, 256) < 64 ? ceil_div(row_bytes, 256) : 64),
              unsigned(rows < 65535 ? rows : 65535));
    hipLaunchKernelGGL(zero_kernel, grid, dim3(256), 0, s, static_cast<uint8_t*>(C), rows,
                       row_bytes, ld * elem_bytes);
    return hipGetLastError();
}

}  // namespace gf2e

namespace gf2e {

hipError_t launch_batched_slice(const BatchProduct* prods, int count, int max_blocks, int* err,
                                hipStream_t s)
{
    if (count <= 0 || max_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(batched_slice_kernel, dim3(max_blocks, count), dim3(kThreads), 0, s, prods, err);
    return hipGetLastError();
}

hipError_t launch_batched_combine(const BatchProduct* prods, int count, int max_blocks, hipStream_t s)
{
    if (count <= 0 || max_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(batched_combine_kernel, dim3(max_blocks, count), dim3(kThreads), 0, s, prods);
    return hipGetLastError();
}

int batch_threads_per_block() { return kThreads; }

}  // namespace gf2e
