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

// Row slicing: thread (r, kw) reads A[r][64kw .. 64kw+63].
template <int E>
__global__ __launch_bounds__(kThreads) void slice_rows_kernel(
    const void* __restrict__ A, int64_t lda, int64_t m, int64_t k, uint64_t* __restrict__ planes,
    int64_t Mp, int64_t K64p, int* __restrict__ err)
{
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
    const int64_t r = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t kw = blockIdx.y;
    if (r >= Mp) return;
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
                for (int64_t c = 0; c < valid; ++c)
                    lo[c >> 3] |= uint64_t(row[c]) << (8 * (c & 7));
            }
#pragma unroll
            for (int g = 0; g < 8; ++g) bad |= bytes_out_of_field(lo[g], E);
        } else {
            for (int64_t c = 0; c < valid; ++c) {
                const uint32_t x = row[c];
                bad |= (x >> E) != 0;
                lo[c >> 3] |= uint64_t(x & 0xFFu) << (8 * (c & 7));
                hi[c >> 3] |= uint64_t(x >> 8) << (8 * (c & 7));
            }
        }
    }
    if (bad) atomicOr(err, 1);
    uint64_t pl[E];
    bytes_to_planes<E>(lo, hi, pl);
    store_operands<E>(pl, planes + kw * Mp + r, K64p * Mp);
}

// Column slicing: thread (j, kw) reads B[64kw .. 64kw+63][j]; consecutive
// threads take consecutive columns, so every load instruction is coalesced.
template <int E>
__global__ __launch_bounds__(kThreads) void slice_cols_kernel(
    const void* __restrict__ B, int64_t ldb, int64_t k, int64_t n, uint64_t* __restrict__ planes,
    int64_t Np, int64_t K64p, int* __restrict__ err)
{
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
    const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t kw = blockIdx.y;
    if (j >= Np) return;
    uint64_t lo[8] = {}, hi[8] = {};
    bool bad = false;
    const int64_t r0 = kw * 64;
    if (j < n && r0 < k) {
        const elem_t* col = reinterpret_cast<const elem_t*>(B) + r0 * ldb + j;
        const int64_t valid = (k - r0) < 64 ? (k - r0) : 64;
        if (valid == 64) {
#pragma unroll
            for (int c = 0; c < 64; ++c) {
                const uint32_t x = col[c * ldb];
                bad |= (x >> E) != 0;
                lo[c >> 3] |= uint64_t(x & 0xFFu) << (8 * (c & 7));
                if constexpr (E > 8) hi[c >> 3] |= uint64_t(x >> 8) << (8 * (c & 7));
            }
        } else {
            for (int64_t c = 0; c < valid; ++c) {
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

// Combine: thread (i, w) turns word w of row i of every product plane into
// 64 elements of C.
template <int E>
__global__ __launch_bounds__(kThreads) void combine_kernel(
    const uint64_t* __restrict__ P, int64_t Mp, int64_t ldp, int64_t m, int64_t n, uint32_t f,
    void* __restrict__ C, int64_t ldc)
{
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
    constexpr Schedule S = build_schedule(E);
    constexpr int D = 2 * E - 1;
    const int64_t nw = (n + 63) / 64;
    const int64_t w = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (w >= nw) return;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y) {
    uint64_t p[S.t];
#pragma unroll
    for (int s = 0; s < S.t; ++s) p[s] = P[s * Mp * ldp + i * ldp + w];

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
            continue;
        }
    }
    for (int b = 0; b < valid; ++b) dst[b] = out[b];
    }
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
