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

#include <algorithm>
#include <type_traits>

#include "cling.hpp"
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

// Operand planes of the schedule: out[s] = XOR of planes[i] for i in u[s]
// (A side) or v[s] (B side).
template <int E, int SID, bool BSIDE>
__device__ inline void store_operands(const uint64_t (&planes)[E], uint64_t* dst,
                                      int64_t plane_stride)
{
    constexpr KernelSchedule S = kernel_schedule(E, SID);
    static_assert(S.e == E, "schedule and field size differ");
#pragma unroll
    for (int s = 0; s < S.t; ++s) {
        uint64_t w = 0;
#pragma unroll
        for (int i = 0; i < E; ++i)
            if (((BSIDE ? S.v[s] : S.u[s]) >> i) & 1u) w ^= planes[i];
        dst[s * plane_stride] = w;
    }
}

// Loads nbytes (at most 16) bytes at p, zero beyond, with the aligned
// dwords that hold them: p need not be aligned, and no dword is read that
// holds none of the bytes (so nothing outside the buffer's aligned words).
__device__ __attribute__((always_inline)) inline uint4 load16_any(const uint8_t* p, int nbytes)
{
    const uintptr_t pa = reinterpret_cast<uintptr_t>(p);
    const uint32_t* w = reinterpret_cast<const uint32_t*>(pa & ~uintptr_t(3));
    const int off = int(pa & 3);
    uint32_t d[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) d[i] = 4 * i < off + nbytes ? w[i] : 0u;
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t x = __builtin_amdgcn_alignbyte(d[j + 1], d[j], uint32_t(off));
        const int b = nbytes - 4 * j;
        o[j] = b >= 4 ? x : b <= 0 ? 0u : x & ((1u << (8 * b)) - 1u);
    }
    return make_uint4(o[0], o[1], o[2], o[3]);
}

// Row slicing of one plane word: row r of A, k-bits [64kw, 64kw+64).
template <int E, int SID>
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
        const int valid = int((k - c0) < 64 ? (k - c0) : 64);
        // 16-byte pieces of the row: vector loads when aligned and whole,
        // else the aligned dwords that hold the piece's valid bytes
        constexpr int EB = int(sizeof(elem_t)), NQ = 4 * EB;
        const uint8_t* rb = reinterpret_cast<const uint8_t*>(row);
        const bool fast = valid == 64 && (reinterpret_cast<uintptr_t>(rb) & 15) == 0;
        uint4 q[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i)
            q[i] = fast ? reinterpret_cast<const uint4*>(rb)[i] : load16_any(rb + 16 * i, valid * EB - 16 * i);
        if constexpr (E <= 8) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                lo[2 * i] = uint64_t(q[i].x) | (uint64_t(q[i].y) << 32);
                lo[2 * i + 1] = uint64_t(q[i].z) | (uint64_t(q[i].w) << 32);
            }
#pragma unroll
            for (int g = 0; g < 8; ++g) bad |= bytes_out_of_field(lo[g], E);
        } else {
            // piece i holds elements 8i..8i+7 as uint16: split low and high bytes
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t w4[4] = {q[i].x, q[i].y, q[i].z, q[i].w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    bad |= ((w4[h] & 0xFFFFu) >> E) != 0 || ((w4[h] >> 16) >> E) != 0;
                    lo[i] |= uint64_t((w4[h] & 0xFFu) | ((w4[h] >> 8) & 0xFF00u)) << (16 * h);
                    hi[i] |= uint64_t(((w4[h] >> 8) & 0xFFu) | ((w4[h] >> 16) & 0xFF00u)) << (16 * h);
                }
            }
        }
    }
    if (bad) atomicOr(err, 1);
    uint64_t pl[E];
    bytes_to_planes<E>(lo, hi, pl);
    store_operands<E, SID, false>(pl, planes + kw * Mp + r, K64p * Mp);
}

// Bit-planes of one column word for a block of 64 columns (one wave per
// block): the 64 x 64 tile of B (k-bits [64kw, 64kw+64), columns
// j0..j0+63) is read with 16-byte row pieces where they are aligned, staged
// in LDS row-major (tile_mem: col_tile_bytes of LDS for this wave), and each
// lane then reads its own column from LDS.  That replaces 64 narrow global
// loads per lane by a few wide ones.  Every thread of the block calls it.
// LDS bytes of one wave's tile for elements of EB bytes (rows padded by 16).
constexpr int col_tile_bytes(int EB) { return 64 * (64 * EB + 16); }

template <int E>
__device__ __attribute__((always_inline)) inline void load_col_planes_tile(const void* __restrict__ B, int64_t ldb,
                                                                            int64_t k, int64_t n,
                                                                            int* __restrict__ err, int64_t j0,
                                                                            int64_t kw, int lane, uint8_t* tile_mem,
                                                                            uint64_t (&pl)[E])
{
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
    constexpr int EB = int(sizeof(elem_t)), RB = 64 * EB, CH = RB / 16, PE = 16 / EB;
    auto tile = reinterpret_cast<uint8_t(*)[RB + 16]>(tile_mem);  // this wave's 64 rows
    const elem_t* base = static_cast<const elem_t*>(B);
    const int64_t r0 = kw * 64;
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        const int q = lane + 64 * i, row = q / CH, pc = q % CH;
        const int64_t gr = r0 + row, gc = j0 + int64_t(pc) * PE;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gr < k && gc < n) {
            const elem_t* src = base + gr * ldb + gc;
            if (gc + PE <= n && (reinterpret_cast<uintptr_t>(src) & 15) == 0)
                v = *reinterpret_cast<const uint4*>(src);
            else
                v = load16_any(reinterpret_cast<const uint8_t*>(src), int(n - gc < PE ? n - gc : PE) * EB);
        }
        *reinterpret_cast<uint4*>(&tile[row][pc * 16]) = v;
    }
    __syncthreads();
    uint64_t lo[8] = {}, hi[8] = {};
    bool bad = false;
    // bit c of the column word takes k-row b_side_bit(c) of the tile
#pragma unroll
    for (int c = 0; c < 64; ++c) {
        const uint32_t x = reinterpret_cast<const elem_t*>(tile[b_side_bit(c)])[lane];
        bad |= (x >> E) != 0;
        lo[c >> 3] |= uint64_t(x & 0xFFu) << (8 * (c & 7));
        if constexpr (E > 8) hi[c >> 3] |= uint64_t(x >> 8) << (8 * (c & 7));
    }
    if (bad) atomicOr(err, 1);
    bytes_to_planes<E>(lo, hi, pl);
}

// Alpha-power slicing of one column word (alpha = x, the class of x in
// F_2[x]/<f>).  With C_c = sum_i A_i * (plane c of alpha^i B), the product
// becomes one GF(2) product of [A_0 .. A_{E-1}] (m x Ek) with the Ek x En
// matrix whose block (i, c) is plane c of alpha^i B; the reduction modulo f
// is folded into that matrix.  Block (i, c), word (kw, j) is stored at
// planes[(i*K64p + kw)*E*Np + c*Np + j].  alpha^(i+1) B = x * alpha^i B on
// bit-planes: shift up by one and fold the plane that leaves back in with f.
// This writes the blocks (i, c) of column j, k-word kw, from the bit-planes
// cur of B (cur is consumed).
template <int E>
__device__ __attribute__((always_inline)) inline void store_alpha_blocks(uint64_t (&cur)[E], uint32_t f,
                                                                          uint64_t* __restrict__ planes, int64_t Np,
                                                                          int64_t K64p, int64_t j, int64_t kw)
{
    uint64_t fm[E];
#pragma unroll
    for (int b = 0; b < E; ++b) fm[b] = 0ull - uint64_t((f >> b) & 1u);
    const int64_t ld = int64_t(E) * Np;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        uint64_t* row = planes + (int64_t(i) * K64p + kw) * ld + j;
#pragma unroll
        for (int c = 0; c < E; ++c) row[int64_t(c) * Np] = cur[c];
        if (i + 1 < E) {
            const uint64_t top = cur[E - 1];
#pragma unroll
            for (int b = E - 1; b > 0; --b) cur[b] = cur[b - 1] ^ (top & fm[b]);
            cur[0] = top & fm[0];
        }
    }
}

// Combine of one word: word w of row i of every product plane becomes 64
// elements of C.  Product s, row i, word w is at P[s*pstride + i*ldp + w].
// k0 set: the product has an empty inner dimension, C = 0.  acc set: the
// result is added to C (C += A*B) instead of replacing it.
template <int E, int SID>
__device__ __attribute__((always_inline)) inline void combine_word(const uint64_t* __restrict__ P, int64_t pstride,
                                    int64_t ldp, int64_t n, uint32_t f, void* __restrict__ C,
                                    int64_t ldc, int64_t i, int64_t w, bool k0, bool acc = false)
{
    constexpr KernelSchedule S = kernel_schedule(E, SID);
    constexpr int D = 2 * E - 1;
    // Products are streamed into the planes they feed, so only the 2e-1
    // coefficient planes (or e result planes) are live, whatever t is.
    uint64_t c[D];
#pragma unroll
    for (int d = 0; d < D; ++d) c[d] = 0;
#pragma unroll
    for (int s = 0; s < S.t; ++s) {
        const uint64_t ps = k0 ? 0ull : P[s * pstride + i * ldp + w];
        if constexpr (S.folded) {
            // The schedule already reduces modulo its f: plane q is the XOR
            // of the products whose output set holds q.
#pragma unroll
            for (int q = 0; q < E; ++q)
                if ((S.c[s] >> q) & 1u) c[q] ^= ps;
        } else {
            // Coefficient planes of the polynomial product: C~_d = XOR_{s in w[d]} P_s.
#pragma unroll
            for (int d = 0; d < D; ++d)
                if ((S.w[d] >> s) & 1u) c[d] ^= ps;
        }
    }
    if constexpr (!S.folded) {
        // Reduction modulo f: x^d = x^(d-E) * (f - x^E) for d >= E, highest first.
        uint64_t fm[E];
#pragma unroll
        for (int b = 0; b < E; ++b) fm[b] = 0ull - uint64_t((f >> b) & 1u);
#pragma unroll
        for (int d = D - 1; d >= E; --d)
#pragma unroll
            for (int b = 0; b < E; ++b) c[d - E + b] ^= c[d] & fm[b];
    }

    cling_store<E>(c, n, C, ldc, i, w, acc);
}

template <int E, int SID>
__global__ __launch_bounds__(kThreads) void slice_rows_kernel(
    const void* __restrict__ A, int64_t lda, int64_t m, int64_t k, uint64_t* __restrict__ planes,
    int64_t Mp, int64_t K64p, int* __restrict__ err)
{
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= Mp) return;
    slice_row_word<E, SID>(A, lda, m, k, planes, Mp, K64p, err, r, blockIdx.y);
}

// Column slicing: one wave per block of 64 columns and one k-word.
constexpr int kColBlock = 64;

template <int E, int SID>
__global__ __launch_bounds__(kColBlock) void slice_cols_kernel(
    const void* __restrict__ B, int64_t ldb, int64_t k, int64_t n, uint64_t* __restrict__ planes,
    int64_t Np, int64_t K64p, int* __restrict__ err)
{
    __shared__ __align__(16) uint8_t tile[col_tile_bytes(E > 8 ? 2 : 1)];
    const int64_t j0 = int64_t(blockIdx.x) * kColBlock, kw = blockIdx.y;
    uint64_t pl[E];
    load_col_planes_tile<E>(B, ldb, k, n, err, j0, kw, threadIdx.x, tile, pl);
    store_operands<E, SID, true>(pl, planes + kw * Np + j0 + threadIdx.x, K64p * Np);
}

template <int E>
__global__ __launch_bounds__(kColBlock) void slice_cols_alpha_kernel(
    const void* __restrict__ B, int64_t ldb, int64_t k, int64_t n, uint32_t f, uint64_t* __restrict__ planes,
    int64_t Np, int64_t K64p, int* __restrict__ err)
{
    __shared__ __align__(16) uint8_t tile[col_tile_bytes(E > 8 ? 2 : 1)];
    const int64_t j0 = int64_t(blockIdx.x) * kColBlock, kw = blockIdx.y;
    uint64_t cur[E];
    load_col_planes_tile<E>(B, ldb, k, n, err, j0, kw, threadIdx.x, tile, cur);
    store_alpha_blocks<E>(cur, f, planes, Np, K64p, j0 + threadIdx.x, kw);
}

template <int E, int SID>
__global__ __launch_bounds__(kThreads) void combine_kernel(
    const uint64_t* __restrict__ P, int64_t pstride, int64_t ldp, int64_t m, int64_t n, uint32_t f,
    void* __restrict__ C, int64_t ldc, int acc)
{
    const int64_t nw = (n + 63) / 64;
    const int64_t w = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (w >= nw) return;
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y)
        combine_word<E, SID>(P, pstride, ldp, n, f, C, ldc, i, w, false, acc != 0);
}

// ---------------------------------------------------------------------------
// Batched forms: blockIdx.y selects the product, blockIdx.x a 256-thread job
// of that product (blocks past the product's job count return at once).
// ---------------------------------------------------------------------------
// Calls fn.template operator()<E>() for e in [E, EMAX].
template <int E, int EMAX, class Fn>
__host__ __device__ inline bool with_e_in(int e, Fn&& fn)
{
    if constexpr (E > EMAX) {
        return false;
    } else {
        if (e == E) {
            fn.template operator()<E>();
            return true;
        }
        return with_e_in<E + 1, EMAX>(e, fn);
    }
}

template <class Fn>
__host__ __device__ inline bool with_e(int e, Fn&& fn)
{
    return with_e_in<2, kMaxE>(e, fn);
}

// Calls fn.template operator()<E, SID>() for the schedule of (e, sid): field
// schedule sid (>= 0, when its e is in [EMIN, EMAX]) or the Karatsuba
// schedule (sid < 0) for e in [EMIN, EMAX].
template <int I, int EMIN, int EMAX, class Fn>
__host__ __device__ inline bool with_field_schedule(int sid, Fn& fn)
{
    if constexpr (I < kNumFieldSchedules) {
        if constexpr (kFieldSchedules[I].e >= EMIN && kFieldSchedules[I].e <= EMAX) {
            if (sid == I) {
                fn.template operator()<kFieldSchedules[I].e, I>();
                return true;
            }
        }
        return with_field_schedule<I + 1, EMIN, EMAX>(sid, fn);
    } else {
        return false;
    }
}

template <int EMIN = 2, int EMAX = kMaxE, class Fn>
__host__ __device__ inline bool with_schedule(int e, int sid, Fn&& fn)
{
    if (sid >= 0) return with_field_schedule<0, EMIN, EMAX>(sid, fn);
    return with_e_in<EMIN, EMAX>(e, [&]<int E>() { fn.template operator()<E, -1>(); });
}

// As with_schedule, and sid = kIdentitySchedule too (host launches only, so
// the batched kernels do not carry the identity instantiations).
template <class Fn>
inline bool with_any_schedule(int e, int sid, Fn&& fn)
{
    if (sid == kIdentitySchedule)
        return with_e(e, [&]<int E>() { fn.template operator()<E, kIdentitySchedule>(); });
    return with_schedule(e, sid, fn);
}

// The batched kernels are instantiated for two ranges of e, so that the
// large fields do not raise the register use of the kernels that serve the
// common small ones; each launch skips the products outside its range.
constexpr int kSmallE = kBatchSmallE;

// Index i with first[i] <= b < first[i + 1] (b is uniform in the block, so
// the search runs on scalar loads).
__device__ inline int job_owner(const int* __restrict__ first, int n, int b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int EMIN, int EMAX>
__global__ __launch_bounds__(kThreads) void batched_slice_kernel(const BatchProduct* __restrict__ prods,
                                                                 const int* __restrict__ first,
                                                                 const int* __restrict__ owner, int nprod,
                                                                 int* __restrict__ err)
{
    const int b = int(blockIdx.x), i = job_owner(first, nprod, b);
    const BatchProduct& P = prods[owner[i]];
    if (P.e < EMIN || P.e > EMAX) return;
    int64_t job = b - first[i];
    // Rows past m and columns past n are not written: they only feed product
    // rows and columns that the combine never reads (the padding of k, which
    // enters every product, is written as zeros).
    if (job < P.slice_a_blocks) {
        const int64_t rb_count = P.Mp / kThreads;
        const int64_t r = (job % rb_count) * kThreads + threadIdx.x, kw = job / rb_count;
        if (r >= P.m) return;
        with_schedule<EMIN, EMAX>(P.e, P.sid, [&]<int E, int SID>() {
            slice_row_word<E, SID>(P.A, P.lda, P.m, P.k, P.Apl, P.Mp, P.K64p, err, r, kw);
        });
        return;
    }
    job -= P.slice_a_blocks;
    if (job < P.slice_b_blocks) {
        // 256 consecutive columns of one k-word; each wave slices 64 of them
        // through its own LDS tile (the branch is uniform in the block)
        __shared__ __align__(16) uint8_t tiles[kThreads / 64][col_tile_bytes(EMAX > 8 ? 2 : 1)];
        const int64_t cb_count = P.Np / kThreads;
        const int wave = int(threadIdx.x) / 64, lane = int(threadIdx.x) % 64;
        const int64_t j0 = (job % cb_count) * kThreads + 64 * wave, kw = job / cb_count;
        with_schedule<EMIN, EMAX>(P.e, P.sid, [&]<int E, int SID>() {
            uint64_t pl[E];
            load_col_planes_tile<E>(P.B, P.ldb, P.k, P.n, err, j0, kw, lane, tiles[wave], pl);
            if (j0 + lane < P.n) store_operands<E, SID, true>(pl, P.Bpl + kw * P.Np + j0 + lane, P.K64p * P.Np);
        });
    }
}

template <int EMIN, int EMAX>
__global__ __launch_bounds__(kThreads) void batched_combine_kernel(const BatchProduct* __restrict__ prods,
                                                                   const int* __restrict__ first,
                                                                   const int* __restrict__ owner, int nprod)
{
    const int b = int(blockIdx.x), j = job_owner(first, nprod, b);
    const BatchProduct& P = prods[owner[j]];
    if (P.e < EMIN || P.e > EMAX) return;
    const int64_t nw = (P.n + 63) / 64;
    const int64_t idx = int64_t(b - first[j]) * kThreads + threadIdx.x;
    if (idx >= P.m * nw) return;
    const int64_t i = idx / nw, w = idx % nw;
    with_schedule<EMIN, EMAX>(P.e, P.sid, [&]<int E, int SID>() {
        combine_word<E, SID>(P.P, P.Mp * (P.Np / 64), P.Np / 64, P.n, P.f, P.C, P.ldc, i, w, P.k == 0);
    });
}

// Pseudo-random field elements (a 64-bit mix of the index and the seed,
// masked to e bits), used as tuning inputs so the timed kernels see data of
// realistic density.
__global__ void fill_elements_kernel(void* X, int64_t count, int elem_bytes, uint32_t mask, uint64_t seed)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * blockDim.x) {
        uint64_t z = uint64_t(i) + seed * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const uint32_t v = uint32_t(z) & mask;
        if (elem_bytes == 1) static_cast<uint8_t*>(X)[i] = uint8_t(v);
        else static_cast<uint16_t*>(X)[i] = uint16_t(v);
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

// Threads per block of a slicing launch over `words` plane words (one per
// thread): small launches take 64-thread blocks, so that their work spreads
// over more compute units.
static unsigned slice_block(int64_t words) { return words < 256 * 1024 ? 64u : unsigned(kThreads); }

hipError_t launch_slice_rows(int e, int sid, const void* A, int64_t lda, int64_t m, int64_t k,
                             uint64_t* planes, int64_t Mp, int64_t K64p, int* err, hipStream_t s)
{
    if (Mp <= 0 || K64p <= 0) return hipSuccess;
    const unsigned bs = slice_block(Mp * K64p);
    dim3 grid(unsigned(ceil_div(Mp, bs)), unsigned(K64p));
    if (!with_any_schedule(e, sid, [&]<int E, int SID>() {
            hipLaunchKernelGGL((slice_rows_kernel<E, SID>), grid, dim3(bs), 0, s, A, lda, m, k, planes,
                               Mp, K64p, err);
        }))
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_slice_cols(int e, int sid, const void* B, int64_t ldb, int64_t k, int64_t n,
                             uint64_t* planes, int64_t Np, int64_t K64p, int* err, hipStream_t s)
{
    if (Np <= 0 || K64p <= 0) return hipSuccess;
    dim3 grid(unsigned(ceil_div(Np, kColBlock)), unsigned(K64p));
    if (!with_schedule(e, sid, [&]<int E, int SID>() {
            hipLaunchKernelGGL((slice_cols_kernel<E, SID>), grid, dim3(kColBlock), 0, s, B, ldb, k, n, planes,
                               Np, K64p, err);
        }))
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_slice_cols_alpha(int e, uint32_t f, const void* B, int64_t ldb, int64_t k, int64_t n,
                                   uint64_t* planes, int64_t Np, int64_t K64p, int* err, hipStream_t s)
{
    if (Np <= 0 || K64p <= 0) return hipSuccess;
    dim3 grid(unsigned(ceil_div(Np, kColBlock)), unsigned(K64p));
    if (!with_e(e, [&]<int E>() {
            hipLaunchKernelGGL((slice_cols_alpha_kernel<E>), grid, dim3(kColBlock), 0, s, B, ldb, k, n, f,
                               planes, Np, K64p, err);
        }))
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_combine(int e, int sid, uint32_t f, const uint64_t* P, int64_t pstride, int64_t ldp,
                          int64_t m, int64_t n, void* C, int64_t ldc, hipStream_t s, bool acc)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid(unsigned(ceil_div(ceil_div(n, 64), kThreads)), unsigned(m < 65535 ? m : 65535));
    if (!with_any_schedule(e, sid, [&]<int E, int SID>() {
            hipLaunchKernelGGL((combine_kernel<E, SID>), grid, dim3(kThreads), 0, s, P, pstride, ldp, m, n, f,
                               C, ldc, acc ? 1 : 0);
        }))
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_fill_elements(void* X, int64_t count, int e, uint64_t seed, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(ceil_div(count, 256), 8192);
    hipLaunchKernelGGL(fill_elements_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, X, count, e <= 8 ? 1 : 2,
                       (1u << e) - 1u, seed);
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

// One block per job of the products in each e-range (no idle blocks: a grid
// of the largest product's jobs times the product count was mostly empty).
hipError_t launch_batched_slice(const BatchProduct* prods, const JobList (&jobs)[2], int* err, hipStream_t s)
{
    if (jobs[0].total > 0)
        hipLaunchKernelGGL((batched_slice_kernel<2, kSmallE>), dim3(unsigned(jobs[0].total)), dim3(kThreads), 0, s,
                           prods, jobs[0].first, jobs[0].owner, jobs[0].n, err);
    if (jobs[1].total > 0)
        hipLaunchKernelGGL((batched_slice_kernel<kSmallE + 1, kMaxE>), dim3(unsigned(jobs[1].total)), dim3(kThreads),
                           0, s, prods, jobs[1].first, jobs[1].owner, jobs[1].n, err);
    return hipGetLastError();
}

hipError_t launch_batched_combine(const BatchProduct* prods, const JobList (&jobs)[2], hipStream_t s)
{
    if (jobs[0].total > 0)
        hipLaunchKernelGGL((batched_combine_kernel<2, kSmallE>), dim3(unsigned(jobs[0].total)), dim3(kThreads), 0, s,
                           prods, jobs[0].first, jobs[0].owner, jobs[0].n);
    if (jobs[1].total > 0)
        hipLaunchKernelGGL((batched_combine_kernel<kSmallE + 1, kMaxE>), dim3(unsigned(jobs[1].total)),
                           dim3(kThreads), 0, s, prods, jobs[1].first, jobs[1].owner, jobs[1].n);
    return hipGetLastError();
}

int batch_threads_per_block() { return kThreads; }

}  // namespace gf2e
