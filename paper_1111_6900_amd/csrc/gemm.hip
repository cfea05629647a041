// GF(2) plane products P_s = Ahat_s * Bhat_s^T for all s of a schedule, in
// one grouped launch (gfx950).  These are the t(e) matrix products over F_2
// that the Bradshaw-Boothby reduction of Section 5 turns one product over
// F_{2^e} into.
//
// MFMA path: every bit is expanded to a 0/1 byte in LDS and fed to
// v_mfma_i32_16x16x64_i8; the int32 accumulator holds the exact number of
// k with A[i][k] = B[k][j] = 1 (exact for k < 2^31), and its low bit is the
// GF(2) product.  Only the parities are written back, bit-packed.
//
// The order of k inside a 64-bit step does not matter for the sum, only that
// both operands use the same order.  B words come in B-side bit order (k-bits
// 4g and 4g+2 of each group of four trade places, b_side_bit); every kernel
// undoes that swap when it expands or stages B, so that A and B are read with
// the same (lane group, byte) -> k assignment.
//
// VALU path: the same planes, AND/XOR on 32-bit words (acc ^= a & b, one
// v_bitop3 per 32 bit-products), parity by popcount at the end.
#include <hip/hip_runtime.h>
#include <algorithm>

#include "cling.hpp"
#include "gf2e_internal.hpp"

namespace gf2e {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// Expanded chunk c (0..7) of a 128-bit k-step held in two words: 16 bytes,
// byte (4*q + b) of the chunk = k-bit (8*b + 4*(c&1) + q) of 32-bit half
// c>>1.  On the B side that k-bit sits at bit b_side_bit(q) of its nibble, so
// dwords 0 and 2 take their bits from the other position (same cost).
template <bool BSIDE>
__device__ inline uint4 expand_chunk(uint64_t w0, uint64_t w1, int c)
{
    const uint64_t w = (c < 4) ? w0 : w1;
    const uint32_t h = uint32_t(w >> (32 * ((c >> 1) & 1)));
    const uint32_t s = 4 * (c & 1);
    const uint32_t M = 0x01010101u;
    constexpr int q0 = BSIDE ? 2 : 0, q2 = BSIDE ? 0 : 2;
    return make_uint4((h >> (s + q0)) & M, (h >> (s + 1)) & M, (h >> (s + q2)) & M, (h >> (s + 3)) & M);
}

template <int BM, int BN, int WM, int WN>
struct MfmaTile {
    static constexpr int kWavesN = BN / WN;
    static constexpr int kWaves = (BM / WM) * kWavesN;
    static constexpr int kThreads = kWaves * 64;
    static constexpr int FM = WM / 16;
    static constexpr int FN = WN / 16;
    static constexpr int kRows = BM + BN;  // staged rows per k-step (A then B)
    static constexpr int kRowsPerThread = (kRows + kThreads - 1) / kThreads;
    static_assert(WN % 64 == 0, "a wave must own whole 64-bit output words");
    static_assert(WM % 16 == 0 && BM % WM == 0 && BN % WN == 0, "tile shape");
};

// One BM x BN tile of P = Ahat * Bhat^T (planes already offset to product s).
template <int BM, int BN, int WM, int WN>
__device__ __attribute__((always_inline)) inline void mfma_tile(const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl,
                                 uint64_t* __restrict__ Ps, int64_t Mp, int64_t Np, int64_t K64p,
                                 int tile_m, int tile_n)
{
    using TL = MfmaTile<BM, BN, WM, WN>;
    // Two stages of 8 chunk-major arrays: lds[stage][chunk][row], 16 B each.
    __shared__ uint4 lds[2][8][BM + BN];
    constexpr int FM = TL::FM, FN = TL::FN, NT = TL::kThreads, RPT = TL::kRowsPerThread;
    const uint64_t* Ap = Apl + int64_t(tile_m) * BM;
    const uint64_t* Bp = Bpl + int64_t(tile_n) * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::kWavesN, wc = wave % TL::kWavesN;
    const int K128 = int(K64p / 2);

    v4i acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = v4i{0, 0, 0, 0};

    uint64_t stg[RPT][2];
    auto gload = [&](int kb) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = tid + q * NT;
            if (TL::kRows % NT == 0 || r < TL::kRows) {
                const bool isA = r < BM;
                const uint64_t* src = isA ? Ap + r : Bp + (r - BM);
                const int64_t ld = isA ? Mp : Np;
                stg[q][0] = src[int64_t(2 * kb) * ld];
                stg[q][1] = src[int64_t(2 * kb + 1) * ld];
            }
        }
    };
    auto expand_store = [&](int st) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = tid + q * NT;
            if (r < TL::kRows) {
                // BM and NT are multiples of 64: the side is uniform in a wave
                if (__builtin_amdgcn_readfirstlane(r) < BM) {
#pragma unroll
                    for (int c = 0; c < 8; ++c) lds[st][c][r] = expand_chunk<false>(stg[q][0], stg[q][1], c);
                } else {
#pragma unroll
                    for (int c = 0; c < 8; ++c) lds[st][c][r] = expand_chunk<true>(stg[q][0], stg[q][1], c);
                }
            }
        }
    };

    gload(0);
    expand_store(0);
    __syncthreads();
    const int g = lane >> 4, l16 = lane & 15;
    for (int kb = 0; kb < K128; ++kb) {
        const int st = kb & 1;
        const bool more = kb + 1 < K128;
        if (more) gload(kb + 1);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int c = 4 * kk + g;
            v4i a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const uint4 x = lds[st][c][wr * WM + 16 * i + l16];
                a[i] = v4i{int(x.x), int(x.y), int(x.z), int(x.w)};
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const uint4 x = lds[st][c][BM + wc * WN + 16 * j + l16];
                b[j] = v4i{int(x.x), int(x.y), int(x.z), int(x.w)};
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) expand_store(st ^ 1);
        __syncthreads();
    }

    // Epilogue: lane (g, l16) of block (i, j) holds rows 4g..4g+3, column l16.
    // The parity ballots of register r give 16 bits of each of 4 rows; lane L
    // (< 16 * WN/64) assembles row 4*(L&3) + ((L>>2)&3), word L>>4.
    const int64_t ldp = Np / 64;
    const int rg = lane & 3, rr = (lane >> 2) & 3, wsel = lane >> 4;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        uint64_t word = 0;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t bal = __builtin_amdgcn_ballot_w64((acc[i][j][r] & 1) != 0);
                if (rr == r && wsel == (j >> 2)) word |= ((bal >> (16 * rg)) & 0xFFFFull) << (16 * (j & 3));
            }
        if (lane < 16 * (WN / 64)) {
            const int64_t row = int64_t(tile_m) * BM + wr * WM + 16 * i + 4 * rg + rr;
            const int64_t colw = (int64_t(tile_n) * BN + wc * WN) / 64 + wsel;
            Ps[row * ldp + colw] = word;
        }
    }
}

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((MfmaTile<BM, BN, WM, WN>::kThreads)) void gemm_mfma_kernel(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, uint64_t* __restrict__ P,
    int64_t Mp, int64_t Np, int64_t K64p, int tiles_m, int tiles_n)
{
    const int64_t s = blockIdx.z;
    mfma_tile<BM, BN, WM, WN>(Apl + s * K64p * Mp, Bpl + s * K64p * Np, P + s * Mp * (Np / 64),
                              Mp, Np, K64p, blockIdx.y, blockIdx.x);
}

// Persistent grouped form: every workgroup takes work items (product, plane,
// tile) in list order from a global counter until the list is exhausted.
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((MfmaTile<BM, BN, WM, WN>::kThreads)) void gemm_mfma_persistent(
    const BatchProduct* __restrict__ prods, const WorkItem* __restrict__ items, int nitems,
    int* __restrict__ counter)
{
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(next);  // uniform: item fields go to SGPRs
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const BatchProduct& P = prods[w.prod];
        for (int64_t s = w.plane; s < w.plane + w.nplanes; ++s)
            mfma_tile<BM, BN, WM, WN>(P.Apl + s * P.K64p * P.Mp, P.Bpl + s * P.K64p * P.Np,
                                      P.P + s * P.Mp * (P.Np / 64), P.Mp, P.Np, P.K64p, w.tile_m,
                                      w.tile_n);
    }
}

__global__ void reset_counters_kernel(int* counters, int n)
{
    if (int(threadIdx.x) < n) counters[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// FP4 MFMA path (v_mfma_f32_16x16x128_f8f6f4, both operands e2m1, no block
// scales): every bit becomes a nibble that is 0 or a power of two, chosen per
// side so that each product of two set bits is exactly 1.0.  Each f32
// accumulator starts at 2^23 and then holds 2^23 plus the exact count of
// common ones (exact while the count is at most 2^23; launches with more k
// are refused), so bit 0 of its bit pattern is the GF(2) product, as in the
// int8 path, at twice its MFMA rate.  The MFMAs take the B fragment as their
// first operand, so each accumulator block holds a block of P^T: a lane holds
// four consecutive columns of one row, which the parity epilogue packs with
// shifts and a reduction over the four lane groups.  A stage holds KB consecutive
// 128-bit k-blocks; how each side sits in LDS (packed, split or expanded, see
// Fp4Side) trades VALU work in the reading waves against LDS bytes.  With
// operands expanded before the store the kernel was bound by LDS traffic;
// with all expansion in the reading waves, by VALU issue next to the MFMAs.
// ---------------------------------------------------------------------------
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr float kFp4Bias = 8388608.0f;  // 2^23

// fp4 operands occupy the low four dwords of the builtin's 8-dword operand;
// the upper half is left undefined so no registers are spent on it.
__device__ inline v8i fp4_operand(const uint4& x)
{
    const v4i v{int(x.x), int(x.y), int(x.z), int(x.w)};
    return __builtin_shufflevector(v, v, 0, 1, 2, 3, -1, -1, -1, -1);
}

// Nibble codes.  Dword q of an operand holds k-bits 4j+q (j < 8) of a 32-bit
// chunk h as nibble j; e2m1 codes 0b0001, 0b0010 and 0b0100 are 0.5, 1.0 and
// 2.0.  The A side gives dwords q = 0..3 the values 0.5, 1, 2, 2 and the B
// side 2, 1, 0.5, 0.5, so the product of two set bits is exactly 1.0 for
// every q and the f32 accumulator counts common ones.  Bit q of an A nibble
// already is the code of its value for q < 3.  B words hold k-bit q of a
// nibble at bit b_side_bit(q) (positions 2, 1, 0, 3), which again is the code
// of its value for q < 3: each side takes four masks and one shift.
template <bool BSIDE>
__device__ __attribute__((always_inline)) inline uint4 expand_fp4(uint32_t h)
{
    if constexpr (!BSIDE)
        return make_uint4(h & 0x11111111u, h & 0x22222222u, h & 0x44444444u, (h >> 1) & 0x44444444u);
    else
        return make_uint4(h & 0x44444444u, h & 0x22222222u, h & 0x11111111u, (h >> 3) & 0x11111111u);
}

// Split form of a chunk: dwords 0..2 of the expansion use disjoint bits and
// share one word, dword 3 is the other; expanding it again takes three masks.
template <bool BSIDE>
__device__ __attribute__((always_inline)) inline uint2 split_fp4(uint32_t h)
{
    const uint4 d = expand_fp4<BSIDE>(h);
    return make_uint2(d.x | d.y | d.z, d.w);
}

template <bool BSIDE>
__device__ __attribute__((always_inline)) inline uint4 unsplit_fp4(uint2 s)
{
    if constexpr (!BSIDE)
        return make_uint4(s.x & 0x11111111u, s.x & 0x22222222u, s.x & 0x44444444u, s.y);
    else
        return make_uint4(s.x & 0x44444444u, s.x & 0x22222222u, s.x & 0x11111111u, s.y);
}

// Orders a stage's products before the LDS stores that follow them.  Those
// stores fill the other buffer with data loaded at the top of the stage; the
// compiler may otherwise sink the products below them, so that each wave
// waits for its global loads right after issuing them.  The empty asm
// statements read and write every accumulator (no instruction is emitted),
// and the last one is a memory barrier.
template <int FM, int FN>
__device__ __attribute__((always_inline)) inline void products_before_stores(v4f (&acc)[FM][FN])
{
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) asm volatile("" : "+v"(acc[i][j]));
    asm volatile("" ::: "memory");
}

// One operand side (A rows or B columns) of the double-buffered stage in
// LDS, in one of three forms.  Packed: one 32-bit chunk per (chunk, row),
// expanded by every wave that reads it (VALU work per wave).  Expanded: the
// 16-byte nibble form, built once by the staging thread (four times the LDS
// bytes).  Split: the two-word form (twice the LDS bytes, three masks per
// read).
enum Fp4Form : int { kPacked = 0, kExpanded = 1, kSplit = 2 };

// PAD: words of padding per chunk row of the packed form.
template <int ROWS, int CH, int FORM, bool BSIDE, int PAD = 16>
struct Fp4Side;

template <int ROWS, int CH, bool BSIDE, int PAD>
struct Fp4Side<ROWS, CH, kPacked, BSIDE, PAD> {
    // Row pitch padded by 16 words: the 4 lane groups of one read (same rows,
    // chunks 4kb..4kb+3) fall on 4 disjoint sets of 16 banks.  Reads in the
    // grouped column order (fp4_planes_tile) use a pitch padded by 4 words
    // instead, for the same property.
    uint32_t w[2][CH][ROWS + PAD];
    __device__ __attribute__((always_inline)) void put(int buf, int c, int r, uint32_t h) { w[buf][c][r] = h; }
    __device__ __attribute__((always_inline)) v8i get(int buf, int c, int r) const
    {
        return fp4_operand(expand_fp4<BSIDE>(w[buf][c][r]));
    }
};

template <int ROWS, int CH, bool BSIDE, int PAD>
struct Fp4Side<ROWS, CH, kExpanded, BSIDE, PAD> {
    uint4 w[2][CH][ROWS];
    __device__ __attribute__((always_inline)) void put(int buf, int c, int r, uint32_t h)
    {
        w[buf][c][r] = expand_fp4<BSIDE>(h);
    }
    __device__ __attribute__((always_inline)) v8i get(int buf, int c, int r) const
    {
        return fp4_operand(w[buf][c][r]);
    }
};

template <int ROWS, int CH, bool BSIDE, int PAD>
struct Fp4Side<ROWS, CH, kSplit, BSIDE, PAD> {
    // Pitch padded by 16 rows (128 bytes): the two lane groups of a half-wave
    // read fall on disjoint halves of the banks.
    uint2 w[2][CH][ROWS + 16];
    __device__ __attribute__((always_inline)) void put(int buf, int c, int r, uint32_t h)
    {
        w[buf][c][r] = split_fp4<BSIDE>(h);
    }
    __device__ __attribute__((always_inline)) v8i get(int buf, int c, int r) const
    {
        return fp4_operand(unsplit_fp4<BSIDE>(w[buf][c][r]));
    }
};

// Parities of a wave's accumulators as plane words.  Block (i, j) holds P^T:
// lane (g, l16) register r is row 16 i + l16, column 16 j + 4 g + r of the
// wave tile, and bit 0 of its pattern is the parity.  Each lane packs its 16
// bits of a 64-column word (4 per block), shifted to its lane group's
// columns; an OR over the four lane groups (lanes l16, l16 + 16, + 32, + 48)
// then gives every lane the word of row 16 i + l16, and lane group g owns
// the words (i, w) with (i * NW + w) % 4 == g: fn(row, word column, word) is
// called for those.
template <int BM, int BN, int WM, int WN, class Fn>
__device__ __attribute__((always_inline)) inline void fp4_parity_words(
    const v4f (&acc)[MfmaTile<BM, BN, WM, WN>::FM][MfmaTile<BM, BN, WM, WN>::FN], int tile_m, int tile_n, int wr,
    int wc, int lane, Fn&& fn)
{
    constexpr int FM = MfmaTile<BM, BN, WM, WN>::FM, NW = WN / 64;
    const int g = lane >> 4, l16 = lane & 15;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t half[2] = {0u, 0u};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    half[jj >> 1] |= (__float_as_uint(acc[i][4 * w + jj][r]) & 1u) << (16 * (jj & 1) + r);
            // (shuffled as int: every bit of the pattern is kept)
            int lo = int(half[0] << (4 * g)), hi = int(half[1] << (4 * g));
            lo |= __shfl_xor(lo, 16);
            hi |= __shfl_xor(hi, 16);
            lo |= __shfl_xor(lo, 32);
            hi |= __shfl_xor(hi, 32);
            if (((i * NW + w) & 3) == g) {
                const int64_t row = int64_t(tile_m) * BM + wr * WM + 16 * i + l16;
                const int64_t colw = (int64_t(tile_n) * BN + wc * WN) / 64 + w;
                fn(row, colw, uint64_t(uint32_t(lo)) | (uint64_t(uint32_t(hi)) << 32));
            }
        }
}

// Stores the parity words of a wave's accumulators into plane Ps.
template <int BM, int BN, int WM, int WN>
__device__ __attribute__((always_inline)) inline void fp4_store_parity(
    const v4f (&acc)[MfmaTile<BM, BN, WM, WN>::FM][MfmaTile<BM, BN, WM, WN>::FN], uint64_t* __restrict__ Ps,
    int64_t Np, int tile_m, int tile_n, int wr, int wc, int lane)
{
    const int64_t ldp = Np / 64;
    fp4_parity_words<BM, BN, WM, WN>(acc, tile_m, tile_n, wr, wc, lane,
                                     [&](int64_t row, int64_t colw, uint64_t word) { Ps[row * ldp + colw] = word; });
}

// Parity words in the grouped column order of fp4_planes_tile: the B
// fragment of block j = 4 w + jj at lane x carries column
// 64 w + 16 (x >> 2) + 4 jj + (x & 3) of the wave tile, so that lane (g, l16)
// holds, in blocks 4w..4w+3 and registers r, the sixteen consecutive columns
// 64 w + 16 g + 4 jj + r of row 16 i + l16.  A funnel shift per value moves
// bit 0 of its pattern in at the top of a word (one instruction per bit), so
// after sixteen of them bit 16 + 4 jj + r holds column 16 g + 4 jj + r; two
// exchanges between lane groups then give every lane the whole word.  As in
// fp4_parity_words, lane group g owns the words (i, w) with
// (i * NW + w) % 4 == g, and fn(row, word column, word) is called for those.
template <int BM, int BN, int WM, int WN, class Fn>
__device__ __attribute__((always_inline)) inline void fp4_parity_words_grouped(
    const v4f (&acc)[MfmaTile<BM, BN, WM, WN>::FM][MfmaTile<BM, BN, WM, WN>::FN], int tile_m, int tile_n, int wr,
    int wc, int lane, Fn&& fn)
{
    constexpr int FM = MfmaTile<BM, BN, WM, WN>::FM, NW = WN / 64;
    const int g = lane >> 4, l16 = lane & 15;
    const uint32_t down = (g & 1) ? 0u : 16u;  // groups 0 and 2 fill bits 0..15 of their half
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t x = 0;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int r = 0; r < 4; ++r) x = __builtin_amdgcn_alignbit(__float_as_uint(acc[i][4 * w + jj][r]), x, 1);
            const int v = int(x >> down);
            const int y = v | __shfl_xor(v, 16);  // groups 0, 1: columns 0..31; groups 2, 3: 32..63
            const int o = __shfl_xor(y, 32);
            const uint32_t lo = uint32_t(g < 2 ? y : o), hi = uint32_t(g < 2 ? o : y);
            if (((i * NW + w) & 3) == g) {
                const int64_t row = int64_t(tile_m) * BM + wr * WM + 16 * i + l16;
                const int64_t colw = (int64_t(tile_n) * BN + wc * WN) / 64 + w;
                fn(row, colw, uint64_t(lo) | (uint64_t(hi) << 32));
            }
        }
}

// Stores the parity words of a wave's accumulators (grouped column order).
template <int BM, int BN, int WM, int WN>
__device__ __attribute__((always_inline)) inline void fp4_store_parity_grouped(
    const v4f (&acc)[MfmaTile<BM, BN, WM, WN>::FM][MfmaTile<BM, BN, WM, WN>::FN], uint64_t* __restrict__ Ps,
    int64_t Np, int tile_m, int tile_n, int wr, int wc, int lane)
{
    const int64_t ldp = Np / 64;
    fp4_parity_words_grouped<BM, BN, WM, WN>(
        acc, tile_m, tile_n, wr, wc, lane, [&](int64_t row, int64_t colw, uint64_t word) { Ps[row * ldp + colw] = word; });
}

template <int BM, int BN, int WM, int WN, int KB, int FA, int FB>
__device__ __attribute__((always_inline)) inline void fp4_tile(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, uint64_t* __restrict__ Ps,
    int64_t Mp, int64_t Np, int64_t K64p, int tile_m, int tile_n)
{
    using TL = MfmaTile<BM, BN, WM, WN>;
    constexpr int FM = TL::FM, FN = TL::FN, NT = TL::kThreads, RPT = TL::kRowsPerThread;
    constexpr int CH = 4 * KB;  // 32-bit chunks per row per stage
    __shared__ Fp4Side<BM, CH, FA, false> sa;
    __shared__ Fp4Side<BN, CH, FB, true> sb;
    const uint64_t* Ap = Apl + int64_t(tile_m) * BM;
    const uint64_t* Bp = Bpl + int64_t(tile_n) * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::kWavesN, wc = wave % TL::kWavesN;
    static_assert(KB == 1 || KB == 2, "a stage is one or two 128-bit k-blocks (K64p a multiple of 2 * KB)");
    static_assert(BM % 64 == 0 && NT % 64 == 0, "a wave stages rows of one side only");
    const int nstages = int(K64p / (2 * KB));

    v4f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = v4f{kFp4Bias, kFp4Bias, kFp4Bias, kFp4Bias};

    using Stage = uint64_t[RPT][2 * KB];
    auto gload = [&](int st, Stage& dst) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = tid + q * NT;
            if (r < TL::kRows) {
                const bool isA = r < BM;
                const uint64_t* src = isA ? Ap + r : Bp + (r - BM);
                const int64_t ld = isA ? Mp : Np;
#pragma unroll
                for (int w = 0; w < 2 * KB; ++w) dst[q][w] = src[(int64_t(st) * 2 * KB + w) * ld];
            }
        }
    };
    auto store = [&](int buf, const Stage& src) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = tid + q * NT;
            if (r < TL::kRows) {
                // BM and NT are multiples of 64, so a wave stages A rows or B
                // columns only; deciding on lane 0 gives a scalar branch.
                if (__builtin_amdgcn_readfirstlane(r) < BM) {
#pragma unroll
                    for (int c = 0; c < CH; ++c) sa.put(buf, c, r, uint32_t(src[q][c >> 1] >> (32 * (c & 1))));
                } else {
#pragma unroll
                    for (int c = 0; c < CH; ++c)
                        sb.put(buf, c, r - BM, uint32_t(src[q][c >> 1] >> (32 * (c & 1))));
                }
            }
        }
    };
    const int g = lane >> 4, l16 = lane & 15;
    auto compute = [&](int buf) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int c = 4 * kb + g;
            v8i a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = sa.get(buf, c, wr * WM + 16 * i + l16);
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = sb.get(buf, c, wc * WN + 16 * j + l16);
            // The wave raises its issue priority for its block of MFMAs, so
            // that the SIMD's arbiter keeps the matrix core fed from it while
            // the other waves' LDS reads and stores fill the gaps; the
            // scheduling barriers keep the block whole.
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    // Formats 4/4 select e2m1 for both operands; zero scale
                    // operands make the compiler emit the unscaled form.
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(b[j], a[i], acc[i][j], 4, 4, 0,
                                                                                0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // Loads for stage st + 1 are in flight while stage st computes.
    Stage s0;
    gload(0, s0);
    store(0, s0);
    __syncthreads();
    for (int st = 0; st < nstages; ++st) {
        const bool more = st + 1 < nstages;
        if (more) gload(st + 1, s0);
        compute(st & 1);
        products_before_stores(acc);
        if (more) store((st & 1) ^ 1, s0);
        __syncthreads();
    }

    fp4_store_parity<BM, BN, WM, WN>(acc, Ps, Np, tile_m, tile_n, wr, wc, lane);
}

// Tile of a workgroup, XCD-aware.  Workgroups are dispatched to the 8 XCDs
// in turn (linear id modulo 8), and each XCD has its own L2.  When the
// tile counts allow it, the tiles of a plane are cut into a 2 x 4 grid of
// regions and XCD x takes region x, in row-major order inside it: an XCD
// then reads half of A's row tiles and a quarter of B's column tiles instead
// of all of A.  Otherwise the launch grid maps to tiles directly.
__device__ __attribute__((always_inline)) inline void xcd_tile(int tiles_m, int tiles_n, int& tm, int& tn)
{
    constexpr int kXcds = 8, kRegM = 2, kRegN = 4;
    tm = blockIdx.y;
    tn = blockIdx.x;
    if (tiles_m % kRegM || tiles_n % kRegN) return;
    const int lin = int(blockIdx.y) * tiles_n + int(blockIdx.x);
    const int xcd = lin % kXcds, local = lin / kXcds;
    const int rm = tiles_m / kRegM, rn = tiles_n / kRegN;
    tm = (xcd / kRegN) * rm + local / rn;
    tn = (xcd % kRegN) * rn + local % rn;
}

// Waits until at most N of this wave's vector memory operations are in
// flight (loads complete in the order they were issued); expcnt and lgkmcnt
// are not waited for.
template <int N>
__device__ __attribute__((always_inline)) inline void wait_vmcnt()
{
    static_assert(N >= 0 && N <= 15, "the immediate's low vmcnt field");
    __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}
// The wait of a pipeline stage whose loads (PER per wave and stage) must be
// done while those of the `ahead` (at most 2) later stages stay in flight.
template <int PER>
__device__ __attribute__((always_inline)) inline void wait_stage_loads(int ahead)
{
    if (ahead >= 2)
        wait_vmcnt<2 * PER>();
    else if (ahead == 1)
        wait_vmcnt<PER>();
    else
        wait_vmcnt<0>();
}
typedef __attribute__((address_space(3))) void lds_void;
// The LDS address of p as the destination of a direct global-to-LDS load,
// passed through an empty asm statement: the compiler then does not know
// which LDS array the load writes, and does not make every LDS read wait
// for all such loads in flight (the kernels order them with their own
// vmcnt waits and barriers).
__device__ __attribute__((always_inline)) inline lds_void* lds_dst(const void* p)
{
    uint32_t a = uint32_t(uintptr_t((const lds_void*)p));
    asm("" : "+s"(a));
    return (lds_void*)uintptr_t(a);
}

// Workgroup barrier without the memory fence of __syncthreads, whose fence
// would wait for every load in flight; the empty asm statements keep the
// compiler from moving memory accesses across it.
__device__ __attribute__((always_inline)) inline void stage_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// A BM x BN tile (multiples of 128; the product kernel runs 128 x 128) with
// both sides packed, its operands moved from HBM into LDS by the direct
// global-to-LDS load (16 bytes per lane: two rows of one k-word, lane l's
// pair at 16 l bytes from the wave's LDS address), four LDS buffers deep:
// stages st + 1 .. st + 3 are in flight while stage st computes, with no
// staging registers and no LDS store instructions.  LDS holds each side as
// [buffer][k-word][row] 64-bit words, rows padded by 16 so that the two
// k-words a read touches fall on different halves of the 64 banks (37 KiB
// per 128 x 128 workgroup, four workgroups per compute unit).
template <int BM, int BN, int WM, int WN>
__device__ __attribute__((always_inline)) inline void fp4_tile_dma(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, uint64_t* __restrict__ Ps,
    int64_t Mp, int64_t Np, int64_t K64p, int tile_m, int tile_n)
{
    using TL = MfmaTile<BM, BN, WM, WN>;
    constexpr int FM = TL::FM, FN = TL::FN;
    constexpr int KW = 4, NB = 4, PR = 16;
    // Loads per stage: one per k-word and 128 rows of a side, LA of A and LB
    // of B per wave; wave w issues loads w, w + W, w + 2 W, ... of each side
    // (load t moves k-word t % KW of rows 128 (t / KW) ..).
    constexpr int W = TL::kWaves, LA = KW * BM / 128 / W, LB = KW * BN / 128 / W, PER = LA + LB;
    static_assert(BM % 128 == 0 && BN % 128 == 0 && LA * W * 128 == KW * BM && LB * W * 128 == KW * BN,
                  "whole wave loads of 128 rows of one k-word per side");
    static_assert(NB == 4, "the waits count at most NB - 2 = 2 stages ahead");
    __shared__ uint64_t la[NB][KW][BM + PR];
    __shared__ uint64_t lb[NB][KW][BN + PR];
    const uint64_t* Ap = Apl + int64_t(tile_m) * BM;
    const uint64_t* Bp = Bpl + int64_t(tile_n) * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::kWavesN, wc = wave % TL::kWavesN;
    const int nstages = int(K64p / KW);
    const int uw = __builtin_amdgcn_readfirstlane(wave);
    auto issue = [&](int st, int buf) {
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int t = uw + W * q, kw = t % KW, rb = 128 * (t / KW);
            const uint64_t* src = Ap + (int64_t(st) * KW + kw) * Mp + rb + 2 * lane;
            __builtin_amdgcn_global_load_lds((const void*)src, lds_dst(&la[buf][kw][rb]), 16, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int t = uw + W * q, kw = t % KW, rb = 128 * (t / KW);
            const uint64_t* src = Bp + (int64_t(st) * KW + kw) * Np + rb + 2 * lane;
            __builtin_amdgcn_global_load_lds((const void*)src, lds_dst(&lb[buf][kw][rb]), 16, 0, 0);
        }
    };

    v4f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = v4f{kFp4Bias, kFp4Bias, kFp4Bias, kFp4Bias};

    const int g = lane >> 4, l16 = lane & 15;
    // The packed operands of a k-block.  Those of a stage's first k-block
    // are read right after the stage's barrier, ahead of the next loads'
    // issue, and those of its second k-block before the first one's MFMAs,
    // so that their LDS latency passes under them.
    auto read_raw = [&](int buf, int kb, uint32_t (&ra)[FM], uint32_t (&rb)[FN]) {
        const int kw = 2 * kb + (g >> 1), half = g & 1;
#pragma unroll
        for (int i = 0; i < FM; ++i)
            ra[i] = reinterpret_cast<const uint32_t*>(&la[buf][kw][wr * WM + 16 * i + l16])[half];
#pragma unroll
        for (int j = 0; j < FN; ++j)
            rb[j] = reinterpret_cast<const uint32_t*>(&lb[buf][kw][wc * WN + 16 * j + l16])[half];
    };
    uint32_t ra[2][FM], rb[2][FN];
    auto compute = [&](int buf) {
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            v8i a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = fp4_operand(expand_fp4<false>(ra[kb][i]));
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = fp4_operand(expand_fp4<true>(rb[kb][j]));
            if (kb == 0) read_raw(buf, 1, ra[1], rb[1]);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(b[j], a[i], acc[i][j], 4, 4, 0, 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

#pragma unroll
    for (int q = 0; q < NB - 1; ++q)
        if (q < nstages) issue(q, q);
    for (int st = 0; st < nstages; ++st) {
        // This wave's loads of stage st are done once only the two of each
        // later stage in flight remain; the barrier then publishes every
        // wave's.
        wait_stage_loads<PER>(min(NB - 2, nstages - 1 - st));
        stage_barrier();
        // Buffer (st + 3) % 4 was last read by stage st - 1, which every
        // wave finished before the barrier.
        read_raw(st % NB, 0, ra[0], rb[0]);
        if (st + NB - 1 < nstages) issue(st + NB - 1, (st + NB - 1) % NB);
        compute(st % NB);
        products_before_stores(acc);
    }

    fp4_store_parity<BM, BN, WM, WN>(acc, Ps, Np, tile_m, tile_n, wr, wc, lane);
}

template <int BM, int BN, int WM, int WN, int KB, int FA, int FB>
__global__ __launch_bounds__((MfmaTile<BM, BN, WM, WN>::kThreads)) __attribute__((amdgpu_waves_per_eu(2))) void gemm_fp4_kernel(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, uint64_t* __restrict__ P,
    int64_t Mp, int64_t Np, int64_t K64p, int tiles_m, int tiles_n)
{
    const int64_t s = blockIdx.z;
    int tm, tn;
    xcd_tile(tiles_m, tiles_n, tm, tn);
    if constexpr (BM == 128 && KB == 2 && FA == kPacked && FB == kPacked)
        fp4_tile_dma<BM, BN, WM, WN>(Apl + s * K64p * Mp, Bpl + s * K64p * Np, P + s * Mp * (Np / 64), Mp, Np, K64p,
                                     tm, tn);
    else
        fp4_tile<BM, BN, WM, WN, KB, FA, FB>(Apl + s * K64p * Mp, Bpl + s * K64p * Np, P + s * Mp * (Np / 64), Mp,
                                             Np, K64p, tm, tn);
}

// Planes s0..s1-1 of one tile as one pipeline of stages (KB 128-bit
// k-blocks each, K64p a multiple of 2 KB), so that the operands of the next
// plane load while the current one computes and writes its words.  Products
// with little k (KB = 1) and the persistent work items (several planes of a
// tile) are then not bound by one load latency per plane.  After the last
// stage of plane s, plane_done(s, acc, wr, wc, lane) takes the wave's
// accumulators (it writes the plane's words, or folds them into results).
// Where plane s of each side starts and the word pitch along k: the usual
// grouped layout has plane s at s * K64p * Mp (A) and s * K64p * Np (B) with
// pitches Mp and Np.
struct PlaneAddr {
    int64_t a_pstride, b_pstride, lda, ldb;
};

template <int BM, int BN, int WM, int WN, int KB, int FA, int FB, class PlaneDone>
__device__ __attribute__((always_inline)) inline void fp4_planes_tile_at(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, int s0, int s1, PlaneAddr ad, int64_t K64p,
    int tile_m, int tile_n, PlaneDone&& plane_done)
{
    using TL = MfmaTile<BM, BN, WM, WN>;
    constexpr int FM = TL::FM, FN = TL::FN, NT = TL::kThreads, RPT = TL::kRowsPerThread;
    constexpr int CH = 4 * KB;  // 32-bit chunks per row per stage of KB 128-bit k-blocks
    __shared__ Fp4Side<BM, CH, FA, false> sa;
    __shared__ Fp4Side<BN, CH, FB, true, 4> sb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::kWavesN, wc = wave % TL::kWavesN;
    const int nst = int(K64p / (2 * KB));  // stages per plane
    const int G = (s1 - s0) * nst;     // stages of all planes
    static_assert(BM % 64 == 0 && NT % 64 == 0, "a wave stages rows of one side only");
    static_assert(FB == kPacked, "the grouped column order is laid out for the packed B side");
    static_assert(KB == 1 || KB == 2, "stages of one or two 128-bit k-blocks");

    v4f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = v4f{kFp4Bias, kFp4Bias, kFp4Bias, kFp4Bias};

    using Stage = uint64_t[RPT][2 * KB];
    auto gload = [&](int g, Stage& dst) {
        const int64_t s = s0 + g / nst, st = g % nst;
        const uint64_t* Ap = Apl + s * ad.a_pstride + int64_t(tile_m) * BM;
        const uint64_t* Bp = Bpl + s * ad.b_pstride + int64_t(tile_n) * BN;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = tid + q * NT;
            if (r < TL::kRows) {
                const bool isA = r < BM;
                const uint64_t* src = isA ? Ap + r : Bp + (r - BM);
                const int64_t ld = isA ? ad.lda : ad.ldb;
#pragma unroll
                for (int w = 0; w < 2 * KB; ++w) dst[q][w] = src[(st * 2 * KB + w) * ld];
            }
        }
    };
    auto store = [&](int buf, const Stage& src) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = tid + q * NT;
            if (r < TL::kRows) {
                if (__builtin_amdgcn_readfirstlane(r) < BM) {
#pragma unroll
                    for (int c = 0; c < CH; ++c) sa.put(buf, c, r, uint32_t(src[q][c >> 1] >> (32 * (c & 1))));
                } else {
#pragma unroll
                    for (int c = 0; c < CH; ++c)
                        sb.put(buf, c, r - BM, uint32_t(src[q][c >> 1] >> (32 * (c & 1))));
                }
            }
        }
    };
    const int g4 = lane >> 4, l16 = lane & 15;
    auto compute = [&](int buf) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            v8i a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = sa.get(buf, 4 * kb + g4, wr * WM + 16 * i + l16);
#pragma unroll
            for (int j = 0; j < FN; ++j)  // grouped column order (fp4_parity_words_grouped)
                b[j] = sb.get(buf, 4 * kb + g4, wc * WN + 64 * (j >> 2) + 16 * (l16 >> 2) + 4 * (j & 3) + (l16 & 3));
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(b[j], a[i], acc[i][j], 4, 4, 0, 0, 0, 0);
        }
    };

    Stage sr;
    gload(0, sr);
    store(0, sr);
    __syncthreads();
    for (int g = 0; g < G; ++g) {
        const bool more = g + 1 < G;
        if (more) gload(g + 1, sr);
        compute(g & 1);
        products_before_stores(acc);
        if ((g + 1) % nst == 0) {  // last stage of plane s0 + g / nst
            plane_done(s0 + g / nst, acc, wr, wc, lane);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = v4f{kFp4Bias, kFp4Bias, kFp4Bias, kFp4Bias};
        }
        if (more) store((g & 1) ^ 1, sr);
        __syncthreads();
    }
}

// Planes s0..s1-1 of one 128x128 tile as one pipeline of stages of 2 KB
// k-words, as fp4_planes_tile_at computes them, with the operands moved by
// the direct global-to-LDS load (see fp4_tile_dma): four LDS buffers, the
// next three stages in flight across plane boundaries, KB loads per wave and
// stage.  The B side is read in the grouped column order; its rows sit in
// LDS in pairs permuted by slot = column ^ (bit 5 of column) << 2 (lane l of
// a load takes the pair that belongs at slots 2l, 2l + 1), and its pitch is
// padded by 8 rows, so that the 32 words one read touches in each k-word
// cover half of the 64 banks and the two k-words the other half.  The A side
// is read in row order, pitch padded by 16 rows.
template <int KB, class PlaneDone>
__device__ __attribute__((always_inline)) inline void fp4_planes_tile_dma(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, int s0, int s1, PlaneAddr ad, int64_t K64p,
    int tile_m, int tile_n, PlaneDone&& plane_done)
{
    using TL = MfmaTile<128, 128, 64, 64>;
    constexpr int FM = TL::FM, FN = TL::FN, WM = 64, WN = 64;
    constexpr int KW = 2 * KB, NB = 4, PA = 16, PB = 8;
    static_assert(KB == 1 || KB == 2, "stages of one or two 128-bit k-blocks");
    __shared__ uint64_t la[NB][KW][128 + PA];
    __shared__ uint64_t lb[NB][KW][128 + PB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::kWavesN, wc = wave % TL::kWavesN;
    const int nst = int(K64p / KW);  // stages per plane
    const int G = (s1 - s0) * nst;   // stages of all planes
    // Wave w moves k-words KB (w & 1) .. KB (w & 1) + KB - 1 of side w >> 1.
    const int uw = __builtin_amdgcn_readfirstlane(wave);
    const bool aside = uw < 2;
    const int kw0 = KB * (uw & 1);
    const int bcol = (2 * lane) ^ (((lane >> 4) & 1) << 2);  // B column pair loaded into slots 2 lane, + 1
    auto issue = [&](int g, int buf) {
        const int64_t s = s0 + g / nst, st = g % nst;
#pragma unroll
        for (int q = 0; q < KB; ++q) {
            const int kw = kw0 + q;
            const int64_t word = st * KW + kw;
            const uint64_t* src = aside ? Apl + s * ad.a_pstride + int64_t(tile_m) * 128 + word * ad.lda + 2 * lane
                                        : Bpl + s * ad.b_pstride + int64_t(tile_n) * 128 + word * ad.ldb + bcol;
            __builtin_amdgcn_global_load_lds((const void*)src, lds_dst(aside ? &la[buf][kw][0] : &lb[buf][kw][0]), 16,
                                             0, 0);
        }
    };

    v4f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = v4f{kFp4Bias, kFp4Bias, kFp4Bias, kFp4Bias};

    const int g4 = lane >> 4, l16 = lane & 15;
    auto compute = [&](int buf) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int kw = 2 * kb + (g4 >> 1), half = g4 & 1;
            v8i a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = fp4_operand(expand_fp4<false>(
                    reinterpret_cast<const uint32_t*>(&la[buf][kw][wr * WM + 16 * i + l16])[half]));
#pragma unroll
            for (int j = 0; j < FN; ++j) {  // grouped column order (fp4_parity_words_grouped)
                const int col = wc * WN + 64 * (j >> 2) + 16 * (l16 >> 2) + 4 * (j & 3) + (l16 & 3);
                const int slot = col ^ (((col >> 5) & 1) << 2);
                b[j] = fp4_operand(
                    expand_fp4<true>(reinterpret_cast<const uint32_t*>(&lb[buf][kw][slot])[half]));
            }
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(b[j], a[i], acc[i][j], 4, 4, 0, 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

#pragma unroll
    for (int q = 0; q < NB - 1; ++q)
        if (q < G) issue(q, q);
    for (int g = 0; g < G; ++g) {
        wait_stage_loads<KB>(min(NB - 2, G - 1 - g));
        stage_barrier();
        // Buffer (g + 3) % 4 was last read at stage g - 1.
        if (g + NB - 1 < G) issue(g + NB - 1, (g + NB - 1) % NB);
        compute(g % NB);
        products_before_stores(acc);
        if ((g + 1) % nst == 0) {  // last stage of plane s0 + g / nst
            plane_done(s0 + g / nst, acc, wr, wc, lane);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = v4f{kFp4Bias, kFp4Bias, kFp4Bias, kFp4Bias};
        }
    }
}

template <int BM, int BN, int WM, int WN, int KB, int FA, int FB, class PlaneDone>
__device__ __attribute__((always_inline)) inline void fp4_planes_tile(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, int s0, int s1, int64_t Mp, int64_t Np,
    int64_t K64p, int tile_m, int tile_n, PlaneDone&& plane_done)
{
    const PlaneAddr ad{K64p * Mp, K64p * Np, Mp, Np};
    if constexpr (BM == 128 && BN == 128 && WM == 64 && WN == 64 && FA == kPacked && FB == kPacked)
        fp4_planes_tile_dma<KB>(Apl, Bpl, s0, s1, ad, K64p, tile_m, tile_n, plane_done);
    else
        fp4_planes_tile_at<BM, BN, WM, WN, KB, FA, FB>(Apl, Bpl, s0, s1, ad, K64p, tile_m, tile_n, plane_done);
}

template <int BM, int BN, int WM, int WN, int FA, int FB>
__global__ __launch_bounds__((MfmaTile<BM, BN, WM, WN>::kThreads)) __attribute__((amdgpu_waves_per_eu(2))) void gemm_fp4_planes_kernel(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, uint64_t* __restrict__ P, int T, int ppw,
    int64_t Mp, int64_t Np, int64_t K64p)
{
    const int s0 = int(blockIdx.z) * ppw, s1 = min(T, s0 + ppw);
    const int tm = blockIdx.y, tn = blockIdx.x;
    fp4_planes_tile<BM, BN, WM, WN, 1, FA, FB>(
        Apl, Bpl, s0, s1, Mp, Np, K64p, tm, tn, [&](int s, const auto& acc, int wr, int wc, int lane) {
            fp4_store_parity_grouped<BM, BN, WM, WN>(acc, P + int64_t(s) * Mp * (Np / 64), Np, tm, tn, wr, wc,
                                                     lane);
        });
}

// Persistent form: workgroups take (product, planes, tile) items in order
// from *counter; the planes of an item run as one pipeline.  The 128x128
// form is held to 128 VGPRs (four waves per SIMD, no spills), which serves
// the short items of a batch better than three.
template <int BM, int BN, int WM, int WN, int FA, int FB>
__global__ __launch_bounds__((MfmaTile<BM, BN, WM, WN>::kThreads)) __attribute__((amdgpu_waves_per_eu(BM == 128 ? 4 : 2))) void gemm_fp4_persistent(
    const BatchProduct* __restrict__ prods, const WorkItem* __restrict__ items, int nitems,
    int* __restrict__ counter)
{
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(next);  // uniform: item fields go to SGPRs
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const BatchProduct& P = prods[w.prod];
        // K64p is a multiple of 4 here: stages of two 128-bit k-blocks
        uint64_t* Pp = P.P;
        const int64_t Np = P.Np, pstride = P.Mp * (P.Np / 64);
        fp4_planes_tile<BM, BN, WM, WN, 2, FA, FB>(
            P.Apl, P.Bpl, w.plane, w.plane + w.nplanes, P.Mp, Np, P.K64p, w.tile_m, w.tile_n,
            [&](int s, const auto& acc, int wr, int wc, int lane) {
                fp4_store_parity_grouped<BM, BN, WM, WN>(acc, Pp + int64_t(s) * pstride, Np, w.tile_m, w.tile_n,
                                                         wr, wc, lane);
            });
    }
}

// Persistent form with the recombination fused into the epilogue: an item is
// one tile of every plane of a product.  After each plane, every lane folds
// the one parity word it owns into the result planes that product feeds
// (its bits in omask[s]: the merged map of recombination and reduction
// modulo f, Section 5); the running result planes sit in LDS, one slot per
// thread and plane.  After the last plane each lane clings its e result
// words to 64 elements of C.  No product planes are written and no
// combining pass runs.  For e <= kFusedMaxE.
template <int BM, int BN, int WM, int WN, int FA, int FB>
__global__ __launch_bounds__((MfmaTile<BM, BN, WM, WN>::kThreads)) __attribute__((amdgpu_waves_per_eu(4))) void gemm_fp4_fused_persistent(
    const BatchProduct* __restrict__ prods, const WorkItem* __restrict__ items, int nitems,
    int* __restrict__ counter)
{
    using TL = MfmaTile<BM, BN, WM, WN>;
    constexpr int NT = TL::kThreads;
    static_assert(TL::FM * (WN / 64) == 4, "each lane owns one parity word of a plane");
    static_assert(kFusedMaxE == 10, "the clinging switch below covers e = 2..10");
    __shared__ uint64_t res[kFusedMaxE][NT];
    __shared__ int next;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const BatchProduct& P = prods[w.prod];
        const uint32_t* __restrict__ om = P.omask;
#pragma unroll
        for (int q = 0; q < kFusedMaxE; ++q) res[q][tid] = 0;  // this thread's slots only
        // Stages of one 128-bit k-block: four LDS buffers of them beside the
        // result slots keep four workgroups on a compute unit.
        fp4_planes_tile<BM, BN, WM, WN, 1, FA, FB>(
            P.Apl, P.Bpl, 0, P.T, P.Mp, P.Np, P.K64p, w.tile_m, w.tile_n,
            [&](int s, const auto& acc, int wr, int wc, int lane) {
                uint64_t mine = 0;
                fp4_parity_words_grouped<BM, BN, WM, WN>(acc, w.tile_m, w.tile_n, wr, wc, lane,
                                                         [&](int64_t, int64_t, uint64_t word) { mine = word; });
                const uint32_t mask = om[s];  // uniform
#pragma unroll
                for (int q = 0; q < kFusedMaxE; ++q)
                    if ((mask >> q) & 1u) res[q][tid] ^= mine;
            });
        // The word a lane owns (fp4_parity_words: lane group g owns row
        // block i = g, so its row in the wave tile is 16 g + l16 = lane).
        const int wave = tid >> 6, lane = tid & 63;
        const int64_t row = int64_t(w.tile_m) * BM + (wave / TL::kWavesN) * WM + lane;
        const int64_t colw = (int64_t(w.tile_n) * BN + (wave % TL::kWavesN) * WN) / 64;
        if (row < P.m && colw * 64 < P.n) {
            uint64_t c[kFusedMaxE];
#pragma unroll
            for (int q = 0; q < kFusedMaxE; ++q) c[q] = res[q][tid];
            switch (P.e) {
                case 2: cling_store<2>(c, P.n, P.C, P.ldc, row, colw, false); break;
                case 3: cling_store<3>(c, P.n, P.C, P.ldc, row, colw, false); break;
                case 4: cling_store<4>(c, P.n, P.C, P.ldc, row, colw, false); break;
                case 5: cling_store<5>(c, P.n, P.C, P.ldc, row, colw, false); break;
                case 6: cling_store<6>(c, P.n, P.C, P.ldc, row, colw, false); break;
                case 7: cling_store<7>(c, P.n, P.C, P.ldc, row, colw, false); break;
                case 8: cling_store<8>(c, P.n, P.C, P.ldc, row, colw, false); break;
                case 9: cling_store<9>(c, P.n, P.C, P.ldc, row, colw, false); break;
                case 10: cling_store<10>(c, P.n, P.C, P.ldc, row, colw, false); break;
                default: break;
            }
        }
    }
}

// Alpha-power form with the clinging in the epilogue.  The form's one
// product has E column blocks (block c of B starts at column c * Np, its
// words along k at pitch E * Np; A is the same for every block), and column
// block c of the result is plane c of C.  A workgroup takes a 128 x 128 tile
// of C and runs the E blocks over it as planes, so that after block c each
// lane holds plane c of its word of the result (kept in LDS); it then clings
// the E planes into C (C = A * B, or C += A * B with acc).  No product
// planes are written and no combining pass runs.  For E <= kFusedMaxE; Kw
// (words of k) even.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gemm_fp4_fused_alpha(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, int E, int64_t Mp, int64_t Np, int64_t Kw,
    int64_t m, int64_t n, void* __restrict__ C, int64_t ldc, int acc)
{
    using TL = MfmaTile<128, 128, 64, 64>;
    static_assert(kFusedMaxE == 10, "the clinging switch below covers e = 2..10");
    __shared__ uint64_t res[kFusedMaxE][TL::kThreads];
    const int tid = threadIdx.x, tm = blockIdx.y, tn = blockIdx.x;
    fp4_planes_tile_dma<1>(
        Apl, Bpl, 0, E, PlaneAddr{0, Np, Mp, int64_t(E) * Np}, Kw, tm, tn,
        [&](int c, const auto& a, int wr, int wc, int lane) {
            uint64_t mine = 0;
            fp4_parity_words_grouped<128, 128, 64, 64>(a, tm, tn, wr, wc, lane,
                                                       [&](int64_t, int64_t, uint64_t word) { mine = word; });
            res[c][tid] = mine;
        });
    // the word a lane owns: row 16 g + l16 = lane of its wave's tile
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t row = int64_t(tm) * 128 + (wave / TL::kWavesN) * 64 + lane;
    const int64_t colw = (int64_t(tn) * 128 + (wave % TL::kWavesN) * 64) / 64;
    if (row >= m || colw * 64 >= n) return;
    uint64_t c[kFusedMaxE];
#pragma unroll
    for (int q = 0; q < kFusedMaxE; ++q) c[q] = q < E ? res[q][tid] : 0ull;
    const bool add = acc != 0;
    switch (E) {
        case 2: cling_store<2>(c, n, C, ldc, row, colw, add); break;
        case 3: cling_store<3>(c, n, C, ldc, row, colw, add); break;
        case 4: cling_store<4>(c, n, C, ldc, row, colw, add); break;
        case 5: cling_store<5>(c, n, C, ldc, row, colw, add); break;
        case 6: cling_store<6>(c, n, C, ldc, row, colw, add); break;
        case 7: cling_store<7>(c, n, C, ldc, row, colw, add); break;
        case 8: cling_store<8>(c, n, C, ldc, row, colw, add); break;
        case 9: cling_store<9>(c, n, C, ldc, row, colw, add); break;
        case 10: cling_store<10>(c, n, C, ldc, row, colw, add); break;
        default: break;
    }
}

// ---------------------------------------------------------------------------
// VALU path: WG tile 128x128, 4 waves of 64x64, thread (ty, tx) of its wave
// owns rows 8*ty + r and columns tx + 8*c (r, c < 8), so that one ballot per
// (r, c) yields whole bytes of output words.
// ---------------------------------------------------------------------------
constexpr int kValuTile = 128;

__global__ __launch_bounds__(256) void gemm_valu_kernel(
    const uint64_t* __restrict__ Apl, const uint64_t* __restrict__ Bpl, uint64_t* __restrict__ P,
    int64_t Mp, int64_t Np, int64_t K64p, int tiles_m, int tiles_n)
{
    // lds[stage][k-dword][row]: 128 A rows then 128 B columns (permuted).
    __shared__ __align__(16) uint32_t lds[2][4][2 * kValuTile];
    const int s = blockIdx.z;
    const int tile_m = blockIdx.y, tile_n = blockIdx.x;
    const uint64_t* Ap = Apl + int64_t(s) * K64p * Mp + int64_t(tile_m) * kValuTile;
    const uint64_t* Bp = Bpl + int64_t(s) * K64p * Np + int64_t(tile_n) * kValuTile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int ty = lane >> 3, tx = lane & 7;
    const int K128 = int(K64p / 2);

    // Staging row of this thread and its LDS slot (B columns permuted so that
    // column tx + 8c of a 64-column half sits at 8*tx + c).
    const bool isA = tid < kValuTile;
    const int srow = isA ? tid : tid - kValuTile;
    const uint64_t* src = isA ? Ap + srow : Bp + srow;
    const int64_t ld = isA ? Mp : Np;
    int slot;
    if (isA) {
        slot = srow;
    } else {
        const int half = srow >> 6, cc = srow & 63;
        slot = kValuTile + half * 64 + (cc & 7) * 8 + (cc >> 3);
    }

    uint32_t acc[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[r][c] = 0;

    // A words are staged in B-side bit order (k-bits 4g and 4g+2 swapped), so
    // both operands of the AND hold the same k at each bit.
    const uint64_t swap_mask = isA ? 0x1111111111111111ull : 0ull;
    auto to_b_order = [&](uint64_t x) {
        const uint64_t d = ((x >> 2) ^ x) & swap_mask;
        return x ^ (d | (d << 2));
    };
    uint64_t w0 = to_b_order(src[0]), w1 = to_b_order(src[ld]);
    auto store = [&](int st) {
        lds[st][0][slot] = uint32_t(w0);
        lds[st][1][slot] = uint32_t(w0 >> 32);
        lds[st][2][slot] = uint32_t(w1);
        lds[st][3][slot] = uint32_t(w1 >> 32);
    };
    store(0);
    __syncthreads();
    for (int kb = 0; kb < K128; ++kb) {
        const int st = kb & 1;
        const bool more = kb + 1 < K128;
        if (more) {
            w0 = to_b_order(src[int64_t(2 * kb + 2) * ld]);
            w1 = to_b_order(src[int64_t(2 * kb + 3) * ld]);
        }
#pragma unroll
        for (int kd = 0; kd < 4; ++kd) {
            uint32_t a[8], b[8];
            const uint4* pa = reinterpret_cast<const uint4*>(&lds[st][kd][wr * 64 + ty * 8]);
            const uint4* pb = reinterpret_cast<const uint4*>(&lds[st][kd][kValuTile + wc * 64 + tx * 8]);
            const uint4 a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
            a[0] = a0.x; a[1] = a0.y; a[2] = a0.z; a[3] = a0.w;
            a[4] = a1.x; a[5] = a1.y; a[6] = a1.z; a[7] = a1.w;
            b[0] = b0.x; b[1] = b0.y; b[2] = b0.z; b[3] = b0.w;
            b[4] = b1.x; b[5] = b1.y; b[6] = b1.z; b[7] = b1.w;
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[r][c] ^= a[r] & b[c];
        }
        if (more) store(st ^ 1);
        __syncthreads();
    }

    const int64_t ldp = Np / 64;
    uint64_t* Ps = P + int64_t(s) * Mp * ldp;
    uint64_t word = 0;
    const int my_ty = lane >> 3, my_r = lane & 7;
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint64_t bal = __builtin_amdgcn_ballot_w64((__builtin_popcount(acc[r][c]) & 1) != 0);
            if (my_r == r) word |= ((bal >> (8 * my_ty)) & 0xFFull) << (8 * c);
        }
    const int64_t row = int64_t(tile_m) * kValuTile + wr * 64 + lane;
    const int64_t colw = (int64_t(tile_n) * kValuTile + wc * 64) / 64;
    Ps[row * ldp + colw] = word;
}

template <int BM, int BN, int WM, int WN>
hipError_t launch_mfma(int T, const uint64_t* Apl, const uint64_t* Bpl, uint64_t* P, int64_t m,
                       int64_t n, int64_t Mp, int64_t Np, int64_t K64p, hipStream_t st)
{
    using TL = MfmaTile<BM, BN, WM, WN>;
    const int tm = int(ceil_div(m, BM)), tn = int(ceil_div(n, BN));
    if (tm * int64_t(BM) > Mp || tn * int64_t(BN) > Np) return hipErrorInvalidValue;
    dim3 grid(tn, tm, T);
    hipLaunchKernelGGL((gemm_mfma_kernel<BM, BN, WM, WN>), grid, dim3(TL::kThreads), 0, st, Apl,
                       Bpl, P, Mp, Np, K64p, tm, tn);
    return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, int KB, int FA, int FB>
hipError_t launch_fp4(int T, const uint64_t* Apl, const uint64_t* Bpl, uint64_t* P, int64_t m,
                      int64_t n, int64_t Mp, int64_t Np, int64_t K64p, hipStream_t st)
{
    using TL = MfmaTile<BM, BN, WM, WN>;
    const int tm = int(ceil_div(m, BM)), tn = int(ceil_div(n, BN));
    if (tm * int64_t(BM) > Mp || tn * int64_t(BN) > Np || K64p * 64 > kFp4MaxK) return hipErrorInvalidValue;
    dim3 grid(tn, tm, T);
    hipLaunchKernelGGL((gemm_fp4_kernel<BM, BN, WM, WN, KB, FA, FB>), grid, dim3(TL::kThreads), 0, st, Apl, Bpl,
                       P, Mp, Np, K64p, tm, tn);
    return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, int FA, int FB>
hipError_t launch_fp4_planes(int T, const uint64_t* Apl, const uint64_t* Bpl, uint64_t* P, int64_t m, int64_t n,
                             int64_t Mp, int64_t Np, int64_t K64p, hipStream_t st)
{
    using TL = MfmaTile<BM, BN, WM, WN>;
    const int tm = int(ceil_div(m, BM)), tn = int(ceil_div(n, BN));
    if (tm * int64_t(BM) > Mp || tn * int64_t(BN) > Np || K64p % 2 || K64p * 64 > kFp4MaxK)
        return hipErrorInvalidValue;
    // Planes per workgroup: keep about 4096 workgroups (16 per compute unit)
    // when there are more (tile, plane) pairs than that.
    const int ppw = int(std::clamp<int64_t>(int64_t(T) * tm * tn / 4096, 1, T));
    dim3 grid(tn, tm, unsigned(ceil_div(T, ppw)));
    hipLaunchKernelGGL((gemm_fp4_planes_kernel<BM, BN, WM, WN, FA, FB>), grid, dim3(TL::kThreads), 0, st, Apl, Bpl,
                       P, T, ppw, Mp, Np, K64p);
    return hipGetLastError();
}

template <class Kern>
int blocks_filling_device(Kern kernel, int threads)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
}

template <int BM, int BN, int WM, int WN>
int persistent_blocks()
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_mfma_persistent<BM, BN, WM, WN>,
                                                     MfmaTile<BM, BN, WM, WN>::kThreads, 0) != hipSuccess)
        return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
}

}  // namespace

int persistent_grid(int kind)
{
    switch (kind) {
        case GEMM_MFMA_256x256_W8: return persistent_blocks<256, 256, 128, 64>();
        case GEMM_MFMA_128x128: return persistent_blocks<128, 128, 64, 64>();
        case GEMM_FP4_256x256_W8:
            return blocks_filling_device(gemm_fp4_persistent<256, 256, 128, 64, kSplit, kPacked>,
                                         MfmaTile<256, 256, 128, 64>::kThreads);
        case GEMM_FP4_128x128:
            return blocks_filling_device(gemm_fp4_persistent<128, 128, 64, 64, kPacked, kPacked>,
                                         MfmaTile<128, 128, 64, 64>::kThreads);
        default: return 0;
    }
}

hipError_t launch_persistent_gemm(int kind, const BatchProduct* prods, const WorkItem* items,
                                  int nitems, int* counter, int grid, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (grid <= 0) return hipErrorInvalidValue;
    switch (kind) {
        case GEMM_MFMA_256x256_W8:
            hipLaunchKernelGGL((gemm_mfma_persistent<256, 256, 128, 64>), dim3(grid),
                               dim3(MfmaTile<256, 256, 128, 64>::kThreads), 0, s, prods, items, nitems,
                               counter);
            break;
        case GEMM_MFMA_128x128:
            hipLaunchKernelGGL((gemm_mfma_persistent<128, 128, 64, 64>), dim3(grid),
                               dim3(MfmaTile<128, 128, 64, 64>::kThreads), 0, s, prods, items, nitems,
                               counter);
            break;
        case GEMM_FP4_256x256_W8:
            hipLaunchKernelGGL((gemm_fp4_persistent<256, 256, 128, 64, kSplit, kPacked>), dim3(grid),
                               dim3(MfmaTile<256, 256, 128, 64>::kThreads), 0, s, prods, items, nitems,
                               counter);
            break;
        case GEMM_FP4_128x128:
            hipLaunchKernelGGL((gemm_fp4_persistent<128, 128, 64, 64, kPacked, kPacked>), dim3(grid),
                               dim3(MfmaTile<128, 128, 64, 64>::kThreads), 0, s, prods, items, nitems,
                               counter);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fused_alpha(int e, const uint64_t* Apl, const uint64_t* Bpl, int64_t m, int64_t n, int64_t Mp,
                              int64_t Np, int64_t Kw, void* C, int64_t ldc, bool acc, hipStream_t s)
{
    const int64_t tm = ceil_div(m, 128), tn = ceil_div(n, 128);
    if (e < 2 || e > kFusedMaxE || Kw % 2 || Kw * 64 > kFp4MaxK || tm * 128 > Mp || tn * 128 > Np)
        return hipErrorInvalidValue;
    if (m == 0 || n == 0) return hipSuccess;
    const dim3 grid{unsigned(tn), unsigned(tm)}, block{unsigned(MfmaTile<128, 128, 64, 64>::kThreads)};
    hipLaunchKernelGGL(gemm_fp4_fused_alpha, grid, block, 0, s, Apl, Bpl, e, Mp, Np, Kw, m, n, C, ldc, acc ? 1 : 0);
    return hipGetLastError();
}

int fused_persistent_grid()
{
    return blocks_filling_device(gemm_fp4_fused_persistent<128, 128, 64, 64, kPacked, kPacked>,
                                 MfmaTile<128, 128, 64, 64>::kThreads);
}

hipError_t launch_fused_persistent(const BatchProduct* prods, const WorkItem* items, int nitems, int* counter,
                                   int grid, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_fp4_fused_persistent<128, 128, 64, 64, kPacked, kPacked>), dim3(grid),
                       dim3(MfmaTile<128, 128, 64, 64>::kThreads), 0, s, prods, items, nitems, counter);
    return hipGetLastError();
}

hipError_t launch_reset_counters(int* counters, int n, hipStream_t s)
{
    if (n <= 0 || n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, counters, n);
    return hipGetLastError();
}

GemmShape gemm_shape(int kind)
{
    switch (kind) {
        case GEMM_MFMA_256x256: return {256, 256};
        case GEMM_MFMA_128x128: return {128, 128};
        case GEMM_MFMA_256x128: return {256, 128};
        case GEMM_MFMA_64x64: return {64, 64};
        case GEMM_VALU_128x128: return {kValuTile, kValuTile};
        case GEMM_MFMA_256x256_W8: return {256, 256};
        case GEMM_FP4_256x256_W8: return {256, 256};
        case GEMM_FP4_128x128: return {128, 128};
        case GEMM_FP4_128x128_PLANES: return {128, 128};
        default: return {0, 0};
    }
}

const char* gemm_name(int kind)
{
    switch (kind) {
        case GEMM_MFMA_256x256: return "mfma_i8_256x256";
        case GEMM_MFMA_128x128: return "mfma_i8_128x128";
        case GEMM_MFMA_256x128: return "mfma_i8_256x128";
        case GEMM_MFMA_64x64: return "mfma_i8_64x64";
        case GEMM_VALU_128x128: return "valu_xor_128x128";
        case GEMM_MFMA_256x256_W8: return "mfma_i8_256x256_w8";
        case GEMM_FP4_256x256_W8: return "mfma_fp4_256x256_w8";
        case GEMM_FP4_128x128: return "mfma_fp4_128x128";
        case GEMM_FP4_128x128_PLANES: return "mfma_fp4_128x128_planes";
        default: return "unknown";
    }
}

hipError_t launch_gemm(int kind, int T, const uint64_t* Apl, const uint64_t* Bpl, uint64_t* P,
                       int64_t m, int64_t n, int64_t Mp, int64_t Np, int64_t K64p, hipStream_t st)
{
    if (T <= 0 || m <= 0 || n <= 0 || K64p <= 0) return hipSuccess;
    if (kind == GEMM_FP4_128x128_PLANES)
        return launch_fp4_planes<128, 128, 64, 64, kPacked, kPacked>(T, Apl, Bpl, P, m, n, Mp, Np, K64p, st);
    if (K64p % 4 != 0) return hipErrorInvalidValue;  // the other kernels step 256-bit stages
    switch (kind) {
        case GEMM_MFMA_256x256:
            return launch_mfma<256, 256, 128, 128>(T, Apl, Bpl, P, m, n, Mp, Np, K64p, st);
        case GEMM_MFMA_128x128:
            return launch_mfma<128, 128, 64, 64>(T, Apl, Bpl, P, m, n, Mp, Np, K64p, st);
        case GEMM_MFMA_256x128:
            return launch_mfma<256, 128, 128, 64>(T, Apl, Bpl, P, m, n, Mp, Np, K64p, st);
        case GEMM_MFMA_64x64:
            return launch_mfma<64, 64, 64, 64>(T, Apl, Bpl, P, m, n, Mp, Np, K64p, st);
        case GEMM_MFMA_256x256_W8:
            return launch_mfma<256, 256, 128, 64>(T, Apl, Bpl, P, m, n, Mp, Np, K64p, st);
        case GEMM_FP4_256x256_W8:
            return launch_fp4<256, 256, 128, 64, 2, kSplit, kPacked>(T, Apl, Bpl, P, m, n, Mp, Np, K64p, st);
        case GEMM_FP4_128x128:
            return launch_fp4<128, 128, 64, 64, 2, kPacked, kPacked>(T, Apl, Bpl, P, m, n, Mp, Np, K64p, st);

        case GEMM_VALU_128x128: {
            const int tm = int(ceil_div(m, kValuTile)), tn = int(ceil_div(n, kValuTile));
            if (tm * int64_t(kValuTile) > Mp || tn * int64_t(kValuTile) > Np) return hipErrorInvalidValue;
            hipLaunchKernelGGL(gemm_valu_kernel, dim3(tn, tm, T), dim3(256), 0, st, Apl, Bpl, P, Mp,
                               Np, K64p, tm, tn);
            return hipGetLastError();
        }
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gf2e
