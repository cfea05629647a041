// Internal interfaces between the host library and the gfx950 kernels.
//
// Bit-plane layouts in device memory (all words are uint64_t, bit b of a
// word is column/index 64*word + b, LSB first):
//
//   operand planes (A side):  plane s of T, word (kw, r) at
//       base + s*K64p*Mp + kw*Mp + r      -- row r of A, k-bits [64kw, 64kw+64)
//   operand planes (B side):  plane s of T, word (kw, j) at
//       base + s*K64p*Np + kw*Np + j      -- column j of B, k-bits [64kw, 64kw+64)
//       in B-side bit order: inside every aligned group of four k, bits
//       4g, 4g+1, 4g+2, 4g+3 hold k = 4g+2, 4g+1, 4g, 4g+3 (b_side_bit)
//   product planes:           plane s of T, word (i, w) at
//       base + s*Mp*ldp + i*ldp + w       -- row i, columns [64w, 64w+64), ldp = Np/64
//
// Rows are padded to Mp (Np) and the k dimension to K64p words (a multiple of
// four, so the product kernels step through whole 256-bit stages; products of
// the plain path with k <= 128 use K64p = 2 and the one kernel with 128-bit
// stages).  Padding bits are written as zero by the slicing kernels, so padded
// k contributes nothing; the batched slicer leaves the padding rows (and
// columns) of its planes unwritten, since they only reach product rows and
// columns that are never combined.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gf2e {

constexpr int kRowAlign = 256;  // padding of plane rows (largest product tile)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
// B-side bit order: the bit of a B-side word that holds k-bit k of its
// 64-bit step (an involution that swaps the first and third k of each group
// of four).  With it the fp4 kernels expand a B chunk with the same four
// masks and one shift as an A chunk; the other kernels read B in this order.
constexpr int b_side_bit(int k) { return (k & 1) ? k : (k ^ 2); }

// Largest k the fp4 product kernels take: their f32 accumulators start at
// 2^23 and stay exact integers up to 2^24, so counts up to 2^23 are exact.
// Larger products run on the int8 kernels (exact for any k < 2^31).
constexpr int64_t kFp4MaxK = int64_t(1) << 23;

// k is padded to whole 256-bit steps, so every product kernel's stages are
// full and its loads need no bounds guard.
inline int64_t kwords_padded(int64_t k) { return 4 * ceil_div(k, 256); }

// Product-kernel variants the planner and the autotuner choose among.
enum GemmKind : int {
    GEMM_MFMA_256x256 = 0,  // int8 MFMA, 4 waves of 128x128
    GEMM_MFMA_128x128 = 1,  // int8 MFMA, 4 waves of 64x64
    GEMM_MFMA_256x128 = 2,  // int8 MFMA, 4 waves of 128x64
    GEMM_MFMA_64x64 = 3,    // int8 MFMA, 1 wave of 64x64
    GEMM_VALU_128x128 = 4,  // AND/XOR on packed words, 4 waves of 64x64
    GEMM_MFMA_256x256_W8 = 5,  // int8 MFMA, 8 waves of 128x64
    GEMM_FP4_256x256_W8 = 6,   // fp4 MFMA, 8 waves of 128x64 (k <= 2^23)
    GEMM_FP4_128x128 = 7,      // fp4 MFMA, 4 waves of 64x64 (k <= 2^23)
    GEMM_FP4_128x128_PLANES = 8,  // as 7 with 128-bit stages, several planes per workgroup (short k)
    GEMM_NUM_KINDS = 9
};

struct GemmShape {
    int bm, bn;
};
GemmShape gemm_shape(int kind);
const char* gemm_name(int kind);

// The kernels of one product run the schedule (e, sid): sid < 0 is the
// Karatsuba schedule for e (reduction mod f at run time), sid >= 0 the field
// schedule kFieldSchedules[sid] (see gf2e_schedule.hpp).

// Slice rows of A (m x k elements) into the schedule's A-side operand planes.
hipError_t launch_slice_rows(int e, int sid, const void* A, int64_t lda, int64_t m, int64_t k,
                             uint64_t* planes, int64_t Mp, int64_t K64p, int* err,
                             hipStream_t s);
// Slice columns of B (k x n elements) into its transposed B-side planes.
hipError_t launch_slice_cols(int e, int sid, const void* B, int64_t ldb, int64_t k, int64_t n,
                             uint64_t* planes, int64_t Np, int64_t K64p, int* err,
                             hipStream_t s);
// T plane products P_s = Ahat_s * Bhat_s^T over GF(2), one grouped launch.
hipError_t launch_gemm(int kind, int T, const uint64_t* Apl, const uint64_t* Bpl, uint64_t* P,
                       int64_t m, int64_t n, int64_t Mp, int64_t Np, int64_t K64p,
                       hipStream_t s);
// Alpha-power form: slice columns of B into the Ek x En operand whose block
// (i, c) is plane c of alpha^i B (block rows of K64p words, row pitch E*Np).
hipError_t launch_slice_cols_alpha(int e, uint32_t f, const void* B, int64_t ldb, int64_t k, int64_t n,
                                   uint64_t* planes, int64_t Np, int64_t K64p, int* err, hipStream_t s);
// Recombine the T products into result planes (reducing mod f for Karatsuba
// schedules) and write C (m x n elements), or add to C when acc is set.
// Product s, row i, word w is at P[s*pstride + i*ldp + w] (pstride = Mp*ldp
// for the grouped layout above).
hipError_t launch_combine(int e, int sid, uint32_t f, const uint64_t* P, int64_t pstride, int64_t ldp,
                          int64_t m, int64_t n, void* C, int64_t ldc, hipStream_t s, bool acc = false);
// One product of a batch, as the batched kernels read it from device memory.
struct BatchProduct {
    const void* A;
    const void* B;
    void* C;
    int64_t lda, ldb, ldc;
    int64_t m, k, n;
    int64_t Mp, Np, K64p;
    uint64_t* Apl;  // operand and product planes of this product (batch arena)
    uint64_t* Bpl;
    uint64_t* P;
    int32_t e, T;
    uint32_t f;
    int32_t sid;  // schedule: < 0 Karatsuba, else field schedule index
    int32_t slice_a_blocks;  // 256-thread jobs of A-side slicing (0 when k = 0)
    int32_t slice_b_blocks;
    int32_t combine_blocks;
    // Fused recombination (batched products with e <= kFusedMaxE): omask[s]
    // has bit c set when product plane s feeds result plane c (T entries,
    // device memory); the product kernel then writes C itself and P is unused.
    const uint32_t* omask;
    int32_t fused;
};

// One tile of planes plane..plane+nplanes-1 of a product in a persistent
// launch (the fp4 kernels run those planes as one pipeline).
struct WorkItem {
    int32_t prod, plane, tile_m, tile_n, nplanes;
};
// Planes per work item in the batched and served forms: as many as keep an
// item within this many k-words in all (at least one plane).
constexpr int64_t kItemKWords = 256;

// The batched slicing and combining kernels are instantiated for two ranges
// of e (up to kBatchSmallE, and above), each launched over its own products.
constexpr int kBatchSmallE = 10;

// A flattened launch over the products of one e-range: block b belongs to
// product owner[i] when first[i] <= b < first[i + 1] (device arrays; first
// has n + 1 entries, first[n] = total blocks).
struct JobList {
    const int* first = nullptr;
    const int* owner = nullptr;
    int n = 0, total = 0;
};
hipError_t launch_batched_slice(const BatchProduct* prods, const JobList (&jobs)[2], int* err, hipStream_t s);
hipError_t launch_batched_combine(const BatchProduct* prods, const JobList (&jobs)[2], hipStream_t s);
int batch_threads_per_block();
// Largest e whose products the fused persistent kernel serves.
constexpr int kFusedMaxE = 10;

// Persistent grouped products: workgroups take items in order from *counter
// until it passes nitems.  kind: GEMM_MFMA_256x256_W8 or GEMM_MFMA_128x128.
hipError_t launch_persistent_gemm(int kind, const BatchProduct* prods, const WorkItem* items,
                                  int nitems, int* counter, int grid, hipStream_t s);
int persistent_grid(int kind);  // workgroups that fill the device once
// The fp4 128x128 persistent kernel with the recombination and clinging in
// its epilogue: items cover all T planes of a tile of a fused product.
hipError_t launch_fused_persistent(const BatchProduct* prods, const WorkItem* items, int nitems, int* counter,
                                   int grid, hipStream_t s);
int fused_persistent_grid();
// Alpha-power form (plan with E = e column blocks, Kw words of k) with the
// clinging fused into the fp4 product: C = A * B (or C += A * B) straight
// from the operand planes.  e <= kFusedMaxE, Kw even and Kw * 64 <= kFp4MaxK.
hipError_t launch_fused_alpha(int e, const uint64_t* Apl, const uint64_t* Bpl, int64_t m, int64_t n, int64_t Mp,
                              int64_t Np, int64_t Kw, void* C, int64_t ldc, bool acc, hipStream_t s);
hipError_t launch_reset_counters(int* counters, int n, hipStream_t s);

// count pseudo-random elements of F_{2^e} (uint8 for e <= 8, else uint16).
hipError_t launch_fill_elements(void* X, int64_t count, int e, uint64_t seed, hipStream_t s);
// C = 0 (the k = 0 product).
hipError_t launch_zero(void* C, int64_t rows, int64_t cols, int64_t ld, int elem_bytes,
                       hipStream_t s);

}  // namespace gf2e
