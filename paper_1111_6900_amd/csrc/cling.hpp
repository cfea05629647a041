// Clinging (the inverse of slicing, Section 3.2): e result bit-planes of one
// 64-bit word become 64 elements of a row of C.  Shared by the combining
// kernels and the fused epilogue of the persistent product kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

#include "gf2e_device.hpp"

namespace gf2e {

// Word w of row i: element 64w + 8g + b takes bit 8g + b of planes
// c[0..E-1].  Writes the elements of columns < n (n - 64w of them when that
// is less than 64), or XORs them into C when acc is set.
template <int E, int N>
__device__ __attribute__((always_inline)) inline void cling_store(const uint64_t (&c)[N], int64_t n,
                                                                   void* __restrict__ C, int64_t ldc, int64_t i,
                                                                   int64_t w, bool acc)
{
    static_assert(N >= E, "fewer planes than the field has bits");
    using elem_t = typename std::conditional<(E > 8), uint16_t, uint8_t>::type;
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
                uint4 o = make_uint4(wd[0], wd[1], wd[2], wd[3]);
                if (acc) {
                    const uint4 old = v[q];
                    o.x ^= old.x; o.y ^= old.y; o.z ^= old.z; o.w ^= old.w;
                }
                v[q] = o;
            }
            return;
        }
    }
    // Unaligned or partial run: the dwords inside it are written whole, the
    // bytes of the partial dwords at its ends one by one (the neighbouring
    // runs own the other bytes of those dwords).
    constexpr int EB = int(sizeof(elem_t)), NW = 16 * EB;
    uint32_t o[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        if constexpr (EB == 1)
            o[j] = uint32_t(out[4 * j]) | (uint32_t(out[4 * j + 1]) << 8) | (uint32_t(out[4 * j + 2]) << 16) |
                   (uint32_t(out[4 * j + 3]) << 24);
        else
            o[j] = uint32_t(out[2 * j]) | (uint32_t(out[2 * j + 1]) << 16);
    }
    const int nbytes = int(valid) * EB;
    const uintptr_t pa = reinterpret_cast<uintptr_t>(dst);
    const int off = int(pa & 3);
    uint32_t* aw = reinterpret_cast<uint32_t*>(pa & ~uintptr_t(3));
#pragma unroll
    for (int t = 0; t <= NW; ++t) {
        const int first = 4 * t - off;  // run offset of the dword's byte 0
        if (first >= nbytes) break;
        const uint32_t lo = t > 0 ? o[t - 1] : 0u, hi = t < NW ? o[t] : 0u;
        const uint32_t v = off ? __builtin_amdgcn_alignbyte(hi, lo, uint32_t(4 - off)) : hi;
        if (first >= 0 && first + 4 <= nbytes) {
            aw[t] = acc ? aw[t] ^ v : v;
        } else {
            uint8_t* ab = reinterpret_cast<uint8_t*>(aw + t);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (first + b >= 0 && first + b < nbytes) {
                    const uint8_t x = uint8_t(v >> (8 * b));
                    ab[b] = acc ? uint8_t(ab[b] ^ x) : x;
                }
        }
    }
}

}  // namespace gf2e
