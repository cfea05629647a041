// Device-side helpers shared by the gfx950 kernels of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gf2e {

// 8x8 bit-matrix transpose of a 64-bit word read as 8 rows of 8 bits
// (row r = byte r, column c = bit c of that byte): bit 8r+c moves to 8c+r.
// Three rounds of block swaps (2x2, 4x4, 8x8 blocks of bits).
__host__ __device__ inline uint64_t transpose8x8(uint64_t x)
{
    uint64_t t;
    t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x = x ^ t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x = x ^ t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x = x ^ t ^ (t << 28);
    return x;
}

__device__ inline uint32_t byte_of(uint64_t x, int b) { return uint32_t(x >> (8 * b)) & 0xFFu; }

// Bits at or above e set in a packed row of byte elements (any element >= 2^e).
__device__ inline bool bytes_out_of_field(uint64_t x, int e)
{
    if (e >= 8) return false;
    const uint64_t keep = 0x0101010101010101ull * ((1u << e) - 1u);
    return (x & ~keep) != 0;
}

}  // namespace gf2e
