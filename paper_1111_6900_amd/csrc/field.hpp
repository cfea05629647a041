// Host-side field set-up for F_{2^e} = F_2[x]/<f> (M4RIE paper, Section 2):
// irreducibility of f and the reduction matrix x^d mod f.
#pragma once
#include <cstdint>

#include "gf2e_schedule.hpp"

namespace gf2e {

// Product of a and b modulo f (deg f = e), both reduced, in F_2[x].
inline uint32_t polymulmod(uint32_t a, uint32_t b, uint32_t f, int e)
{
    uint32_t r = 0;
    while (b) {
        if (b & 1u) r ^= a;
        b >>= 1;
        a <<= 1;
        if ((a >> e) & 1u) a ^= f;
    }
    return r;
}

inline int poly_deg(uint32_t p)
{
    int d = -1;
    while (p) { ++d; p >>= 1; }
    return d;
}

inline uint32_t poly_gcd(uint32_t a, uint32_t b)
{
    while (b) {
        while (poly_deg(a) >= poly_deg(b)) a ^= b << (poly_deg(a) - poly_deg(b));
        uint32_t t = a; a = b; b = t;
    }
    return a;
}

// Ben-Or's test: f of degree e is irreducible iff gcd(x^(2^i) - x, f) = 1
// for every 1 <= i <= e/2 (repeated squaring of x modulo f).
inline bool is_irreducible(int e, uint32_t f)
{
    if (e < 1 || e > 16 || poly_deg(f) != e) return false;
    uint32_t xp = 2u % f;  // x mod f (f has degree >= 1)
    if (e == 1) return true;
    for (int i = 1; i <= e / 2; ++i) {
        xp = polymulmod(xp, xp, f, e);
        if (poly_gcd(f, xp ^ 2u) != 1u) return false;
    }
    return true;
}

// Column d of the reduction matrix: the bits of x^d mod f.
inline uint32_t x_pow_mod(int d, uint32_t f, int e)
{
    uint32_t r = 1;
    for (int i = 0; i < d; ++i) {
        r <<= 1;
        if ((r >> e) & 1u) r ^= f;
    }
    return r;
}

// Multiplicative order of a nonzero element a.
inline uint32_t element_order(uint32_t a, uint32_t f, int e)
{
    uint32_t x = a, k = 1;
    while (x != 1u) {
        x = polymulmod(x, a, f, e);
        ++k;
    }
    return k;
}

// Smallest generator of the multiplicative group of F_2[x]/<f> (it is cyclic
// of order 2^e - 1; f need not be primitive).
inline uint32_t find_generator(int e, uint32_t f)
{
    const uint32_t q = (1u << e) - 1u;
    for (uint32_t g = 2; g <= q; ++g)
        if (element_order(g, f, e) == q) return g;
    return 1u;  // F_4 has q = 3 and generator 2; only reached for e < 2
}

}  // namespace gf2e
