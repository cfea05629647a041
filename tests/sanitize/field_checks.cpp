// Runs the product library's host-side field set-up (irreducibility test,
// reduction columns, generators, the Karatsuba schedules and the folded field
// schedules) over every case it serves and checks each against a definition
// written out here.  The test suite builds this file under AddressSanitizer
// and UndefinedBehaviorSanitizer.  Exit status 0: every check passed.
#include <cstdint>
#include <cstdio>

#include "field.hpp"

using namespace gf2e;

static int failures = 0;
#define CHECK(cond, ...)                                              \
    do {                                                              \
        if (!(cond)) {                                                \
            ++failures;                                               \
            std::fprintf(stderr, "%s:%d: ", __FILE__, __LINE__);      \
            std::fprintf(stderr, __VA_ARGS__);                        \
            std::fputc('\n', stderr);                                 \
        }                                                             \
    } while (0)

static uint64_t state = 0x243F6A8885A308D3ull;
static uint32_t rnd()  // splitmix64
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return uint32_t((z ^ (z >> 31)) >> 16);
}

static int deg(uint64_t p)
{
    int d = -1;
    while (p) { ++d; p >>= 1; }
    return d;
}
// Remainder of a by b in F_2[x], by long division.
static uint64_t rem(uint64_t a, uint64_t b)
{
    while (deg(a) >= deg(b)) a ^= b << (deg(a) - deg(b));
    return a;
}
// Carry-less product of a and b.
static uint64_t clmul(uint64_t a, uint64_t b)
{
    uint64_t r = 0;
    for (int i = 0; i < 32; ++i)
        if ((b >> i) & 1u) r ^= a << i;
    return r;
}
// Irreducible iff no polynomial of degree 1..e/2 divides f (trial division).
static bool irreducible_by_division(int e, uint32_t f)
{
    for (uint32_t d = 2; deg(d) <= e / 2; ++d)
        if (rem(f, d) == 0) return false;
    return true;
}
static int parity(uint64_t x) { return __builtin_popcountll(x) & 1; }

int main()
{
    // Irreducibility over every f of degree e, e <= 12, and a sample above.
    for (int e = 1; e <= 16; ++e) {
        const uint32_t lo = 1u << e, hi = 2u << e;
        for (uint32_t f = lo; f < hi; f += (e <= 12 ? 1u : 97u))
            CHECK(is_irreducible(e, f) == irreducible_by_division(e, f), "e=%d f=%#x", e, f);
        // f of another degree (and f = 0) is never accepted
        CHECK(!is_irreducible(e, 0u), "e=%d f=0", e);
        CHECK(!is_irreducible(e, lo >> 1), "e=%d short f", e);
        CHECK(!is_irreducible(e, hi | 3u), "e=%d long f", e);
    }
    // Reduction columns, field products and generators for one f per degree.
    static const uint32_t polys[17] = {0, 0x3, 0x7, 0xB, 0x13, 0x25, 0x43, 0x83, 0x11D, 0x211, 0x409,
                                       0x805, 0x1053, 0x201B, 0x4443, 0x8003, 0x1002B};
    for (int e = 2; e <= 16; ++e) {
        const uint32_t f = polys[e];
        CHECK(is_irreducible(e, f), "e=%d f=%#x", e, f);
        for (int d = 0; d < 2 * e - 1; ++d)
            CHECK(x_pow_mod(d, f, e) == rem(uint64_t(1) << d, f), "x^%d mod %#x", d, f);
        for (int s = 0; s < 2000; ++s) {
            const uint32_t a = rnd() & ((1u << e) - 1u), b = rnd() & ((1u << e) - 1u);
            CHECK(polymulmod(a, b, f, e) == rem(clmul(a, b), f), "e=%d %u*%u", e, a, b);
        }
        if (e <= 12) {
            const uint32_t g = find_generator(e, f);
            CHECK(element_order(g, f, e) == (1u << e) - 1u, "generator e=%d", e);
        }
    }
    // Karatsuba schedules: P_s = (a restricted to u[s]) (b restricted to v[s]),
    // coefficient d of a*b = XOR of P_s over s in w[d].
    for (int n = 1; n <= kMaxE; ++n) {
        const Schedule s = build_schedule(n);
        CHECK(s.n == n && s.t == num_products(n) && s.t <= kMaxT, "schedule n=%d t=%d", n, s.t);
        for (int trial = 0; trial < (n <= 5 ? 1024 : 3000); ++trial) {
            uint32_t a, b;
            if (n <= 5) { a = uint32_t(trial) & ((1u << n) - 1u); b = uint32_t(trial >> n) & ((1u << n) - 1u); }
            else { a = rnd() & ((1u << n) - 1u); b = rnd() & ((1u << n) - 1u); }
            uint64_t c = 0;
            for (int d = 0; d < 2 * n - 1; ++d) {
                int bit = 0;
                for (int p = 0; p < s.t; ++p)
                    if ((s.w[d] >> p) & 1u) bit ^= parity(a & s.u[p]) & parity(b & s.v[p]);
                c |= uint64_t(bit) << d;
            }
            CHECK(c == clmul(a, b), "schedule n=%d a=%u b=%u", n, a, b);
        }
    }
    // Folded field schedules: result plane r = XOR over products s with bit
    // r of c[s] of (a restricted to a[s]) (b restricted to b[s]).
    for (const FieldSchedule& fs : kFieldSchedules) {
        const int e = fs.e;
        CHECK(is_irreducible(e, fs.f) && fs.t <= 64, "field schedule e=%d", e);
        const int trials = e <= 8 ? (1 << (2 * e)) : 20000;
        for (int trial = 0; trial < trials; ++trial) {
            uint32_t a, b;
            if (e <= 8) { a = uint32_t(trial) & ((1u << e) - 1u); b = uint32_t(trial >> e); }
            else { a = rnd() & ((1u << e) - 1u); b = rnd() & ((1u << e) - 1u); }
            uint32_t c = 0;
            for (int p = 0; p < fs.t; ++p)
                if (parity(a & fs.a[p]) & parity(b & fs.b[p])) c ^= fs.c[p];
            CHECK(c == polymulmod(a, b, fs.f, e), "field schedule e=%d f=%#x a=%u b=%u", e, fs.f, a, b);
        }
    }
    if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
    else std::printf("field checks passed\n");
    return failures ? 1 : 0;
}
