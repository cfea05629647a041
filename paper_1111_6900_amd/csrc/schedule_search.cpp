// schedule_search: looks for bilinear schedules with few GF(2) products for
// multiplication in F_2[x]/<f> (not part of the library; run by
// gen_schedules.py, whose output table the kernels compile in).
//
// A schedule is a list of rank-one terms (a, b, c): product s multiplies
// (XOR_{i in a} A_i) by (XOR_{j in b} B_j) and is added to every result plane
// in c.  It is correct when, for all i, j < e, the terms with i in a and j in
// b add up to the bits of x^(i+j) mod f -- the multiplication tensor of the
// field with the reduction of Section 5 folded in.
//
// Method: a random walk on the "flip graph" of such decompositions.  Two
// terms sharing a factor can be rewritten into two other terms with the same
// sum (a flip); a term with a zero factor disappears, and two terms sharing
// two factors merge into one.  Starting from the Karatsuba schedule of
// gf2e_schedule.hpp, the walk applies random flips, merges whenever
// possible, and occasionally splits a term in two to leave a plateau.
//
// usage: schedule_search e f seconds [seed] [target] [-]
// With "-" the walk starts from the schedule read from stdin (lines "a b c")
// instead of Karatsuba.  Prints "rank r" for the best schedule, then its
// terms "a b c" (decimal).
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "gf2e_schedule.hpp"

namespace {

struct Term {
    uint32_t a, b, c;
};

int g_e;
uint32_t g_f;

uint32_t xpow_mod(int d)
{
    uint32_t r = 1;
    for (int i = 0; i < d; ++i) {
        r <<= 1;
        if ((r >> g_e) & 1u) r ^= g_f;
    }
    return r;
}

bool is_schedule(const std::vector<Term>& s)
{
    for (int i = 0; i < g_e; ++i)
        for (int j = 0; j < g_e; ++j) {
            uint32_t acc = 0;
            for (const Term& t : s)
                if (((t.a >> i) & 1u) && ((t.b >> j) & 1u)) acc ^= t.c;
            if (acc != xpow_mod(i + j)) return false;
        }
    return true;
}

// Drops terms with a zero factor and merges terms that share two factors.
void simplify(std::vector<Term>& s)
{
    for (bool again = true; again;) {
        again = false;
        for (size_t i = 0; i < s.size() && !again; ++i)
            if (!s[i].a || !s[i].b || !s[i].c) {
                s[i] = s.back();
                s.pop_back();
                again = true;
            }
        for (size_t i = 0; i < s.size() && !again; ++i)
            for (size_t j = i + 1; j < s.size() && !again; ++j) {
                Term &x = s[i], &y = s[j];
                if (x.a == y.a && x.b == y.b) x.c ^= y.c;
                else if (x.a == y.a && x.c == y.c) x.b ^= y.b;
                else if (x.b == y.b && x.c == y.c) x.a ^= y.a;
                else continue;
                s[j] = s.back();
                s.pop_back();
                again = true;
            }
    }
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc < 4) {
        std::fprintf(stderr, "usage: %s e f seconds [seed] [target] [-]\n", argv[0]);
        return 2;
    }
    g_e = std::atoi(argv[1]);
    g_f = uint32_t(std::strtoul(argv[2], nullptr, 0));
    const double seconds = std::atof(argv[3]);
    const auto t_end = std::chrono::steady_clock::now() +
                       std::chrono::milliseconds(long(seconds * 1000.0));
    const unsigned long seed = argc > 4 ? std::strtoul(argv[4], nullptr, 10) : 1;
    const size_t target = argc > 5 ? size_t(std::atoi(argv[5])) : 0;
    if (g_e < 2 || g_e > gf2e::kMaxE) return 2;

    std::vector<Term> s;
    if (argc > 6 && argv[6][0] == '-') {
        // Start: the schedule on stdin.
        unsigned a, b, c;
        while (std::scanf("%u %u %u", &a, &b, &c) == 3) s.push_back({a, b, c});
    } else {
        // Start: the Karatsuba schedule with the reduction mod f folded into c.
        const gf2e::Schedule K = gf2e::build_schedule(g_e);
        for (int p = 0; p < K.t; ++p) {
            uint32_t c = 0;
            for (int d = 0; d < 2 * g_e - 1; ++d)
                if ((K.w[d] >> p) & 1u) c ^= xpow_mod(d);
            s.push_back({K.u[p], K.v[p], c});
        }
    }
    simplify(s);
    if (!is_schedule(s)) return 1;
    std::vector<Term> best = s;
    std::mt19937_64 rng(seed);
    std::vector<std::pair<int, int>> flips;
    const long plateau_limit = 3000;
    const size_t band = 3;
    long plateau = 0;
    for (long it = 0; best.size() > target; ++it) {
        if ((it & 4095) == 0 && std::chrono::steady_clock::now() > t_end) break;
        flips.clear();
        for (int i = 0; i < int(s.size()); ++i)
            for (int j = 0; j < int(s.size()); ++j) {
                if (i == j) continue;
                if (s[i].a == s[j].a) flips.push_back({i, 3 * j});
                if (s[i].b == s[j].b) flips.push_back({i, 3 * j + 1});
                if (s[i].c == s[j].c) flips.push_back({i, 3 * j + 2});
            }
        if (flips.empty() || (plateau > plateau_limit && rng() % 64 == 0)) {
            // Split: (a, b, c) = (a + a', b, c) + (a', b, c) with a' taken
            // from another term (likewise for b or c).
            const int i = int(rng() % s.size()), j = int(rng() % s.size());
            if (i == j) continue;
            const Term x = s[i], y = s[j];
            switch (rng() % 3) {
                case 0: if (x.a != y.a) { s[i].a ^= y.a; s.push_back({y.a, x.b, x.c}); } break;
                case 1: if (x.b != y.b) { s[i].b ^= y.b; s.push_back({x.a, y.b, x.c}); } break;
                default: if (x.c != y.c) { s[i].c ^= y.c; s.push_back({x.a, x.b, y.c}); } break;
            }
            plateau = 0;
            continue;
        }
        const auto [i, jk] = flips[rng() % flips.size()];
        Term &x = s[i], &y = s[jk / 3];
        switch (jk % 3) {
            case 0: x.b ^= y.b; y.c ^= x.c; break;  // shared a
            case 1: x.a ^= y.a; y.c ^= x.c; break;  // shared b
            default: x.a ^= y.a; y.b ^= x.b; break; // shared c
        }
        simplify(s);
        ++plateau;
        if (s.size() < best.size()) {
            if (!is_schedule(s)) return 1;
            best = s;
            plateau = 0;
        }
        if (s.size() > best.size() + band) s = best;
    }
    if (!is_schedule(best)) return 1;
    std::printf("rank %zu\n", best.size());
    for (const Term& t : best) std::printf("%u %u %u\n", t.a, t.b, t.c);
    return 0;
}
