// Karatsuba-style bilinear schedules for the product of two polynomials of
// length n over F_2 (the Bradshaw-Boothby reduction of Section 5 of the M4RIE
// paper: a product over F_{2^e} becomes a product of polynomials whose
// coefficients are GF(2) matrices, followed by reduction modulo f).
//
// A schedule with t products computes, for A = sum_i A_i x^i and
// B = sum_j B_j x^j (i, j < n),
//     P_s = (XOR_{i in u[s]} A_i) * (XOR_{j in v[s]} B_j)        s < t
//     C~_d = XOR_{s in w[d]} P_s                                   d < 2n-1
// with C~ = A * B as polynomials.  Built recursively from
//   * the 2-way split of Section 5 (its F_4 example is the n = 2 case:
//     P_0 = A_0 B_0, P_1 = A_1 B_1, P_2 = (A_0+A_1)(B_0+B_1)),
//     C = L + x^lo (M + L + H) + x^(2 lo) H, and
//   * a 3-way split with six block products,
//     c0 = P00, c1 = P01+P00+P11, c2 = P02+P00+P11+P22, c3 = P12+P11+P22,
//     c4 = P22,
// taking whichever needs fewer products.  Counts for n = 2..16 are
// 3, 6, 9, 15, 18, 24, 27, 36, 45, 51, 54, 66, 72, 78, 81 (the paper's Table 3
// lists 3, 6, 9 and 27 as the best known for n = 2, 3, 4, 8).
//
// Everything here is constexpr so that the device kernels can take the
// schedule as compile-time constants; the host library uses the same
// functions for its own set-up and for the exported schedule query.
#pragma once
#include <cstdint>

namespace gf2e {

constexpr int kMaxE = 16;
constexpr int kMaxT = 96;  // t(16) = 81
constexpr int kMaxD = 2 * kMaxE - 1;

// A set of products s < kMaxT, one bit each.
using ProductMask = unsigned __int128;
constexpr ProductMask product_bit(int s) { return ProductMask(1) << s; }

struct Schedule {
    int n = 0;
    int t = 0;
    uint32_t u[kMaxT] = {};
    uint32_t v[kMaxT] = {};
    ProductMask w[kMaxD] = {};
};

constexpr int split2_count(int n, int lo);
constexpr int split3_count(int n);

// Fewest products over the constructions above.
constexpr int best_count(int n)
{
    if (n <= 1) return 1;
    int best = n * n;  // schoolbook
    for (int lo = (n + 1) / 2; lo < n; ++lo) {
        int c = split2_count(n, lo);
        if (c < best) best = c;
    }
    int c3 = split3_count(n);
    if (c3 > 0 && c3 < best) best = c3;
    return best;
}

constexpr int split2_count(int n, int lo) { return 2 * best_count(lo) + best_count(n - lo); }

constexpr int split3_count(int n)
{
    int b = (n + 2) / 3;
    int last = n - 2 * b;
    if (n < 3 || last < 1) return 0;
    return 5 * best_count(b) + best_count(last);
}

// Appends sub (a schedule for length sub.n) whose i-th input coefficient is
// the XOR of the original coefficients in amap[i]; returns the index of its
// first product in dst.
constexpr int append_sub(Schedule& dst, const Schedule& sub, const uint32_t* amap)
{
    int off = dst.t;
    for (int s = 0; s < sub.t; ++s) {
        uint32_t uu = 0, vv = 0;
        for (int i = 0; i < sub.n; ++i) {
            if ((sub.u[s] >> i) & 1u) uu ^= amap[i];
            if ((sub.v[s] >> i) & 1u) vv ^= amap[i];
        }
        dst.u[off + s] = uu;
        dst.v[off + s] = vv;
    }
    dst.t += sub.t;
    return off;
}

// dst.w[d + shift] ^= sub.w[d] (renumbered by the product offset off).
constexpr void add_poly(Schedule& dst, const Schedule& sub, int off, int shift)
{
    for (int d = 0; d < 2 * sub.n - 1; ++d) dst.w[d + shift] ^= sub.w[d] << off;
}

constexpr Schedule build_schedule(int n);

constexpr Schedule build_schoolbook(int n)
{
    Schedule s{};
    s.n = n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            s.u[s.t] = 1u << i;
            s.v[s.t] = 1u << j;
            s.w[i + j] ^= product_bit(s.t);
            ++s.t;
        }
    return s;
}

constexpr Schedule build_split2(int n, int lo)
{
    const int hi = n - lo;
    Schedule s{};
    s.n = n;
    Schedule L = build_schedule(lo), H = build_schedule(hi), M = build_schedule(lo);
    uint32_t mapL[kMaxE] = {}, mapH[kMaxE] = {}, mapM[kMaxE] = {};
    for (int i = 0; i < lo; ++i) {
        mapL[i] = 1u << i;
        mapM[i] = (1u << i) | (lo + i < n ? 1u << (lo + i) : 0u);
    }
    for (int i = 0; i < hi; ++i) mapH[i] = 1u << (lo + i);
    int oL = append_sub(s, L, mapL);
    int oH = append_sub(s, H, mapH);
    int oM = append_sub(s, M, mapM);
    // C = L + x^lo (M + L + H) + x^(2 lo) H
    add_poly(s, L, oL, 0);
    add_poly(s, M, oM, lo);
    add_poly(s, L, oL, lo);
    add_poly(s, H, oH, lo);
    add_poly(s, H, oH, 2 * lo);
    return s;
}

constexpr Schedule build_split3(int n)
{
    const int b = (n + 2) / 3;
    const int last = n - 2 * b;
    Schedule s{};
    s.n = n;
    Schedule Kb = build_schedule(b), Kl = build_schedule(last);
    uint32_t m0[kMaxE] = {}, m1[kMaxE] = {}, m2[kMaxE] = {};
    uint32_t m01[kMaxE] = {}, m02[kMaxE] = {}, m12[kMaxE] = {};
    for (int i = 0; i < b; ++i) {
        m0[i] = 1u << i;
        m1[i] = 1u << (b + i);
        uint32_t a2 = i < last ? 1u << (2 * b + i) : 0u;
        m01[i] = m0[i] | m1[i];
        m02[i] = m0[i] | a2;
        m12[i] = m1[i] | a2;
    }
    for (int i = 0; i < last; ++i) m2[i] = 1u << (2 * b + i);
    int o00 = append_sub(s, Kb, m0);
    int o11 = append_sub(s, Kb, m1);
    int o22 = append_sub(s, Kl, m2);
    int o01 = append_sub(s, Kb, m01);
    int o02 = append_sub(s, Kb, m02);
    int o12 = append_sub(s, Kb, m12);
    // c0 = P00
    add_poly(s, Kb, o00, 0);
    // c1 = P01 + P00 + P11
    add_poly(s, Kb, o01, b);
    add_poly(s, Kb, o00, b);
    add_poly(s, Kb, o11, b);
    // c2 = P02 + P00 + P11 + P22
    add_poly(s, Kb, o02, 2 * b);
    add_poly(s, Kb, o00, 2 * b);
    add_poly(s, Kb, o11, 2 * b);
    add_poly(s, Kl, o22, 2 * b);
    // c3 = P12 + P11 + P22
    add_poly(s, Kb, o12, 3 * b);
    add_poly(s, Kb, o11, 3 * b);
    add_poly(s, Kl, o22, 3 * b);
    // c4 = P22
    add_poly(s, Kl, o22, 4 * b);
    return s;
}

constexpr Schedule build_schedule(int n)
{
    if (n <= 1) return build_schoolbook(1);
    const int best = best_count(n);
    for (int lo = (n + 1) / 2; lo < n; ++lo)
        if (split2_count(n, lo) == best) return build_split2(n, lo);
    if (split3_count(n) == best) return build_split3(n);
    return build_schoolbook(n);
}

constexpr int num_products(int e) { return best_count(e); }

}  // namespace gf2e

#include "gf2e_field_schedules.hpp"

namespace gf2e {

// The schedule a set of kernels runs.  sid = -1: the Karatsuba schedule for
// e, whose 2e-1 coefficient planes w are reduced modulo f at run time.
// sid >= 0: kFieldSchedules[sid], a schedule for one field with the reduction
// folded in, so that result plane c is the XOR of the products s with c in
// c[s].  u and v are the operand subsets of the A and B sides.
// sid = kIdentitySchedule: t = e, operand s is bit-plane s and result plane s
// is product s; the alpha-power form uses it to slice A into its bit-planes
// and to cling its e result planes.
constexpr int kIdentitySchedule = -2;
struct KernelSchedule {
    int e = 0;
    int t = 0;
    bool folded = false;
    uint32_t u[kMaxT] = {}, v[kMaxT] = {}, c[kMaxT] = {};
    ProductMask w[kMaxD] = {};
};

constexpr KernelSchedule kernel_schedule(int e, int sid)
{
    KernelSchedule k{};
    if (sid == kIdentitySchedule) {
        k.e = e;
        k.t = e;
        k.folded = true;
        for (int s = 0; s < e; ++s) k.u[s] = k.v[s] = k.c[s] = 1u << s;
    } else if (sid < 0) {
        const Schedule S = build_schedule(e);
        k.e = e;
        k.t = S.t;
        for (int s = 0; s < S.t; ++s) {
            k.u[s] = S.u[s];
            k.v[s] = S.v[s];
        }
        for (int d = 0; d < 2 * e - 1; ++d) k.w[d] = S.w[d];
    } else {
        const FieldSchedule& F = kFieldSchedules[sid];
        k.e = F.e;
        k.t = F.t;
        k.folded = true;
        for (int s = 0; s < F.t; ++s) {
            k.u[s] = F.a[s];
            k.v[s] = F.b[s];
            k.c[s] = F.c[s];
        }
    }
    return k;
}

// Index of the field schedule for (e, f), or -1 (use Karatsuba + reduction).
constexpr int find_field_schedule(int e, uint32_t f)
{
    for (int i = 0; i < kNumFieldSchedules; ++i)
        if (kFieldSchedules[i].e == e && kFieldSchedules[i].f == f) return i;
    return -1;
}

}  // namespace gf2e
