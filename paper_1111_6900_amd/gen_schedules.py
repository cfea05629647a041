"""Generate csrc/gf2e_field_schedules.hpp: product schedules for specific fields.

For each field polynomial below there are two sources of schedules:

* subfield_schedule(): when e has a divisor d in {2, 3, 4}, the field is a
  degree-n extension of its subfield L of order 2^d (n = e/d), and a product
  of two elements is a product of two polynomials of degree < n over L,
  reduced.  That polynomial product is recovered by the Chinese remainder
  theorem from its values at points of L, its leading coefficient (the point
  at infinity) and its residues modulo monic irreducible quadratics over L
  (the interpolation construction of Toom and Winograd); each product in L or
  in a quadratic extension of L is then done by Karatsuba over F_2.  This
  gives e.g. 24 products for e = 8 (Karatsuba: 27) and 60 for e = 16 (81).
* csrc/schedule_search.cpp, a flip-graph random walk over decompositions of
  the multiplication tensor of F_2[x]/<f>, started from the better of
  Karatsuba and the subfield schedule, with several seeds.

The schedule with the fewest GF(2) products is kept if it beats Karatsuba's
count, re-verified here against x^(i+j) mod f, and written to the table.  The
kernels compile the table in; for any other f the library uses the Karatsuba
schedule and reduces modulo f at run time.

usage: python paper_1111_6900_amd/gen_schedules.py [seconds_per_field] [seeds]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(CSRC, "gf2e_field_schedules.hpp")

# Fields the tables are generated for: one polynomial per degree, those the
# library's workloads use.
FIELDS = [(5, 0x25), (6, 0x43), (7, 0x83), (8, 0x11D), (9, 0x211), (10, 0x409),
          (11, 0x805), (12, 0x1053), (13, 0x201B), (14, 0x4443), (15, 0x8003), (16, 0x1100B)]
KARATSUBA = {2: 3, 3: 6, 4: 9, 5: 15, 6: 18, 7: 24, 8: 27, 9: 36, 10: 45,
             11: 51, 12: 54, 13: 66, 14: 72, 15: 78, 16: 81}
MAX_TERMS = 64  # capacity of one table entry


def xpow_mod(d, e, f):
    r = 1
    for _ in range(d):
        r <<= 1
        if (r >> e) & 1:
            r ^= f
    return r


def is_schedule(terms, e, f):
    for i in range(e):
        for j in range(e):
            acc = 0
            for a, b, c in terms:
                if (a >> i) & 1 and (b >> j) & 1:
                    acc ^= c
            if acc != xpow_mod(i + j, e, f):
                return False
    return True


def gf_mul(a, b, e, f):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if (a >> e) & 1:
            a ^= f
    return r


def gf_pow(a, k, e, f):
    r = 1
    while k:
        if k & 1:
            r = gf_mul(r, a, e, f)
        a = gf_mul(a, a, e, f)
        k >>= 1
    return r


def parity(x):
    return bin(x).count("1") & 1


# Karatsuba products for multiplying two polynomials of d coefficients over
# F_2: product s multiplies the XOR of the coefficients in mask s of one
# factor by the same XOR of the other.
KARATSUBA_MASKS = {1: [1], 2: [1, 2, 3], 3: [1, 2, 4, 3, 5, 6],
                   4: [1, 2, 3, 4, 8, 12, 5, 10, 15]}


def solve_outputs(pairs, e, f):
    """c masks such that the products (a_s, b_s) with c_s add up to x^(i+j)
    mod f for all i, j < e (Gaussian elimination over F_2), or None."""
    R = len(pairs)
    rows = []
    for i in range(e):
        for j in range(e):
            coef = 0
            for s, (a, b) in enumerate(pairs):
                if (a >> i) & 1 and (b >> j) & 1:
                    coef |= 1 << s
            rows.append(coef | (xpow_mod(i + j, e, f) << R))
    pivots = []
    r = 0
    for col in range(R):
        p = next((k for k in range(r, len(rows)) if (rows[k] >> col) & 1), None)
        if p is None:
            continue
        rows[r], rows[p] = rows[p], rows[r]
        for k in range(len(rows)):
            if k != r and (rows[k] >> col) & 1:
                rows[k] ^= rows[r]
        pivots.append(col)
        r += 1
    if any(row and not row & ((1 << R) - 1) for row in rows[r:]):
        return None  # inconsistent: the products do not span the field product
    c = [0] * R
    for k, col in enumerate(pivots):
        c[col] = rows[k] >> R
    return c


def subfield_schedule(e, f, d):
    """Schedule for F_2[x]/<f> through its subfield of order 2^d (see the
    module docstring), or None when d does not divide e."""
    if e % d or d == e or d not in KARATSUBA_MASKS:
        return None
    n, q = e // d, 1 << e
    order = q - 1
    primes = [p for p in range(2, order + 1) if order % p == 0 and all(p % r for r in range(2, int(p ** 0.5) + 1))]
    g = next(z for z in range(2, q) if all(gf_pow(z, order // p, e, f) != 1 for p in primes))
    omega = gf_pow(g, order // ((1 << d) - 1), e, f)  # generates L*
    wpow = [gf_pow(omega, u, e, f) for u in range(d)]  # F_2-basis of L
    lcoord = {}
    for bits in range(1 << d):
        z = 0
        for u in range(d):
            if (bits >> u) & 1:
                z ^= wpow[u]
        lcoord[z] = bits
    L = sorted(lcoord)
    # F_2-basis omega^u x^i of the field (x has degree n over L); coordinates
    # of every element, so that a = sum_i a_i x^i with a_i in L.
    basis = [gf_mul(wpow[u], gf_pow(2, i, e, f), e, f) for i in range(n) for u in range(d)]
    coord = {}
    for bits in range(q):
        z = 0
        for t in range(e):
            if (bits >> t) & 1:
                z ^= basis[t]
        coord[z] = bits
    if len(coord) != q:
        return None

    def lcoefs(a):
        bits = coord[a]
        out = []
        for i in range(n):
            z = 0
            for u in range(d):
                if (bits >> (i * d + u)) & 1:
                    z ^= wpow[u]
            out.append(z)
        return out

    def lmul(x, y):
        return gf_mul(x, y, e, f)

    # Places: points of L, infinity, and monic irreducible quadratics over L,
    # until their degrees cover the 2n - 1 coefficients of the product.
    need = 2 * n - 2
    places = [("pt", p) for p in L[:need]] + [("inf", None)]
    deg = min(len(L), need)
    if deg < need:
        for q1 in L:
            for q0 in L:
                if deg >= need:
                    break
                if all(lmul(r, r) ^ lmul(q1, r) ^ q0 for r in L):  # no root in L
                    places.append(("quad", (q0, q1)))
                    deg += 2
        if deg < need:
            return None

    def residue(place, a):
        """Residue of the polynomial of a at the place, as L elements."""
        kind, data = place
        co = lcoefs(a)
        if kind == "inf":
            return [co[n - 1]]
        if kind == "pt":
            r, pk = 0, 1
            for i in range(n):
                r ^= lmul(co[i], pk)
                pk = lmul(pk, data)
            return [r]
        q0, q1 = data
        r0, r1, y0, y1 = 0, 0, 1, 0  # y^i mod (y^2 + q1 y + q0) = y0 + y1 y
        for i in range(n):
            r0 ^= lmul(co[i], y0)
            r1 ^= lmul(co[i], y1)
            y0, y1 = lmul(y1, q0), y0 ^ lmul(y1, q1)
        return [r0, r1]

    pairs = []
    for place in places:
        res = [residue(place, 1 << j) for j in range(e)]  # images of the bit basis
        # Combinations of the residue's L coordinates to multiply: the residue
        # itself, or Karatsuba over L for a quadratic place.
        combos = [[1]] if len(res[0]) == 1 else [[1, 0], [0, 1], [1, 1]]
        for cmb in combos:
            for lm in KARATSUBA_MASKS[d]:
                mask = 0
                for j in range(e):
                    z = 0
                    for k, sel in enumerate(cmb):
                        if sel:
                            z ^= res[j][k]
                    if parity(lcoord[z] & lm):
                        mask |= 1 << j
                pairs.append((mask, mask))
    c = solve_outputs(pairs, e, f)
    if c is None:
        return None
    terms = [(a, b, cc) for (a, b), cc in zip(pairs, c) if cc]
    return terms if is_schedule(terms, e, f) else None


def best_subfield_schedule(e, f):
    cands = [subfield_schedule(e, f, d) for d in (2, 3, 4)]
    cands = [c for c in cands if c]
    return min(cands, key=len) if cands else None


def run_one(exe, e, f, seconds, seed, start=None):
    try:
        args = [exe, str(e), hex(f), str(seconds), str(seed), "0"]
        stdin = None
        if start:
            args.append("-")
            stdin = "\n".join(f"{a} {b} {c}" for a, b, c in start) + "\n"
        out = subprocess.run(args, input=stdin, capture_output=True, text=True,
                             timeout=seconds + 60).stdout
    except (OSError, subprocess.TimeoutExpired):
        return None
    lines = out.strip().splitlines()
    if not lines or not lines[0].startswith("rank"):
        return None
    return [tuple(int(x) for x in l.split()) for l in lines[1:]]


def existing_schedules():
    """Entries of the table as it stands, so that a new run keeps them unless
    it finds fewer products (the walk is random and time-bounded)."""
    import re
    try:
        text = open(OUT).read()
    except OSError:
        return {}
    out = {}
    pat = re.compile(r"\{(\d+), (0x[0-9a-f]+), (\d+),\s*\{([^}]*)\},\s*\{([^}]*)\},\s*\{([^}]*)\}\}")
    for m in pat.finditer(text):
        e, f = int(m.group(1)), int(m.group(2), 16)
        cols = [[int(x) for x in m.group(k).split(",")] for k in (4, 5, 6)]
        terms = list(zip(*cols))
        if len(terms) == int(m.group(3)) and is_schedule(terms, e, f):
            out[(e, f)] = terms
    return out


def main():
    seconds = int(sys.argv[1]) if len(sys.argv) > 1 else 300
    seeds = int(sys.argv[2]) if len(sys.argv) > 2 else 8
    tmp = tempfile.mkdtemp()
    exe = os.path.join(tmp, "schedule_search")
    subprocess.check_call(["g++", "-O2", "-std=c++20", "-I", CSRC, "-o", exe,
                           os.path.join(CSRC, "schedule_search.cpp")])
    found = {}
    old = existing_schedules()
    for e, f in FIELDS:
        sub = best_subfield_schedule(e, f)
        start = sub if sub and len(sub) < KARATSUBA[e] else None
        with cf.ThreadPoolExecutor(max_workers=seeds) as ex:
            res = list(ex.map(lambda sd: run_one(exe, e, f, seconds, sd, start), range(1, seeds + 1)))
        res = [r for r in res if r and is_schedule(r, e, f)] + [r for r in (sub, old.get((e, f))) if r]
        best = min(res, key=len) if res else None
        print(f"e={e} f={f:#x}: best {len(best) if best else None} (subfield {len(sub) if sub else None},"
              f" Karatsuba {KARATSUBA[e]})", flush=True)
        if best and len(best) < KARATSUBA[e] and len(best) <= MAX_TERMS:
            found[(e, f)] = best
    write_header(found)


def write_header(found):
    lines = [
        "// Generated by paper_1111_6900_amd/gen_schedules.py -- do not edit by hand.",
        "//",
        "// Product schedules for multiplication in F_2[x]/<f> with the reduction",
        "// modulo f folded in: product s multiplies (XOR_{i in a} A_i) by",
        "// (XOR_{j in b} B_j) and is added to every result plane in c.  Each was",
        "// found by csrc/schedule_search.cpp and is checked against x^(i+j) mod f",
        "// by the generator and by the test suite.",
        "#pragma once",
        "#include <cstdint>",
        "",
        "namespace gf2e {",
        "",
        "struct FieldSchedule {",
        "    int e;",
        "    uint32_t f;",
        "    int t;",
        "    uint16_t a[64], b[64], c[64];",
        "};",
        "",
        "constexpr FieldSchedule kFieldSchedules[] = {",
    ]
    for (e, f), terms in sorted(found.items()):
        a = ", ".join(str(t[0]) for t in terms)
        b = ", ".join(str(t[1]) for t in terms)
        c = ", ".join(str(t[2]) for t in terms)
        lines.append(f"    {{{e}, {f:#x}, {len(terms)},")
        lines.append(f"     {{{a}}},")
        lines.append(f"     {{{b}}},")
        lines.append(f"     {{{c}}}}},")
    if not found:
        lines.append("    {0, 0, 0, {}, {}, {}},")
    lines += [
        "};",
        f"constexpr int kNumFieldSchedules = {len(found)};",
        "",
        "}  // namespace gf2e",
        "",
    ]
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
