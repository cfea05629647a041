"""Product schedules built through a subfield (the generator of the compiled-in
field schedules), checked on the CPU.

A schedule is checked by running it on field elements: the products it
takes of the operands' bit-planes, added into the result planes it names,
must give the product of the two elements computed by carry-less
multiplication and reduction modulo f (written out here).  Every pair is
tried for e <= 8, a seeded sample above.
"""
import os
import random
import sys

import pytest

import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_1111_6900_amd"))
import gen_schedules  # noqa: E402

# GF(2) products of one multiplication in the subfield of order 2^d
# (Karatsuba): 3, 6, 9 for d = 2, 3, 4.
SUB_COST = {2: 3, 3: 6, 4: 9}


def clmul_mod(a, b, e, f):
    r = 0
    for i in range(e):
        if (b >> i) & 1:
            r ^= a << i
    for d in range(2 * e - 2, e - 1, -1):
        if (r >> d) & 1:
            r ^= f << (d - e)
    return r


def run_schedule(terms, a, b):
    out = 0
    for ta, tb, tc in terms:
        if bin(a & ta).count("1") & 1 and bin(b & tb).count("1") & 1:
            out ^= tc
    return out


def expected_count(e, d):
    """Points of the subfield (at most 2n - 2 of them), the point at
    infinity, and quadratic places for the degrees still missing; each
    quadratic place costs three subfield products."""
    n = e // d
    need = 2 * n - 2
    pts = min(1 << d, need)
    quads = (need - pts + 1) // 2
    return (pts + 1) * SUB_COST[d] + quads * 3 * SUB_COST[d]


CASES = [(4, 0x13, 2), (4, 0x1F, 2), (6, 0x43, 2), (6, 0x43, 3), (8, 0x11D, 2), (8, 0x11B, 2),
         (8, 0x11D, 4), (9, 0x211, 3), (10, 0x409, 2), (12, 0x1053, 2), (12, 0x1053, 3),
         (14, 0x4443, 2), (15, 0x8003, 3), (16, 0x1100B, 2), (16, 0x1100B, 4)]


@pytest.mark.parametrize("e,f,d", CASES)
def test_subfield_schedule_multiplies(e, f, d):
    terms = gen_schedules.subfield_schedule(e, f, d)
    assert terms is not None
    assert len(terms) == expected_count(e, d)
    if e <= 8:
        pairs = [(a, b) for a in range(1 << e) for b in range(1 << e)]
    else:
        rng = random.Random(20260 + e)
        pairs = [(rng.randrange(1 << e), rng.randrange(1 << e)) for _ in range(3000)]
        pairs += [(1 << i, 1 << j) for i in range(e) for j in range(e)]
    for a, b in pairs:
        assert run_schedule(terms, a, b) == clmul_mod(a, b, e, f), (a, b)


def test_subfield_counts_beat_karatsuba():
    """e = 8 through F_4: 4 points, infinity and one quadratic place,
    5 * 3 + 9 = 24 products, three fewer than Karatsuba's 27 (and than the
    27 that Table 3 lists for degree 8); e = 16 through F_4: 60 against 81."""
    assert expected_count(8, 2) == 24
    assert expected_count(16, 2) == 60
    assert expected_count(9, 3) == 30 and expected_count(15, 3) == 54


def test_no_subfield_for_prime_degrees():
    for e, f in [(5, 0x25), (7, 0x83), (11, 0x805), (13, 0x201B)]:
        assert gen_schedules.best_subfield_schedule(e, f) is None


def test_compiled_tables_use_at_most_the_subfield_count():
    """The compiled-in schedule for each default field needs no more products
    than the subfield construction gives for it."""
    import paper_1111_6900_amd as g
    try:
        g.lib()
    except RuntimeError as exc:  # pragma: no cover
        pytest.skip(str(exc))
    fields = dict(workload.DEFAULT_POLY)
    fields.update(workload.WIDE_POLY)
    for e, f in sorted(fields.items()):
        sub = gen_schedules.best_subfield_schedule(e, f)
        if sub is not None:
            assert g.num_products(e, f) <= len(sub), e


def test_generator_table_entries_multiply():
    """Every entry of the generated header, parsed back, multiplies."""
    table = gen_schedules.existing_schedules()
    assert len(table) >= 10
    for (e, f), terms in table.items():
        rng = random.Random(e)
        for _ in range(500):
            a, b = rng.randrange(1 << e), rng.randrange(1 << e)
            assert run_schedule(terms, a, b) == clmul_mod(a, b, e, f), (e, a, b)
