"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: values the
paper prints (Figure 1, the F_4 reduction of the Section 5 example), worked
values from the AES standard, hand-derived powers, the field axioms, an
independent numpy definition (tests/fielddef.py) and brute force on tiny
inputs.
"""
import os

import numpy as np
import pytest

import oracle
import workload
from tests import fielddef

ALL_FIELDS = sorted(workload.DEFAULT_POLY.items())


def test_default_polynomials_are_primitive():
    for e, f in ALL_FIELDS:
        assert fielddef.is_irreducible(e, f)
        assert oracle.is_irreducible(e, f)
        assert oracle.is_primitive(e, f), (e, hex(f))
        assert oracle.order(e, f, 2) == (1 << e) - 1


def test_reducible_and_non_primitive_polynomials():
    # x^2+1 = (x+1)^2 and x^4+1 = (x+1)^4 are reducible.
    for e, f in [(2, 0x5), (4, 0x11), (8, 0x101), (3, 0x9)]:
        assert not fielddef.is_irreducible(e, f)
        assert not oracle.is_irreducible(e, f)
    # x^4+x^3+x^2+x+1 is irreducible, but x has order 5 (x^5 = 1).
    assert oracle.is_irreducible(4, 0x1F) and not oracle.is_primitive(4, 0x1F)
    assert oracle.order(4, 0x1F, 2) == 5
    # The AES polynomial is irreducible, not primitive.
    assert oracle.is_irreducible(8, 0x11B) and not oracle.is_primitive(8, 0x11B)
    # Degree must match e.
    assert not oracle.is_irreducible(3, 0x13)


def test_figure1_encoding(golden_dir):
    meta, _ = fielddef.read_golden(os.path.join(golden_dir, "fig1_f8.txt"))
    e = meta["e"][0]
    f = 0xB  # any cubic works for the encoding; products below use x^3+x+1
    packed = meta["packed"]
    # alpha^2+1, alpha, alpha+1, 1 as integers sum a_i 2^i.
    assert packed == [0b101, 0b010, 0b011, 0b001]
    # Slice i holds bit i of every entry.
    for i in range(e):
        assert meta[f"slice{i}"] == [(v >> i) & 1 for v in packed]
    # alpha*alpha = alpha^2, (alpha+1)^2 = alpha^2+1 in characteristic 2,
    # alpha^2*alpha = alpha^3 = alpha+1 modulo x^3+x+1.
    assert oracle.mul_def(e, f, 2, 2) == 4
    assert oracle.mul_def(e, f, 3, 3) == 5
    assert oracle.mul_def(e, f, 4, 2) == 3


def test_f4_table_from_section5(golden_dir):
    meta, rows = fielddef.read_golden(os.path.join(golden_dir, "f4_table.txt"))
    e, f = meta["e"][0], meta["f"][0]
    expect = np.array(rows)
    assert (oracle.mul_table(e, f) == expect).all()
    for a in range(4):
        for b in range(4):
            assert oracle.mul_def(e, f, a, b) == expect[a, b]
    # In F_4 the element x satisfies x*x = x+1 (2 -> 3).
    assert oracle.mul_def(e, f, 2, 2) == 3


def test_f256_powers(golden_dir):
    meta, rows = fielddef.read_golden(os.path.join(golden_dir, "f256_11d_powers.txt"))
    e, f = meta["e"][0], meta["f"][0]
    x = 1
    powers = {}
    for i in range(15):
        powers[i] = x
        x = oracle.mul_def(e, f, x, 2)
    for i, v in rows:
        assert powers[i] == v, (i, hex(powers[i]), hex(v))
    T = oracle.mul_table(e, f)
    assert T[0x1D, 2] == 0x3A and T[0xE8, 2] == 0xCD


def test_aes_products(golden_dir):
    meta, rows = fielddef.read_golden(os.path.join(golden_dir, "aes_11b_products.txt"))
    e, f = meta["e"][0], meta["f"][0]
    T = oracle.mul_table(e, f)
    for a, b, ab in rows:
        assert oracle.mul_def(e, f, a, b) == ab
        assert T[a, b] == ab and T[b, a] == ab


@pytest.mark.parametrize("e,f", ALL_FIELDS + [(4, 0x1F), (8, 0x11B)])
def test_tables_match_definition(e, f):
    T = oracle.mul_table(e, f)
    assert (T == fielddef.table(e, f)).all()
    # The antilog table visits every nonzero element once.
    exp = oracle.antilog(e, f)
    assert sorted(exp.tolist()) == list(range(1, 1 << e))
    g = oracle.generator(e, f)
    assert oracle.order(e, f, g) == (1 << e) - 1


@pytest.mark.parametrize("e,f", [(e, f) for e, f in ALL_FIELDS if e <= 6] + [(4, 0x1F)])
def test_field_axioms_exhaustive(e, f):
    T = oracle.mul_table(e, f).astype(np.int64)
    s = np.arange(1 << e)
    assert (T == T.T).all()                      # commutative
    assert (T[1] == s).all() and (T[0] == 0).all()  # identity, zero
    # associative: (a*b)*c == a*(b*c) for all triples
    ab = T[s[:, None], s[None, :]]
    lhs = T[ab[:, :, None], s[None, None, :]]
    rhs = T[s[:, None, None], T[s[None, :, None], s[None, None, :]]]
    assert (lhs == rhs).all()
    # distributive: a*(b^c) == a*b ^ a*c
    bc = s[:, None] ^ s[None, :]
    assert (T[s[:, None, None], bc[None]] == (T[:, :, None] ^ T[:, None, :])).all()
    # inverses: every nonzero row holds 1 exactly once
    assert ((T[1:] == 1).sum(axis=1) == 1).all()


@pytest.mark.parametrize("e,f", [(e, f) for e, f in ALL_FIELDS if e > 6] + [(8, 0x11B)])
def test_field_axioms_random(e, f):
    T = oracle.mul_table(e, f).astype(np.int64)
    g = np.random.default_rng(e)
    a, b, c = (g.integers(0, 1 << e, 20000) for _ in range(3))
    assert (T[T[a, b], c] == T[a, T[b, c]]).all()
    assert (T[a, b ^ c] == T[a, b] ^ T[a, c]).all()
    assert (T[a, b] == T[b, a]).all()
    assert ((T[1:] == 1).sum(axis=1) == 1).all()


def _bits(g, shape):
    return g.integers(0, 2, size=shape, dtype=np.int64)


def test_section5_karatsuba_example():
    """Section 5: over F_4 with f = x^2+x+1, C = (A1B1 + A1B0 + A0B1) x
    + A0B0 + A1B1, and the Karatsuba form C1 = (A1+A0)(B1+B0) + A0B0."""
    g = np.random.default_rng(5)
    for m, k, n in [(1, 1, 1), (5, 7, 3), (16, 33, 9), (64, 64, 64)]:
        A0, A1 = _bits(g, (m, k)), _bits(g, (m, k))
        B0, B1 = _bits(g, (k, n)), _bits(g, (k, n))
        C1 = (A1 @ B1 + A1 @ B0 + A0 @ B1) % 2
        C0 = (A0 @ B0 + A1 @ B1) % 2
        K1 = ((A1 ^ A0) @ (B1 ^ B0) + A0 @ B0) % 2
        assert (K1 == C1).all()
        C = oracle.matmul(A0 + 2 * A1, B0 + 2 * B1, 2, 0x7)
        assert (C == C0 + 2 * C1).all()


def test_bruteforce_all_2x2_over_f4():
    """Every product of two 2x2 matrices over F_4 (256 x 256 pairs)."""
    mats = np.array(np.meshgrid(*[np.arange(4)] * 4, indexing="ij")).reshape(4, -1).T
    mats = mats.reshape(-1, 2, 2)                  # 256 matrices
    A = mats.reshape(-1, 2)                        # stacked vertically: 512 x 2
    B = mats.transpose(1, 0, 2).reshape(2, -1)     # side by side: 2 x 512
    C = oracle.matmul(A, B, 2, 0x7).astype(np.int64)
    T = fielddef.table(2, 0x7)
    # Block (p, q) of C is mats[p] @ mats[q].
    expect = T[mats[:, None, :, 0, None], mats[None, :, None, 0, :]] ^ \
        T[mats[:, None, :, 1, None], mats[None, :, None, 1, :]]
    got = C.reshape(256, 2, 256, 2).transpose(0, 2, 1, 3)
    assert (got == expect).all()


@pytest.mark.parametrize("e,f", ALL_FIELDS + [(4, 0x1F), (8, 0x11B)])
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 2), (17, 9, 13), (40, 65, 33)])
def test_matmul_matches_definition(e, f, shape):
    m, k, n = shape
    g = np.random.default_rng(m * 1000 + k * 10 + e)
    A = workload.field_matrix(g, m, k, e)
    B = workload.field_matrix(g, k, n, e)
    assert (oracle.matmul(A, B, e, f) == fielddef.matmul(A, B, e, f)).all()


@pytest.mark.parametrize("e,f", [(2, 0x7), (5, 0x25), (8, 0x11D), (10, 0x409)])
def test_matmul_properties(e, f):
    g = np.random.default_rng(e + 100)
    m, k, n, p = 23, 31, 19, 11
    A = workload.field_matrix(g, m, k, e)
    B = workload.field_matrix(g, k, n, e)
    B2 = workload.field_matrix(g, k, n, e)
    D = workload.field_matrix(g, n, p, e)
    mm = lambda X, Y: oracle.matmul(X, Y, e, f)
    I = np.eye(k, dtype=A.dtype)
    assert (mm(A, I) == A).all()
    assert (mm(mm(A, B), D) == mm(A, mm(B, D))).all()
    assert (mm(A, B ^ B2) == (mm(A, B) ^ mm(A, B2))).all()
    assert (mm(B.T.copy(), A.T.copy()) == mm(A, B).T).all()
    # Frobenius: squaring entrywise commutes with the product.
    sq = fielddef.table(e, f)[np.arange(1 << e), np.arange(1 << e)].astype(A.dtype)
    assert (sq[mm(A, B)] == mm(sq[A], sq[B])).all()
    # Scalar: alpha*I times B multiplies every entry by x.
    xI = (2 * np.eye(k)).astype(A.dtype)
    assert (mm(xI, B) == fielddef.mul(B, 2, e, f)).all()
    # Characteristic 2: a duplicated term cancels.
    A2 = np.concatenate([A[:, :1], A[:, :1]], axis=1)
    Bd = np.concatenate([B[:1], B[:1]], axis=0)
    assert (mm(A2, Bd) == 0).all()


def test_subfield_f4_in_f16():
    """F_4 embeds into F_16 (f = x^4+x+1) by x -> w = x^5: products of
    F_4-valued matrices agree with the e=2 product through the embedding."""
    e16, f16 = 4, 0x13
    T16 = fielddef.table(e16, f16)
    w = 1
    for _ in range(5):
        w = int(T16[w, 2])
    emb = np.array([0, 1, w, w ^ 1])
    assert T16[w, w] == (w ^ 1)  # w^2 = w + 1, as x^2 = x+1 in F_4
    g = np.random.default_rng(7)
    A = workload.field_matrix(g, 21, 30, 2)
    B = workload.field_matrix(g, 30, 12, 2)
    C4 = oracle.matmul(A, B, 2, 0x7)
    C16 = oracle.matmul(emb[A].astype(np.uint8), emb[B].astype(np.uint8), e16, f16)
    assert (C16 == emb[C4]).all()


def test_rows_entries_and_threads_agree():
    e, f = 8, 0x11D
    g = np.random.default_rng(11)
    A = workload.field_matrix(g, 70, 90, e)
    B = workload.field_matrix(g, 90, 50, e)
    C = oracle.matmul(A, B, e, f)
    assert (oracle.matmul(A, B, e, f, rows=(13, 41)) == C[13:41]).all()
    assert (oracle.matmul(A, B, e, f, nthreads=1) == C).all()
    I = g.integers(0, 70, 300)
    J = g.integers(0, 50, 300)
    assert (oracle.entries(A, B, e, f, I, J) == C[I, J]).all()


@pytest.mark.parametrize("e,f", [(2, 0x7), (8, 0x11D), (10, 0x409)])
def test_freivalds_catches_a_planted_error(e, f):
    g = np.random.default_rng(e + 7)
    A = workload.field_matrix(g, 40, 33, e)
    B = workload.field_matrix(g, 33, 29, e)
    C = oracle.matmul(A, B, e, f)
    R = workload.freivalds_vectors(g, 29, e)
    assert oracle.freivalds(A, B, C, e, f, R) == 0
    bad = C.copy()
    bad[17, 5] ^= 1
    assert oracle.freivalds(A, B, bad, e, f, R) == 1


def test_oracle_rejects_bad_input():
    A = np.array([[4]], dtype=np.uint8)
    with pytest.raises(oracle.OracleError):
        oracle.matmul(A, A, 2, 0x7)          # 4 is not in F_4
    with pytest.raises(oracle.OracleError):
        oracle.matmul(A, A, 4, 0x11)         # reducible f
    with pytest.raises(oracle.OracleError):
        oracle.entries(A, A, 2, 0x7, [0], [0])


def test_empty_inner_dimension_gives_zero():
    A = np.zeros((3, 0), dtype=np.uint8)
    B = np.zeros((0, 4), dtype=np.uint8)
    assert (oracle.matmul(A, B, 4, 0x13) == 0).all()


# Fields past the paper's range (11 <= e <= 16): the oracle's tables and
# products against the definitions, on samples (2^(2e) pairs are too many).

@pytest.mark.parametrize("e,f", sorted(workload.WIDE_POLY.items()))
def test_wide_polynomials_are_primitive(e, f):
    assert fielddef.is_irreducible(e, f)
    assert oracle.is_primitive(e, f)
    assert oracle.order(e, f, 2) == (1 << e) - 1


@pytest.mark.parametrize("e,f", sorted(workload.WIDE_POLY.items()))
def test_wide_antilog_and_products_match_definition(e, f):
    g = oracle.generator(e, f)
    ex = oracle.antilog(e, f).astype(np.int64)
    assert len(ex) == (1 << e) - 1 and len(set(ex.tolist())) == len(ex)
    gen = np.random.default_rng(e)
    idx = gen.integers(0, len(ex), 200)
    for i in idx[:20]:
        assert ex[(i + 1) % len(ex)] == oracle.mul_def(e, f, int(ex[i]), g)
    a = gen.integers(0, 1 << e, 5000)
    b = gen.integers(0, 1 << e, 5000)
    want = fielddef.mul(a, b, e, f)
    got = np.array([oracle.mul_def(e, f, int(x), int(y)) for x, y in zip(a[:300], b[:300])])
    assert (got == want[:300]).all()
    # the table-based matrix product against the definition, entry by entry
    A = workload.field_matrix(gen, 7, 11, e).astype(np.int64)
    B = workload.field_matrix(gen, 11, 5, e).astype(np.int64)
    C = np.zeros((7, 5), dtype=np.int64)
    for l in range(11):
        C ^= fielddef.mul(A[:, l][:, None], B[l][None, :], e, f)
    assert (oracle.matmul(A, B, e, f) == C).all()
