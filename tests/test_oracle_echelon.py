"""Pins of the oracle's echelon forms (Section 4.1 elimination, Section 6),
without a GPU.

What fixes the answer independently of the elimination loop: the reduced
row echelon form is the unique matrix in that form with the same row space,
so RREF(M A) = RREF(A) for every invertible M (M A formed with the textbook
product of tests/fielddef.py); for tiny matrices the row space and the rank
are found by enumerating all combinations of the rows."""
import itertools

import numpy as np
import pytest

import oracle
import workload
from tests import fielddef

FIELDS = sorted(workload.DEFAULT_POLY.items()) + [(4, 0x1F), (8, 0x11B)]


def row_space(A, e, f):
    """All vectors sum_i c_i A_i (c in F^m) as a set of tuples."""
    A = np.asarray(A, dtype=np.int64)
    q = 1 << e
    out = set()
    for coeffs in itertools.product(range(q), repeat=A.shape[0]):
        v = np.zeros(A.shape[1], dtype=np.int64)
        for c, row in zip(coeffs, A):
            v ^= fielddef.mul(c, row, e, f)
        out.add(tuple(v))
    return out


def check_structure(E, rank, piv, full):
    E = np.asarray(E, dtype=np.int64)
    m, n = E.shape
    assert (E[rank:] == 0).all()
    assert list(piv) == sorted(set(piv))
    for t in range(rank):
        j = piv[t]
        assert E[t, j] == 1 and (E[t, :j] == 0).all()
        below = E[t + 1:, j]
        assert (below == 0).all()
        if full:
            assert (E[:t, j] == 0).all()


@pytest.mark.parametrize("e,f", [(2, 0x7), (3, 0xB)])
def test_brute_force_rank_and_row_space(e, f):
    gen = np.random.default_rng(e)
    for trial in range(40):
        m, n = int(gen.integers(1, 4)), int(gen.integers(1, 5))
        A = workload.field_matrix(gen, m, n, e)
        if trial % 3 == 0 and m > 1:
            A[-1] = fielddef.mul(int(gen.integers(0, 1 << e)), A[0], e, f)  # a dependent row
        E, r, piv = oracle.echelon(A, e, f)
        space = row_space(A, e, f)
        assert len(space) == (1 << e) ** r
        assert row_space(E, e, f) == space
        check_structure(E, r, piv, True)


def random_invertible(gen, m, e, f):
    L = np.tril(workload.field_matrix(gen, m, m, e).astype(np.int64), -1) + np.eye(m, dtype=np.int64)
    U = np.triu(workload.field_matrix(gen, m, m, e).astype(np.int64), 1)
    np.fill_diagonal(U, gen.integers(1, 1 << e, m))
    return fielddef.matmul(L, U, e, f)


@pytest.mark.parametrize("e,f", FIELDS)
@pytest.mark.parametrize("shape", [(12, 20), (20, 12), (16, 16)])
def test_left_invertible_factor_does_not_change_rref(e, f, shape):
    gen = np.random.default_rng(e * 31 + shape[0])
    m, n = shape
    # rank-deficient input: a product of two thinner factors
    k = min(m, n) - 3
    A = fielddef.matmul(workload.field_matrix(gen, m, k, e), workload.field_matrix(gen, k, n, e), e, f)
    E1, r1, p1 = oracle.echelon(A, e, f)
    MA = fielddef.matmul(random_invertible(gen, m, e, f), A, e, f)
    E2, r2, p2 = oracle.echelon(MA, e, f)
    assert r1 == r2 <= k and (E1 == E2).all() and (p1 == p2).all()
    check_structure(E1, r1, p1, True)
    # the non-reduced form has the same rank and pivots, and reduces to the same RREF
    Eh, rh, ph = oracle.echelon(A, e, f, full=False)
    check_structure(Eh, rh, ph, False)
    assert rh == r1 and (ph == p1).all()
    assert (oracle.echelon(Eh, e, f)[0] == E1).all()


@pytest.mark.parametrize("e,f", [(4, 0x13), (10, 0x409)])
def test_special_cases(e, f):
    gen = np.random.default_rng(7)
    M = random_invertible(gen, 9, e, f)
    E, r, piv = oracle.echelon(M, e, f)
    assert r == 9 and (E == np.eye(9)).all() and list(piv) == list(range(9))
    Z = np.zeros((5, 7), dtype=np.int64)
    assert oracle.echelon(Z, e, f)[1] == 0
    X = workload.field_matrix(gen, 6, 4, e)
    IX = np.concatenate([np.eye(6, dtype=np.int64), X], axis=1)
    E, r, _ = oracle.echelon(IX, e, f)
    assert r == 6 and (E == IX).all()
    with pytest.raises(oracle.OracleError, match="-5"):
        oracle.echelon(np.full((2, 2), 1 << e), e, f)
