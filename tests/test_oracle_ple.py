"""Pins of the oracle's PLE decomposition (Section 4.2), without a GPU.

What fixes the answer independently of the elimination loop: A = P L E
checked with the textbook product of tests/fielddef.py; the shapes the
definition asks for (P a permutation, L lower trapezoidal with nonzero
diagonal, E in row echelon form with leading ones); the pivot columns are
the column rank profile, the same as the echelon form's; E spans the row
space of A (its reduced form equals A's); for tiny matrices the rank is the
dimension of the row space found by enumerating every combination of rows,
and every 2x2 and 2x3 matrix over F_4 is decomposed."""
import itertools

import numpy as np
import pytest

import oracle
import workload
from tests import fielddef
from tests.test_oracle_echelon import row_space

FIELDS = sorted(workload.DEFAULT_POLY.items()) + [(4, 0x1F), (8, 0x11B)]


def check_ple(A, e, f, P, L, E, Q, r):
    """Every property of a PLE decomposition of A, with independent arithmetic."""
    A = np.asarray(A, dtype=np.int64)
    L = np.asarray(L, dtype=np.int64)
    E = np.asarray(E, dtype=np.int64)
    m, n = A.shape
    assert sorted(P.tolist()) == list(range(m))                   # a permutation
    assert L.shape == (m, min(m, n)) and E.shape == (m, n)
    assert (np.triu(L, 1) == 0).all() and (L[:, r:] == 0).all()   # lower trapezoidal, m x rank
    assert all(L[t, t] != 0 for t in range(r))                     # pivots on the diagonal
    assert (E[r:] == 0).all()
    assert list(Q) == sorted(set(Q.tolist())) and len(Q) == r     # increasing pivot columns
    for t in range(r):
        assert E[t, Q[t]] == 1 and (E[t, :Q[t]] == 0).all()      # leading one
        assert (E[t + 1:, Q[t]] == 0).all()                       # zeros below it
    LE = fielddef.matmul(L[:, :r], E[:r], e, f) if r else np.zeros((m, n), dtype=np.int64)
    assert (LE == A[P]).all()                                      # A = P L E


@pytest.mark.parametrize("e,f", FIELDS)
@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (9, 9), (13, 31), (31, 13), (40, 40)])
def test_ple_random(e, f, shape):
    gen = np.random.default_rng(hash((e, f, shape)) % 2**32)
    A = workload.field_matrix(gen, *shape, e)
    P, L, E, Q, r = oracle.ple(A, e, f)
    check_ple(A, e, f, P, L, E, Q, r)
    # same rank and pivot columns as the echelon form; E spans A's row space
    R, rr, piv = oracle.echelon(A, e, f, full=True)
    assert r == rr and list(Q) == list(piv)
    R2, _, _ = oracle.echelon(E, e, f, full=True)
    assert (R2 == R).all()


@pytest.mark.parametrize("e,f", [(2, 0x7), (4, 0x13), (8, 0x11D), (10, 0x409)])
def test_ple_rank_deficient_and_special(e, f):
    gen = np.random.default_rng(42 + e)
    for m, n, k in [(30, 20, 5), (20, 30, 7), (16, 16, 1), (12, 40, 12)]:
        X = workload.field_matrix(gen, m, k, e)
        Y = workload.field_matrix(gen, k, n, e)
        A = fielddef.matmul(X, Y, e, f).astype(workload.elem_dtype(e))
        A[:, 3] = 0                                 # a zero column
        P, L, E, Q, r = oracle.ple(A, e, f)
        check_ple(A, e, f, P, L, E, Q, r)
        assert r <= k and 3 not in Q.tolist()
    Z = np.zeros((5, 6), dtype=workload.elem_dtype(e))
    P, L, E, Q, r = oracle.ple(Z, e, f)
    assert r == 0 and (E == 0).all() and (L == 0).all() and P.tolist() == list(range(5))
    # a row swap is forced: the first row is zero in the first column
    A = np.array([[0, 1], [1, 1]], dtype=workload.elem_dtype(e))
    P, L, E, Q, r = oracle.ple(A, e, f)
    assert P.tolist() == [1, 0] and r == 2
    check_ple(A, e, f, P, L, E, Q, r)


def test_ple_identity_and_diagonal():
    e, f = 8, 0x11D
    D = np.diag(np.arange(1, 9)).astype(np.uint8)
    P, L, E, Q, r = oracle.ple(D, e, f)
    assert r == 8 and P.tolist() == list(range(8)) and Q.tolist() == list(range(8))
    assert (np.diag(L) == np.arange(1, 9)).all() and (np.tril(L, -1) == 0).all()
    assert (E == np.eye(8, dtype=np.uint8)).all()


@pytest.mark.parametrize("shape", [(2, 2), (2, 3)])
def test_ple_every_small_matrix_over_f4(shape):
    """Every 2x2 and 2x3 matrix over F_4: the decomposition and its rank,
    the rank compared with the dimension of the enumerated row space."""
    e, f = 2, 0x7
    m, n = shape
    for entries in itertools.product(range(4), repeat=m * n):
        A = np.array(entries, dtype=np.uint8).reshape(m, n)
        P, L, E, Q, r = oracle.ple(A, e, f)
        check_ple(A, e, f, P, L, E, Q, r)
        assert len(row_space(A, e, f)) == 4 ** r


def test_ple_planted_mistake_is_caught():
    """The checks reject a decomposition with one wrong multiplier."""
    e, f = 4, 0x13
    A = workload.field_matrix(np.random.default_rng(5), 6, 6, e)
    P, L, E, Q, r = oracle.ple(A, e, f)
    L = L.copy()
    L[4, 1] ^= 1
    with pytest.raises(AssertionError):
        check_ple(A, e, f, P, L, E, Q, r)


def test_ple_rejects_entries_outside_the_field():
    A = np.array([[1, 4], [2, 3]], dtype=np.uint8)
    with pytest.raises(oracle.OracleError):
        oracle.ple(A, 2, 0x7)
