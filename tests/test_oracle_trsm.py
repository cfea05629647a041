"""Pins of the oracle's triangular solver (Section 4.3), without a GPU.

The solver is checked against what fixes X = T^{-1} B independently of it:
T X = B under the textbook matrix product of tests/fielddef.py, brute force
over every 2 x 2 system over F_4, and the special cases T = I (X = B) and T
diagonal (X = each row scaled by the inverse, the inverse found by search).
"""
import itertools

import numpy as np
import pytest

import oracle
import workload
from tests import fielddef

FIELDS = sorted(workload.DEFAULT_POLY.items()) + [(4, 0x1F), (8, 0x11B)]


def random_triangular(gen, m, e, lower, unit):
    T = workload.field_matrix(gen, m, m, e).astype(np.int64)
    T = np.tril(T) if lower else np.triu(T)
    d = gen.integers(1, 1 << e, m)
    np.fill_diagonal(T, d)
    if unit:
        # the diagonal is not read: put arbitrary values (zeros included) there
        np.fill_diagonal(T, gen.integers(0, 1 << e, m))
    return T


def with_unit_diagonal(T):
    U = T.copy()
    np.fill_diagonal(U, 1)
    return U


@pytest.mark.parametrize("e,f", FIELDS)
@pytest.mark.parametrize("lower", [False, True])
@pytest.mark.parametrize("unit", [False, True])
def test_solution_satisfies_the_system(e, f, lower, unit):
    gen = np.random.default_rng(e * 11 + lower * 3 + unit)
    m, n = 23, 17
    T = random_triangular(gen, m, e, lower, unit)
    B = workload.field_matrix(gen, m, n, e)
    X = oracle.trsm(T, B, e, f, lower=lower, unit=unit).astype(np.int64)
    Teff = with_unit_diagonal(T) if unit else T
    assert (fielddef.matmul(Teff, X, e, f) == B).all()


def test_brute_force_every_2x2_system_over_f4():
    e, f = 2, 0x7
    vecs = list(itertools.product(range(4), repeat=2))
    for lower in (False, True):
        for d0, d1, t in itertools.product(range(1, 4), range(1, 4), range(4)):
            T = np.array([[d0, 0], [t, d1]]) if lower else np.array([[d0, t], [0, d1]])
            for b in vecs:
                B = np.array(b).reshape(2, 1)
                sols = [x for x in vecs
                        if (fielddef.matmul(T, np.array(x).reshape(2, 1), e, f) == B).all()]
                assert len(sols) == 1
                X = oracle.trsm(T, B, e, f, lower=lower)
                assert tuple(X[:, 0]) == sols[0]


@pytest.mark.parametrize("e,f", FIELDS)
def test_identity_and_diagonal(e, f):
    gen = np.random.default_rng(e)
    m, n = 9, 5
    B = workload.field_matrix(gen, m, n, e)
    assert (oracle.trsm(np.eye(m, dtype=np.int64), B, e, f) == B).all()
    d = gen.integers(1, 1 << e, m)
    elems = np.arange(1 << e)
    inv = [int(elems[fielddef.mul(int(x), elems, e, f) == 1][0]) for x in d]
    want = np.stack([fielddef.mul(inv[i], B[i], e, f) for i in range(m)])
    for lower in (False, True):
        assert (oracle.trsm(np.diag(d), B, e, f, lower=lower) == want).all()


def test_singular_and_range_errors():
    e, f = 4, 0x13
    T = np.triu(np.ones((4, 4), dtype=np.int64))
    T[2, 2] = 0
    B = np.ones((4, 3), dtype=np.int64)
    with pytest.raises(oracle.OracleError, match="-9"):
        oracle.trsm(T, B, e, f)
    # with unit = True the zero on the diagonal is not read
    X = oracle.trsm(T, B, e, f, unit=True)
    assert (fielddef.matmul(with_unit_diagonal(T), X.astype(np.int64), e, f) == B).all()
    T2 = np.eye(4, dtype=np.int64)
    T2[0, 3] = 16
    with pytest.raises(oracle.OracleError, match="-5"):
        oracle.trsm(T2, B, e, f)


def test_threads_agree():
    e, f = 8, 0x11D
    gen = np.random.default_rng(3)
    T = random_triangular(gen, 70, e, False, False)
    B = workload.field_matrix(gen, 70, 300, e)
    assert (oracle.trsm(T, B, e, f, nthreads=1) == oracle.trsm(T, B, e, f, nthreads=4)).all()
