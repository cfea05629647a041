"""The alpha-power form of the product, checked on the CPU (no GPU).

It rests on one identity: with A_i the bit-planes of A (A = sum_i A_i x^i),
C = A*B = sum_i x^i (A_i B), so bit-plane c of C is the GF(2) sum over i of
A_i times bit-plane c of x^i B.  The rows x^k B, k < e, are the first table
of Section 4's Newton-John construction.  Here both sides come from textbook
definitions (the field product of Section 2 in tests/fielddef.py) and the
result is compared with the oracle; the GPU form is compared with the oracle
in tests/test_gpu_mul.py.
"""
import numpy as np
import pytest

import oracle
import workload
from tests import fielddef, planes_model


def x_pow_times(B, i, e, f):
    """x^i * B elementwise, by i multiplications with x (shift, fold with f)."""
    R = np.asarray(B, dtype=np.int64).copy()
    for _ in range(i):
        R = R << 1
        R = np.where((R >> e) & 1, R ^ f, R)
    return R


@pytest.mark.parametrize("e,f", sorted(workload.DEFAULT_POLY.items()) + [(4, 0x1F), (8, 0x11B)])
def test_alpha_power_identity(e, f):
    gen = np.random.default_rng(e * 7 + f)
    A = workload.field_matrix(gen, 9, 13, e)
    B = workload.field_matrix(gen, 13, 11, e)
    Abits = planes_model.bits_of(A, e)  # m, k, e
    C = np.zeros((9, 11), dtype=np.int64)
    for c in range(e):
        acc = np.zeros((9, 11), dtype=np.int64)
        for i in range(e):
            XiB_c = (x_pow_times(B, i, e, f) >> c) & 1
            acc ^= (Abits[:, :, i] @ XiB_c) & 1
        C |= acc << c
    assert (C == oracle.matmul(A, B, e, f)).all()


@pytest.mark.parametrize("e,f", [(2, 0x7), (5, 0x25), (8, 0x11D), (10, 0x409)])
def test_x_power_by_repeated_shift_is_the_field_product(e, f):
    """x^i * b computed by repeated multiplication with x equals the field
    product of x^i (the element 1 << i for i < e) and b."""
    b = np.arange(1 << e)
    for i in range(e):
        assert (x_pow_times(b, i, e, f) == fielddef.mul(1 << i, b, e, f)).all()


def test_single_product_layout():
    """The one GF(2) product [A_0 .. A_{e-1}] (m x ek) times the ek x en
    matrix with block (i, c) = plane c of x^i B has the result planes as its
    column blocks."""
    e, f = 3, 0xB
    gen = np.random.default_rng(5)
    m, k, n = 6, 10, 7
    A = workload.field_matrix(gen, m, k, e)
    B = workload.field_matrix(gen, k, n, e)
    Abits = planes_model.bits_of(A, e)
    big_a = np.concatenate([Abits[:, :, i] for i in range(e)], axis=1)  # m x ek
    big_b = np.zeros((e * k, e * n), dtype=np.int64)
    for i in range(e):
        XiB = x_pow_times(B, i, e, f)
        for c in range(e):
            big_b[i * k:(i + 1) * k, c * n:(c + 1) * n] = (XiB >> c) & 1
    P = (big_a @ big_b) & 1
    C = sum(P[:, c * n:(c + 1) * n] << c for c in range(e))
    assert (C == oracle.matmul(A, B, e, f)).all()
