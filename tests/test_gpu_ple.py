"""PLE decomposition on the GPU (gf2e_ple, Section 4.2) against the oracle.

Several PLE decompositions of one matrix exist (they differ in the pivot
rows chosen), so the unique parts are compared with the oracle bit for bit
(rank, pivot columns, the reduced form of E's row space) and the rest is
checked to be a valid decomposition: A = P L E with the oracle's product,
L lower trapezoidal with the pivots on its diagonal, E in row echelon form
with leading ones."""
import numpy as np
import pytest
import torch

import oracle
import workload
from tests import fielddef

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_1111_6900_amd as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context(0)


def dev(g, M, e):
    return torch.from_numpy(np.ascontiguousarray(M).astype(np.int64)).to(g.elem_dtype(e)).cuda()


def host(t):
    return t.cpu().numpy().astype(np.int64)


def check_gpu_ple(g, ctx, A, e, f, full_product=True):
    m, n = A.shape
    Ad = dev(g, A, e)
    L, P, Q, r = ctx.ple(Ad, e, f)
    E, Lh = host(Ad), host(L)
    R, rr, piv = oracle.echelon(A, e, f, full=True)
    assert r == rr and Q == list(piv)                                   # unique parts
    assert sorted(P) == list(range(m))
    assert Lh.shape == (m, min(m, n))
    assert (np.triu(Lh, 1) == 0).all() and (Lh[:, r:] == 0).all()
    assert all(Lh[t, t] != 0 for t in range(r))
    assert (E[r:] == 0).all()
    for t in range(r):
        assert E[t, Q[t]] == 1 and (E[t, :Q[t]] == 0).all() and (E[t + 1:, Q[t]] == 0).all()
    AP = np.asarray(A, dtype=np.int64)[P]
    if full_product:
        LE = oracle.matmul(Lh[:, :r], E[:r], e, f) if r else np.zeros((m, n), dtype=np.int64)
        assert (LE == AP).all()
        R2, _, _ = oracle.echelon(E, e, f, full=True)
        assert (R2 == R).all()
    else:
        Rv = workload.freivalds_vectors(np.random.default_rng(m + n + e), n, e)
        assert oracle.freivalds(Lh[:, :r], E[:r], AP, e, f, Rv) == 0
    return r


FIELDS = [(2, 0x7), (3, 0xB), (4, 0x13), (8, 0x11D), (10, 0x409), (16, 0x1100B)]


@pytest.mark.parametrize("e,f", FIELDS)
@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (64, 64), (100, 300), (300, 100), (513, 700), (700, 513)])
def test_ple_random(g, ctx, e, f, shape):
    gen = np.random.default_rng(hash((e, shape)) % 2**32)
    A = workload.field_matrix(gen, *shape, e)
    check_gpu_ple(g, ctx, A, e, f)


@pytest.mark.parametrize("e,f", [(2, 0x7), (8, 0x11D), (10, 0x409)])
def test_ple_rank_deficient(g, ctx, e, f):
    gen = np.random.default_rng(300 + e)
    X = workload.field_matrix(gen, 400, 50, e)
    Y = workload.field_matrix(gen, 50, 333, e)
    A = oracle.matmul(X, Y, e, f)
    A[:, 7] = 0
    assert check_gpu_ple(g, ctx, A, e, f) == 50


@pytest.mark.parametrize("e,f", [(4, 0x13), (8, 0x11D)])
def test_ple_pivots_far_down(g, ctx, e, f):
    """The first 300 rows are zero, so every panel's pivots come from the
    tournament over all rows and many rows move."""
    gen = np.random.default_rng(77 + e)
    A = workload.field_matrix(gen, 600, 200, e)
    A[:300] = 0
    A[310] = A[450]                      # a duplicate row
    check_gpu_ple(g, ctx, A, e, f)


def test_ple_large_f256(g, ctx):
    e, f = 8, 0x11D
    A = workload.field_matrix(np.random.default_rng(2048), 2048, 2048, e)
    assert check_gpu_ple(g, ctx, A, e, f, full_product=False) == 2048


def test_ple_errors(g, ctx):
    e, f = 8, 0x11D
    A = dev(g, np.full((8, 6), 3), e)
    with pytest.raises(g.GF2EError) as ei:
        ctx.ple(A, e, f, L=torch.empty((8, 8), dtype=torch.uint8, device="cuda"))
    assert ei.value.code == g.ESHAPE
    with pytest.raises(g.GF2EError) as ei:
        ctx.ple(A, e, 0)
    assert ei.value.code == g.EFIELD
    with pytest.raises(g.GF2EError) as ei:
        ctx.ple(A, e, f, L=A[:, :6])
    assert ei.value.code == g.EALIAS
    bad = dev(g, np.full((4, 4), 2), 2)
    bad[2, 2] = 4
    before = host(bad)
    with pytest.raises(g.GF2EError) as ei:
        ctx.ple(bad, 2, 0x7)
    assert ei.value.code == g.ERANGE
    assert (host(bad) == before).all()
    Z = torch.zeros((3, 0), dtype=torch.uint8, device="cuda")
    L, P, Q, r = ctx.ple(Z, e, f)
    assert r == 0 and P == [0, 1, 2] and Q == []
