"""GPU parity of row echelon forms (Sections 4.1 and 6) against the oracle.

The reduced row echelon form, the rank and the pivot columns are unique, so
they are compared bit for bit.  The plain (non-reduced) form is not unique:
it is checked for its structure, its rank and pivots, and by reducing it
again with the oracle, which must give the oracle's RREF of the input."""
import numpy as np
import pytest
import torch

import oracle
import workload

pytestmark = pytest.mark.gpu

ALL_E = sorted(workload.DEFAULT_POLY.items())


@pytest.fixture(scope="module")
def g():
    import paper_1111_6900_amd as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context(0)


def dev(M, e):
    import paper_1111_6900_amd as g
    return torch.from_numpy(np.ascontiguousarray(M).astype(np.int64)).to(g.elem_dtype(e)).cuda()


def host(t):
    return t.cpu().numpy().astype(np.int64)


def low_rank(gen, m, n, k, e, f):
    """An m x n matrix of rank at most k: a product of m x k and k x n factors."""
    return oracle.matmul(workload.field_matrix(gen, m, k, e), workload.field_matrix(gen, k, n, e), e, f)


def gpu_echelon(ctx, A, e, f, full=True):
    Ad = dev(A, e)
    r, piv = ctx.echelonize(Ad, e, f, full=full)
    return host(Ad), r, piv


@pytest.mark.parametrize("e,f", ALL_E + [(4, 0x1F), (8, 0x11B)])
@pytest.mark.parametrize("shape", [(1, 1), (5, 7), (64, 64), (65, 130), (130, 65), (200, 300)])
def test_rref_every_field(ctx, e, f, shape):
    m, n = shape
    print(f"rref e={e} f={f:#x} shape={shape}", flush=True)
    gen = np.random.default_rng(e * 13 + m + 7 * n)
    A = workload.field_matrix(gen, m, n, e)
    E, r, piv = gpu_echelon(ctx, A, e, f)
    Eo, ro, po = oracle.echelon(A, e, f)
    assert r == ro and piv == list(po)
    assert (E == Eo).all()


@pytest.mark.parametrize("e,f", [(2, 0x7), (8, 0x11D), (10, 0x409)])
@pytest.mark.parametrize("shape,k", [((150, 170), 40), ((170, 150), 100), ((300, 300), 250), ((64, 200), 63)])
def test_rref_rank_deficient(ctx, e, f, shape, k):
    m, n = shape
    print(f"rref low rank e={e} shape={shape} k={k}", flush=True)
    gen = np.random.default_rng(k + e)
    A = low_rank(gen, m, n, k, e, f)
    A[:, 5] = 0  # a zero column
    E, r, piv = gpu_echelon(ctx, A, e, f)
    Eo, ro, po = oracle.echelon(A, e, f)
    assert r == ro <= k and piv == list(po)
    assert (E == Eo).all()


def test_special_matrices(ctx):
    e, f = 4, 0x13
    E, r, piv = gpu_echelon(ctx, np.zeros((70, 90), dtype=np.int64), e, f)
    assert r == 0 and (E == 0).all()
    E, r, piv = gpu_echelon(ctx, np.eye(100, dtype=np.int64) * 3, e, f)
    assert r == 100 and (E == np.eye(100)).all() and piv == list(range(100))
    A = np.zeros((10, 200), dtype=np.int64)
    A[3, 150] = 7
    A[7, 20] = 1
    E, r, piv = gpu_echelon(ctx, A, e, f)
    Eo, ro, po = oracle.echelon(A, e, f)
    assert r == ro == 2 and piv == [20, 150] and (E == Eo).all()


@pytest.mark.parametrize("e,f", [(3, 0xB), (8, 0x11D)])
def test_plain_echelon_form(ctx, e, f):
    gen = np.random.default_rng(e + 100)
    A = low_rank(gen, 180, 220, 90, e, f)
    E, r, piv = gpu_echelon(ctx, A, e, f, full=False)
    Eo, ro, po = oracle.echelon(A, e, f)
    assert r == ro and piv == list(po)
    assert (E[r:] == 0).all()
    for t, j in enumerate(piv):
        assert E[t, j] == 1 and (E[t, :j] == 0).all() and (E[t + 1:, j] == 0).all()
    assert (oracle.echelon(E, e, f)[0] == Eo).all()


def test_errors_leave_a_unchanged(g, ctx):
    e, f = 4, 0x13
    A = np.ones((20, 30), dtype=np.int64)
    A[11, 17] = 16
    Ad = dev(A, e)
    with pytest.raises(g.GF2EError) as ex:
        ctx.echelonize(Ad, e, f)
    assert ex.value.code == g.ERANGE
    assert (host(Ad) == A).all()


@pytest.mark.parametrize("e,f,shape,k", [(8, 0x11D, (1024, 1024), 1024), (2, 0x7, (1024, 1536), 700)])
def test_rref_1024(ctx, e, f, shape, k):
    m, n = shape
    print(f"rref {shape} e={e} k={k}", flush=True)
    gen = np.random.default_rng(1024 + e)
    A = workload.field_matrix(gen, m, n, e) if k >= min(m, n) else low_rank(gen, m, n, k, e, f)
    E, r, piv = gpu_echelon(ctx, A, e, f)
    Eo, ro, po = oracle.echelon(A, e, f)
    assert r == ro and piv == list(po)
    assert (E == Eo).all()


@pytest.mark.parametrize("e,f", [(2, 0x7), (8, 0x11D), (12, 0x1053)])
def test_rref_pivots_beyond_the_first_rows(ctx, e, f):
    """Pivots that only rows far down can supply: the first rows of a panel
    lack a pivot in some column (zero there, or linearly dependent), so the
    pivot search has to look at the remaining rows as well."""
    gen = np.random.default_rng(4000 + e)
    A = workload.field_matrix(gen, 700, 130, e)
    A[:400, 3] = 0
    A[:400, 70] = 0
    B = workload.field_matrix(gen, 600, 64, e)
    B[:300] = B[np.arange(300) % 10]  # rank at most 10 in the first 300 rows
    for M in (A, B):
        print(f"rref beyond first rows e={e} shape={M.shape}", flush=True)
        E, r, piv = gpu_echelon(ctx, M, e, f)
        Eo, ro, po = oracle.echelon(M, e, f)
        assert r == ro and piv == list(po)
        assert (E == Eo).all()


@pytest.mark.parametrize("m,e", [(4096, 2), (8192, 8)])
def test_rref_full_size_properties(g, m, e):
    """The benchmark's echelon inputs at full size (too large for the oracle's
    elimination), checked by properties that hold at any size: R is in
    reduced row echelon form (increasing pivots, unit pivot columns, zeros
    left of each pivot and below the rank), and sampled rows of A lie in the
    row space of R, a_i = sum_t a_i[pivot t] * R_t, with that product taken
    by the oracle."""
    f = workload.DEFAULT_POLY[e]
    print(f"rref full size m={m} e={e}", flush=True)
    A = workload.field_matrix(np.random.default_rng(90000 + m + e), m, m, e)
    c = g.Context(0, autotune=True)
    Ad = dev(A, e)
    r, piv = c.echelonize(Ad, e, f)
    R = Ad.cpu().numpy()  # uint8 elements
    c.close()
    piv = np.asarray(piv, dtype=np.int64)
    assert r >= m - 2 and len(piv) == r and (np.diff(piv) > 0).all()
    assert not R[r:].any()
    assert (R[:r][:, piv] == np.eye(r, dtype=R.dtype)).all()
    left = np.arange(m)[None, :] < piv[:, None]
    assert not (R[:r] * left).any()
    rows = np.random.default_rng(m + e).choice(m, 8, replace=False)
    coeff = A[rows][:, piv]
    assert (oracle.matmul(coeff, R[:r], e, f).astype(np.int64) == A[rows]).all()
