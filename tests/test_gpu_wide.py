"""Fields past the paper's range, 11 <= e <= 16 (its Section 1 footnote),
on the GPU against the oracle: products (both forms, every kernel), C += A*B,
triangular solves, echelon forms and a batch that mixes them with small
fields.  Bit-exact, as everywhere else."""
import numpy as np
import pytest
import torch

import oracle
import workload

pytestmark = pytest.mark.gpu

WIDE = sorted(workload.WIDE_POLY.items())


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


@pytest.mark.parametrize("e,f", WIDE)
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("shape", [(1, 1, 1), (63, 65, 64), (129, 127, 130), (257, 300, 255)])
def test_products(g, e, f, form, shape):
    m, k, n = shape
    print(f"wide mul e={e} form={form} shape={shape}", flush=True)
    c = g.Context(0)
    c.set_form(form)
    gen = np.random.default_rng(e * 41 + m + form)
    A = workload.field_matrix(gen, m, k, e)
    B = workload.field_matrix(gen, k, n, e)
    assert (host(c.mul(dev(A, e), dev(B, e), e, f)) == oracle.matmul(A, B, e, f)).all()
    C0 = workload.field_matrix(gen, m, n, e)
    Cd = dev(C0, e)
    c.mul_add(dev(A, e), dev(B, e), Cd, e, f)
    assert (host(Cd) == (C0.astype(np.int64) ^ oracle.matmul(A, B, e, f).astype(np.int64))).all()
    c.close()


@pytest.mark.parametrize("kind", list(range(9)))
@pytest.mark.parametrize("e", [11, 16])
def test_every_kernel(g, e, kind):
    f = workload.WIDE_POLY[e]
    c = g.Context(0, kernel=kind)
    gen = np.random.default_rng(kind + e)
    A = workload.field_matrix(gen, 300, 517, e)
    B = workload.field_matrix(gen, 517, 270, e)
    assert (host(c.mul(dev(A, e), dev(B, e), e, f)) == oracle.matmul(A, B, e, f)).all()
    c.close()


def test_range_check(g, ctx):
    e, f = 12, workload.WIDE_POLY[12]
    A = np.ones((5, 5), dtype=np.int64)
    A[2, 3] = 1 << 12
    with pytest.raises(g.GF2EError) as ex:
        ctx.mul(dev(A, e), dev(np.ones((5, 5)), e), e, f)
    assert ex.value.code == g.ERANGE


@pytest.mark.parametrize("e,f", [(11, 0x805), (16, 0x1100B)])
@pytest.mark.parametrize("lower", [False, True])
def test_trsm(ctx, e, f, lower):
    gen = np.random.default_rng(e + 3 * lower)
    m, n = 300, 70
    T = workload.field_matrix(gen, m, m, e).astype(np.int64)
    T = np.tril(T) if lower else np.triu(T)
    np.fill_diagonal(T, gen.integers(1, 1 << e, m))
    B = workload.field_matrix(gen, m, n, e)
    Bd = dev(B, e)
    ctx.trsm(dev(T, e), Bd, e, f, lower=lower)
    assert (host(Bd) == oracle.trsm(T, B, e, f, lower=lower)).all()


@pytest.mark.parametrize("e,f", [(12, 0x1053), (16, 0x1100B)])
def test_echelon(ctx, e, f):
    gen = np.random.default_rng(e)
    k = 90
    A = oracle.matmul(workload.field_matrix(gen, 200, k, e), workload.field_matrix(gen, k, 230, e), e, f)
    Ad = dev(A, e)
    r, piv = ctx.echelonize(Ad, e, f)
    Eo, ro, po = oracle.echelon(A, e, f)
    assert r == ro and piv == list(po) and (host(Ad) == Eo).all()


def test_batch_mixing_small_and_wide_fields(g, ctx):
    gen = np.random.default_rng(77)
    specs = [(3, 0xB, 40, 70, 50), (16, 0x1100B, 130, 90, 70), (8, 0x11D, 300, 260, 100),
             (13, 0x201B, 64, 64, 64), (10, 0x409, 33, 500, 20), (11, 0x805, 257, 31, 129)]
    As, Bs, es, fs, want = [], [], [], [], []
    for e, f, m, k, n in specs:
        A = workload.field_matrix(gen, m, k, e)
        B = workload.field_matrix(gen, k, n, e)
        As.append(dev(A, e)); Bs.append(dev(B, e)); es.append(e); fs.append(f)
        want.append(oracle.matmul(A, B, e, f))
    outs = ctx.mul_batched(As, Bs, es, fs)
    for C, w in zip(outs, want):
        assert (host(C) == w).all()
