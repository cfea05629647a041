"""GPU parity of C += A*B and of triangular solving (Section 4.3) against the
CPU oracle.  Bit-exact: the solution of T X = B is unique for a nonsingular
triangular T, and every step is exact field arithmetic."""
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


def triangular(gen, m, e, lower):
    T = workload.field_matrix(gen, m, m, e).astype(np.int64)
    T = np.tril(T) if lower else np.triu(T)
    np.fill_diagonal(T, gen.integers(1, 1 << e, m))
    return T


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("e", [2, 5, 8, 10])
@pytest.mark.parametrize("shape", [(1, 1, 1), (63, 65, 64), (257, 300, 255), (40, 0, 30)])
def test_mul_add(g, e, shape, form):
    f = workload.DEFAULT_POLY[e]
    m, k, n = shape
    print(f"mul_add e={e} shape={shape} form={form}", flush=True)
    c = g.Context(0)
    c.set_form(form)
    gen = np.random.default_rng(e * 5 + m + form)
    A = workload.field_matrix(gen, m, k, e)
    B = workload.field_matrix(gen, k, n, e)
    C0 = workload.field_matrix(gen, m, n, e)
    C = dev(C0, e)
    c.mul_add(dev(A, e), dev(B, e), C, e, f)
    want = C0.astype(np.int64) ^ oracle.matmul(A, B, e, f).astype(np.int64)
    assert (host(C) == want).all()
    c.close()


@pytest.mark.parametrize("e,f", ALL_E + [(4, 0x1F), (8, 0x11B)])
@pytest.mark.parametrize("lower", [False, True])
@pytest.mark.parametrize("unit", [False, True])
@pytest.mark.parametrize("m,n", [(1, 3), (129, 70), (300, 130)])
def test_trsm_every_field(ctx, e, f, lower, unit, m, n):
    print(f"trsm e={e} f={f:#x} lower={lower} unit={unit} m={m} n={n}", flush=True)
    gen = np.random.default_rng(e * 97 + m + 3 * lower + unit)
    T = triangular(gen, m, e, lower)
    if unit:
        np.fill_diagonal(T, gen.integers(0, 1 << e, m))  # not read
    B = workload.field_matrix(gen, m, n, e)
    Bd = dev(B, e)
    ctx.trsm(dev(T, e), Bd, e, f, lower=lower, unit=unit)
    assert (host(Bd) == oracle.trsm(T, B, e, f, lower=lower, unit=unit)).all()


@pytest.mark.parametrize("lower", [False, True])
@pytest.mark.parametrize("m", [5, 127, 128, 256, 257, 700, 1000])
def test_trsm_block_boundaries(ctx, lower, m):
    e, f = 8, 0x11D
    n = 97
    print(f"trsm boundaries lower={lower} m={m}", flush=True)
    gen = np.random.default_rng(m + lower)
    T = triangular(gen, m, e, lower)
    B = workload.field_matrix(gen, m, n, e)
    Bd = dev(B, e)
    ctx.trsm(dev(T, e), Bd, e, f, lower=lower)
    assert (host(Bd) == oracle.trsm(T, B, e, f, lower=lower)).all()


def test_trsm_strided_views(ctx):
    e, f = 4, 0x13
    gen = np.random.default_rng(11)
    m, n = 200, 90
    T = triangular(gen, m, e, False)
    B = workload.field_matrix(gen, m, n, e)
    Tbig = torch.zeros((m, m + 37), dtype=torch.uint8, device="cuda")
    Tbig[:, 5:5 + m] = dev(T, e)
    Bbig = torch.zeros((m, n + 50), dtype=torch.uint8, device="cuda")
    Bbig[:, 20:20 + n] = dev(B, e)
    ctx.trsm(Tbig[:, 5:5 + m], Bbig[:, 20:20 + n], e, f)
    assert (host(Bbig[:, 20:20 + n]) == oracle.trsm(T, B, e, f)).all()
    assert (host(Bbig[:, :20]) == 0).all() and (host(Bbig[:, 20 + n:]) == 0).all()


def test_trsm_errors(g, ctx):
    e, f = 4, 0x13
    m, n = 150, 10
    gen = np.random.default_rng(2)
    T = triangular(gen, m, e, False)
    B = workload.field_matrix(gen, m, n, e)
    Ts = T.copy()
    Ts[140, 140] = 0
    with pytest.raises(g.GF2EError) as ex:
        ctx.trsm(dev(Ts, e), dev(B, e), e, f)
    assert ex.value.code == g.ESINGULAR
    # unit: the diagonal is not read, so the zero does not matter
    Bd = dev(B, e)
    ctx.trsm(dev(Ts, e), Bd, e, f, unit=True)
    assert (host(Bd) == oracle.trsm(Ts, B, e, f, unit=True)).all()
    Tr = T.copy()
    Tr[3, 100] = 16
    with pytest.raises(g.GF2EError) as ex:
        ctx.trsm(dev(Tr, e), dev(B, e), e, f)
    assert ex.value.code == g.ERANGE
    # entries below the diagonal of an upper T are not read
    Tl = T.copy()
    Tl[100, 3] = 16
    Bd = dev(B, e)
    ctx.trsm(dev(Tl, e), Bd, e, f)
    assert (host(Bd) == oracle.trsm(T, B, e, f)).all()
    with pytest.raises(g.GF2EError) as ex:
        ctx.trsm(dev(T[:, :-1], e), dev(B, e), e, f)
    assert ex.value.code == g.ESHAPE
    same = dev(T, e)
    with pytest.raises(g.GF2EError) as ex:
        ctx.trsm(same, same, e, f)
    assert ex.value.code == g.EALIAS


@pytest.mark.parametrize("e,f,lower", [(4, 0x13, False), (8, 0x11D, True)])
def test_trsm_4096_sampled_columns(ctx, e, f, lower):
    m = n = 4096
    print(f"trsm {m}x{m} e={e} lower={lower}", flush=True)
    gen = np.random.default_rng(4096 + e)
    T = triangular(gen, m, e, lower)
    B = workload.field_matrix(gen, m, n, e)
    Bd = dev(B, e)
    ctx.trsm(dev(T, e), Bd, e, f, lower=lower)
    X = host(Bd)
    cols = np.sort(gen.choice(n, 12, replace=False))
    assert (X[:, cols] == oracle.trsm(T, B[:, cols], e, f, lower=lower)).all()
