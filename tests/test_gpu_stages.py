"""Each HIP stage against a numpy model of its documented layout (GPU).

Expected values come from tests/planes_model.py (restating the plane layouts
of include/gf2e.h and the Section 5 schedule, whose bilinear identity is
pinned on the CPU by test_abi.py) -- never from the GPU path itself.
"""
import numpy as np
import pytest
import torch

import workload
from tests import planes_model as pm

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (3, 5, 2), (63, 64, 65), (65, 127, 63), (200, 300, 129), (256, 256, 256),
          (300, 129, 520)]


@pytest.fixture(scope="module")
def g():
    import paper_1111_6900_amd as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context(0)


def dev(M, e):
    import paper_1111_6900_amd as g
    t = torch.from_numpy(np.ascontiguousarray(M).astype(np.int64)).to(g.elem_dtype(e))
    return t.cuda()


def rand_words(gen, shape):
    """Uniform 64-bit words, as the int64 array torch can hold."""
    return gen.integers(0, 2**64, size=shape, dtype=np.uint64).view(np.int64)


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("e", [2, 3, 4, 5, 6, 7, 8, 9, 10])
@pytest.mark.parametrize("shape", SHAPES)
def test_slice_a_and_b(g, ctx, e, shape):
    m, k, n = shape
    print(f"slice e={e} shape={shape}", flush=True)
    f = workload.DEFAULT_POLY[e]
    gen = np.random.default_rng(e * 7919 + m)
    A = workload.field_matrix(gen, m, k, e)
    B = workload.field_matrix(gen, k, n, e)
    geo = g.plane_geometry(e, f, m, k, n)
    S = g.schedule(e, f)
    Ap = torch.full((geo.t, geo.K64p, geo.Mp), -1, dtype=torch.int64, device="cuda")
    Bp = torch.full((geo.t, geo.K64p, geo.Np), -1, dtype=torch.int64, device="cuda")
    ctx.slice_a(dev(A, e), e, f, Ap, geo.Mp, geo.K64p)
    ctx.slice_b(dev(B, e), e, f, Bp, geo.Np, geo.K64p)
    ctx.sync()
    assert (host_u64(Ap) == pm.operand_planes_a(A, e, S["u"], geo.Mp, geo.K64p)).all()
    assert (host_u64(Bp) == pm.operand_planes_b(B, e, S["v"], geo.Np, geo.K64p)).all()


def test_slice_figure1(g, ctx, golden_dir):
    """The raw slices of the Figure 1 matrix over F_8 appear as the operand
    planes of the single-slice products."""
    import os
    from tests import fielddef
    meta, _ = fielddef.read_golden(os.path.join(golden_dir, "fig1_f8.txt"))
    e = meta["e"][0]
    A = np.array(meta["packed"], dtype=np.uint8).reshape(2, 2)
    geo = g.plane_geometry(e, 0xB, 2, 2, 2)
    S = g.schedule(e, 0xB)
    Ap = torch.zeros((geo.t, geo.K64p, geo.Mp), dtype=torch.int64, device="cuda")
    ctx.slice_a(dev(A, e), e, 0xB, Ap, geo.Mp, geo.K64p)
    ctx.sync()
    planes = host_u64(Ap)
    for i in range(e):
        s = S["u"].index(1 << i)
        got = [int(planes[s, 0, r] >> np.uint64(c)) & 1 for r in range(2) for c in range(2)]
        assert got == meta[f"slice{i}"], (i, got)


@pytest.mark.parametrize("kind", list(range(9)))
@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 200, 33), (64, 128, 64), (130, 384, 250),
                                   (256, 64, 512), (513, 1000, 300), (40, 700, 90), (70, 1500, 140),
                                   (129, 2304, 200)])
def test_plane_products(g, ctx, kind, shape):
    """k from 1 to 9 stages of 256 bits: the kernels that keep several
    stages in flight (up to three) also run with fewer stages than that and
    with LDS buffers reused."""
    m, k, n = shape
    print(f"products kind={kind} shape={shape}", flush=True)
    t = 5
    geo = g.plane_geometry(2, 0x7, m, k, n)
    gen = np.random.default_rng(kind * 100 + m)
    # Arbitrary words everywhere, padding included: the product runs over all
    # K64p*64 bits, and only rows < m, columns < n are compared.
    Ah = rand_words(gen, (t, geo.K64p, geo.Mp))
    Bh = rand_words(gen, (t, geo.K64p, geo.Np))
    Ap = torch.from_numpy(Ah).cuda()
    Bp = torch.from_numpy(Bh).cuda()
    P = torch.zeros((t, geo.Mp, geo.Np // 64), dtype=torch.int64, device="cuda")
    ctx.plane_products(kind, t, Ap, Bp, P, m, n, geo.Mp, geo.Np, geo.K64p)
    ctx.sync()
    got = host_u64(P)
    want = pm.gf2_products(Ah.view(np.uint64), Bh.view(np.uint64), m, n)
    for s in range(t):
        assert (pm.unpack_rows(np.ascontiguousarray(got[s, :m]), n) == want[s]).all(), s


def test_plane_products_rejects_unaligned_planes(g, ctx):
    """The fp4 kernels load operand rows in 16-byte pairs: plane buffers off
    a 16-byte boundary are refused before anything is launched."""
    geo = g.plane_geometry(2, 0x7, 64, 256, 64)
    t = 3
    A = torch.zeros(t * geo.K64p * geo.Mp + 1, dtype=torch.int64, device="cuda")
    B = torch.zeros(t * geo.K64p * geo.Np + 1, dtype=torch.int64, device="cuda")
    P = torch.zeros(t * geo.Mp * (geo.Np // 64) + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(g.GF2EError) as err:
        ctx.plane_products(-1, t, A[1:], B[:-1], P[:-1], 64, 64, geo.Mp, geo.Np, geo.K64p)
    assert err.value.code == g.EINVAL
    ctx.plane_products(-1, t, A[:-1], B[:-1], P[:-1], 64, 64, geo.Mp, geo.Np, geo.K64p)
    ctx.sync()
    assert int(P.count_nonzero()) == 0


@pytest.mark.parametrize("e,f", [(2, 0x7), (4, 0x13), (4, 0x1F), (5, 0x25), (8, 0x11D),
                                 (8, 0x11B), (9, 0x211), (10, 0x409)])
@pytest.mark.parametrize("mn", [(1, 1), (5, 70), (64, 64), (130, 257)])
def test_combine(g, ctx, e, f, mn):
    m, n = mn
    print(f"combine e={e} f={f:#x} m={m} n={n}", flush=True)
    geo = g.plane_geometry(e, f, m, 1, n)
    S = g.schedule(e, f)
    gen = np.random.default_rng(e * 31 + m)
    Ph = rand_words(gen, (geo.t, geo.Mp, geo.Np // 64))
    P = torch.from_numpy(Ph).cuda()
    C = torch.full((m, n), 77, dtype=g.elem_dtype(e), device="cuda")
    ctx.combine(e, f, P, geo.Mp, geo.Np, C)
    ctx.sync()
    bits = [pm.unpack_rows(np.ascontiguousarray(Ph.view(np.uint64)[s, :m]), n) for s in range(geo.t)]
    want = pm.combine(bits, S["m"], e)
    assert (C.cpu().numpy().astype(np.int64) == want).all()
