"""gf2e_mul_noalloc_async: the product with its bit-planes in the library's
fixed per-GPU scratch array, for callers that cannot allocate.

Its results must equal gf2e_mul_async's bit for bit (both compute the unique
product over F_{2^e}), also when a smaller product follows a larger one in the
same scratch array, and it must leave the context's own workspace unallocated.
"""
import numpy as np
import pytest
import torch

import workload

pytestmark = pytest.mark.gpu


def _dev(g, M, e):
    return torch.from_numpy(np.ascontiguousarray(M)).to(g.elem_dtype(e)).cuda()


def test_noalloc_equals_mul_async_on_consecutive_calls():
    import paper_1111_6900_amd as g
    ctx = g.Context(0)       # the no-allocation calls run here
    ref = g.Context(0)       # gf2e_mul_async, with its own workspace
    gen = np.random.default_rng(7007)
    cases = [(8, 2048, 2048, 2048),   # the largest e = 8 cube that fits
             (8, 300, 517, 129),      # smaller, ragged: stale planes behind it
             (10, 700, 333, 901),
             (2, 64, 1, 65),
             (4, 1, 4000, 3)]
    for e, m, k, n in cases:
        f = workload.DEFAULT_POLY[e]
        print(f"noalloc e={e} {m}x{k}x{n}", flush=True)
        A = _dev(g, workload.field_matrix(gen, m, k, e), e)
        B = _dev(g, workload.field_matrix(gen, k, n, e), e)
        out = torch.full((m, n), 1, dtype=g.elem_dtype(e), device="cuda")
        ctx.mul_noalloc_async(A, B, e, f, out)
        ctx.sync()
        want = ref.mul(A, B, e, f)
        assert torch.equal(out, want), (e, m, k, n)
    assert ctx.workspace_bytes() == 0
    ctx.close()
    ref.close()


def test_noalloc_limits_and_edges():
    import paper_1111_6900_amd as g
    ctx = g.Context(0)
    e, f = 8, 0x11D
    big = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(big)
    with pytest.raises(g.GF2EError) as ei:     # planes need more than the array
        ctx.mul_noalloc_async(big, big, e, f, out)
    assert ei.value.code == g.ENOMEM
    geo = g.plane_geometry(e, f, 2048, 2048, 2048)
    assert geo.a_bytes + geo.b_bytes + geo.p_bytes <= g.NOALLOC_MAX_BYTES
    A = torch.ones((5, 0), dtype=torch.uint8, device="cuda")
    B = torch.ones((0, 7), dtype=torch.uint8, device="cuda")
    C = torch.full((5, 7), 9, dtype=torch.uint8, device="cuda")
    ctx.mul_noalloc_async(A, B, e, f, C)          # k = 0: the empty sum
    ctx.sync()
    assert (C == 0).all()
    bad = torch.full((4, 4), 7, dtype=torch.uint8, device="cuda")
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul_noalloc_async(bad, bad, 2, 0x7, torch.empty_like(bad))
        ctx.sync()
    assert ei.value.code == g.ERANGE
    assert ctx.workspace_bytes() == 0
    ctx.close()
