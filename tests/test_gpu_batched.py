"""Batched products (one captured graph, persistent grouped kernel) on the GPU.

Every product of a batch must equal the CPU oracle bit for bit and the same
product computed alone by gf2e_mul, whatever the tile class, work order or
replay.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_1111_6900_amd as g
    return g


def to_dev(g, M, e):
    return torch.from_numpy(np.ascontiguousarray(M).astype(np.int64)).to(g.elem_dtype(e)).cuda()


def host(t):
    return t.cpu().numpy().astype(np.int64)


def make_batch(g, specs, tag=3):
    mats = workload.batch_inputs(specs, tag=tag)
    As = [to_dev(g, a, e) for (e, f, m, k, n), (a, b) in zip(specs, mats)]
    Bs = [to_dev(g, b, e) for (e, f, m, k, n), (a, b) in zip(specs, mats)]
    es = [s[0] for s in specs]
    fs = [s[1] for s in specs]
    return mats, As, Bs, es, fs


def test_batch_512_mixed_fields(g):
    """The 512-product workload: e ~ U{2..10}, m, n, k log-uniform in [32, 2048]."""
    specs = workload.batch_specs(512)
    print("building 512-product batch", flush=True)
    mats, As, Bs, es, fs = make_batch(g, specs)
    ctx = g.Context(0)
    outs = ctx.mul_batched(As, Bs, es, fs)
    info = ctx.batch_info()
    assert info["graph_builds"] == 1 and info["items_large"] + info["items_small"] + info["items_fused"] > 0
    assert info["fusion"] == 1 and info["items_fused"] > 0
    print("checking against the oracle and the plain path", flush=True)
    for p, ((e, f, m, k, n), (a, b)) in enumerate(zip(specs, mats)):
        got = host(outs[p])
        assert (got == oracle.matmul(a, b, e, f)).all(), p
        alone = host(ctx.mul(As[p], Bs[p], e, f))
        assert (got == alone).all(), p
    # Replay with new contents in the same buffers: no rebuild, fresh results.
    gen = np.random.default_rng(77)
    for p in range(0, 512, 37):
        e = es[p]
        new = workload.field_matrix(gen, *mats[p][0].shape, e)
        As[p].copy_(to_dev(g, new, e))
        mats[p] = (new, mats[p][1])
    outs2 = ctx.mul_batched(As, Bs, es, fs, outs=outs)
    assert ctx.batch_info()["graph_builds"] == 1
    for p in range(0, 512, 37):
        e, f = es[p], fs[p]
        assert (host(outs2[p]) == oracle.matmul(mats[p][0], mats[p][1], e, f)).all(), p
    ctx.close()


@pytest.mark.parametrize("threshold", [0, 384, 10**9])
def test_tile_classes_and_shuffled_order(g, threshold, monkeypatch):
    specs = workload.batch_specs(48, lo=1, hi=700, tag=5)
    mats, As, Bs, es, fs = make_batch(g, specs, tag=5)
    ctx = g.Context(0)
    ctx.set_batch_threshold(threshold)
    ref = [host(o) for o in ctx.mul_batched(As, Bs, es, fs)]
    for p, ((e, f, m, k, n), (a, b)) in enumerate(zip(specs, mats)):
        assert (ref[p] == oracle.matmul(a, b, e, f)).all(), p
    monkeypatch.setenv("GF2E_BATCH_SHUFFLE", str(1234 + threshold % 97))
    shuf = [host(o) for o in ctx.mul_batched(As, Bs, es, fs)]
    assert ctx.batch_info()["graph_builds"] == 2
    for p in range(len(specs)):
        assert (shuf[p] == ref[p]).all(), p
    ctx.close()


def _other_poly(e, skip):
    """The smallest irreducible f of degree e other than skip (no field
    schedule is compiled for it, so it runs the Karatsuba schedule)."""
    for f in range((1 << e) + 1, 2 << e, 2):
        if f != skip and oracle.is_irreducible(e, f):
            return f
    raise AssertionError(e)


def test_fused_and_plain_recombination_agree(g):
    """Folded field schedules (e = 5..10 with their default f), Karatsuba
    schedules with the merged reduction map (e = 2..4, and e = 5, 8, 10 with
    another f), fields above the fused range (e = 11, 12) and ragged, empty and
    k = 0 products in one batch: with fusion on and off every product equals
    the oracle, and the two runs give the same bytes."""
    gen = np.random.default_rng(2718)
    poly = {**workload.DEFAULT_POLY, **workload.WIDE_POLY}
    fields = [(e, poly[e]) for e in range(2, 13)]
    fields += [(e, _other_poly(e, poly[e])) for e in (5, 8, 10)]
    shapes = [(1, 1, 1), (17, 33, 9), (129, 64, 131), (200, 300, 70), (64, 0, 64), (0, 16, 8), (256, 257, 255),
              (300, 520, 129)]
    specs = []
    for i, (e, f) in enumerate(fields):
        for j in range(3):
            specs.append((e, f) + shapes[(i + 3 * j) % len(shapes)])
    As, Bs, hosts = [], [], []
    for e, f, m, k, n in specs:
        a = workload.field_matrix(gen, m, k, e)
        b = workload.field_matrix(gen, k, n, e)
        hosts.append((a, b))
        As.append(to_dev(g, a, e))
        Bs.append(to_dev(g, b, e))
    es, fs = [s[0] for s in specs], [s[1] for s in specs]
    ctx = g.Context(0)
    ctx.set_batch_threshold(10**9)  # every fp4 product in the 128x128 class
    results = {}
    for fusion in (True, False):
        ctx.set_batch_fusion(fusion)
        outs = [torch.full((m, n), 7, dtype=g.elem_dtype(e), device="cuda") for e, f, m, k, n in specs]
        ctx.mul_batched(As, Bs, es, fs, outs=outs)
        info = ctx.batch_info()
        assert info["fusion"] == int(fusion)
        assert (info["items_fused"] > 0) == fusion
        results[fusion] = [host(o) for o in outs]
        for (e, f, m, k, n), (a, b), got in zip(specs, hosts, results[fusion]):
            assert (got == oracle.matmul(a, b, e, f)).all(), (fusion, e, hex(f), m, k, n)
    for x, y in zip(results[True], results[False]):
        assert (x == y).all()
    with pytest.raises(g.GF2EError) as ei:
        g._check(g.lib().gf2e_set_batch_fusion(ctx.handle, 2))
    assert ei.value.code == g.EINVAL
    ctx.close()


def test_edge_products_in_a_batch(g):
    ctx = g.Context(0)
    gen = np.random.default_rng(5)
    specs = [(2, 0x7, 1, 1, 1), (10, 0x409, 3, 0, 4), (9, 0x211, 0, 5, 6), (8, 0x11D, 7, 9, 0),
             (4, 0x1F, 65, 129, 63), (10, 0x409, 130, 70, 257), (3, 0xB, 256, 256, 256)]
    As, Bs, host_mats = [], [], []
    for e, f, m, k, n in specs:
        a = workload.field_matrix(gen, m, k, e)
        b = workload.field_matrix(gen, k, n, e)
        host_mats.append((a, b))
        As.append(to_dev(g, a, e))
        Bs.append(to_dev(g, b, e))
    outs = [torch.full((m, n), 5, dtype=g.elem_dtype(e), device="cuda") for e, f, m, k, n in specs]
    ctx.mul_batched(As, Bs, [s[0] for s in specs], [s[1] for s in specs], outs=outs)
    for (e, f, m, k, n), (a, b), o in zip(specs, host_mats, outs):
        assert (host(o) == oracle.matmul(a, b, e, f)).all(), (e, m, k, n)
    assert ctx.mul_batched([], [], [], []) == []
    ctx.close()


def test_batch_errors(g):
    ctx = g.Context(0)
    a = to_dev(g, np.ones((4, 4)), 4)
    big = torch.zeros((8, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(g.GF2EError) as ei:   # two outputs overlap
        ctx.mul_batched([a, a], [a, a], [4, 4], [0x13, 0x13], outs=[big[0:4], big[2:6]])
    assert ei.value.code == g.EALIAS
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul_batched([a], [a], [4], [0x11])
    assert ei.value.code == g.EFIELD
    bad = a.clone()
    bad[0, 0] = 16
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul_batched([bad], [a], [4], [0x13])
    assert ei.value.code == g.ERANGE
    ctx.close()


def test_tune_batched_keeps_results(g):
    specs = workload.batch_specs(40, lo=16, hi=1024, tag=6)
    mats, As, Bs, es, fs = make_batch(g, specs, tag=6)
    ctx = g.Context(0)
    outs = [torch.empty((a.size(0), b.size(1)), dtype=a.dtype, device="cuda") for a, b in zip(As, Bs)]
    ctx.tune_batched(As, Bs, es, fs, outs)
    info = ctx.batch_info()
    assert info["threshold"] in (0, 256, 384, 512, 768, 2**63 - 1) and info["fusion"] in (0, 1)
    outs = ctx.mul_batched(As, Bs, es, fs, outs=outs)
    for p, ((e, f, m, k, n), (a, b)) in enumerate(zip(specs, mats)):
        assert (host(outs[p]) == oracle.matmul(a, b, e, f)).all(), p
    ctx.close()


def test_prepared_batch_replays(g):
    """A batch marshalled once replays the cached graph: its results equal the
    oracle's after the inputs change between launches."""
    specs = workload.batch_specs(48, lo=16, hi=300, tag=4)
    mats, As, Bs, es, fs = make_batch(g, specs, tag=9)
    ctx = g.Context(0)
    prep = ctx.prepare_batched(As, Bs, es, fs)
    gen = np.random.default_rng(91)
    for rnd in range(3):
        print(f"prepared batch launch {rnd}", flush=True)
        outs = prep.launch()
        ctx.sync()
        for p, ((e, f, m, k, n), (a, b)) in enumerate(zip(specs, mats)):
            assert (host(outs[p]) == oracle.matmul(a, b, e, f)).all(), (rnd, p)
        for p in range(0, len(specs), 5):
            new = workload.field_matrix(gen, *mats[p][1].shape, es[p])
            Bs[p].copy_(to_dev(g, new, es[p]))
            mats[p] = (mats[p][0], new)
    assert ctx.batch_info()["graph_builds"] == 1
    ctx.close()
