"""Serving loop (continuous batching) on the GPU.

Each served result must be byte-identical to the same product computed alone
by gf2e_mul, and equal to the CPU oracle (in full for small products, on
sampled rows and entries for large ones), while requests of different fields
and sizes arrive during each other's execution under a tight memory budget.
"""
import time

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


def check_against_oracle(a, b, e, f, got, gen):
    m, n = got.shape
    if m * a.shape[1] * n <= 3e8:
        assert (got == oracle.matmul(a, b, e, f)).all()
    else:
        rows = gen.choice(m, 3, replace=False)
        for r in rows:
            assert (got[r] == oracle.matmul(a, b, e, f, rows=(r, r + 1))[0]).all()
        I = gen.integers(0, m, 500)
        J = gen.integers(0, n, 500)
        assert (got[I, J] == oracle.entries(a, b, e, f, I, J)).all()


def test_served_equals_alone_under_memory_pressure(g):
    ctx = g.Context(0)
    # 24 MiB of plane memory (the largest request needs 14.4 MiB, all 60
    # together 159 MiB) and 6 slots: requests of different fields and sizes
    # arrive in bursts while others run.
    srv = g.Server(ctx, memory_budget=24 << 20, max_inflight=6, quantum_macs=1 << 36)
    gen = np.random.default_rng(2024)
    sizes = [1, 17, 64, 129, 300, 513, 700, 1024, 1500]
    reqs = []
    for i in range(60):
        e = int(gen.integers(2, 11))
        f = workload.DEFAULT_POLY[e]
        n = sizes[i % len(sizes)]
        k = int(gen.integers(1, 1100)) if i % 5 else n
        a = workload.field_matrix(gen, n, k, e)
        b = workload.field_matrix(gen, k, n, e)
        reqs.append((e, f, a, b, to_dev(g, a, e), to_dev(g, b, e)))
    print("submitting 60 requests in bursts", flush=True)
    tickets = []
    for i, (e, f, a, b, A, B) in enumerate(reqs):
        tickets.append(srv.submit(A, B, e, f))
        if i % 10 == 9:
            time.sleep(0.002)
    results = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["completed"] == 60
    assert 1 < st["peak_inflight"] <= 6
    assert st["peak_arena_bytes"] <= 24 << 20
    assert st["shared_iterations"] >= 1     # requests shared a launch
    print("comparing with the plain path and the oracle", flush=True)
    for (e, f, a, b, A, B), (out, times) in zip(reqs, results):
        assert times["status"] == 0
        assert times["t_submit_ns"] <= times["t_admit_ns"] <= times["t_done_ns"]
        got = host(out)
        alone = host(ctx.mul(A, B, e, f))
        assert (got == alone).all(), (e, a.shape, b.shape)
        check_against_oracle(a, b, e, f, got, gen)
    srv.close()
    ctx.close()


def test_run_trace_poisson(g):
    ctx = g.Context(0)
    srv = g.Server(ctx, memory_budget=512 << 20, max_inflight=16)
    specs = workload.serve_specs(120, lo=16, hi=1024, tag=9)
    gen = workload.rng(9, 2)
    arrivals = workload.poisson_arrivals(len(specs), 2000.0, tag=9)
    As, Bs, Cs, es, fs, hosts = [], [], [], [], [], []
    for e, f, n in specs:
        a = workload.field_matrix(gen, n, n, e)
        b = workload.field_matrix(gen, n, n, e)
        hosts.append((a, b))
        As.append(to_dev(g, a, e))
        Bs.append(to_dev(g, b, e))
        Cs.append(torch.empty((n, n), dtype=g.elem_dtype(e), device="cuda"))
        es.append(e)
        fs.append(f)
    times = srv.run_trace(As, Bs, Cs, es, fs, arrivals)
    for i, t in enumerate(times):
        assert t["status"] == 0
        assert t["t_done_ns"] >= t["t_admit_ns"] >= t["t_submit_ns"] >= arrivals[i] * 1e9 - 1e6
    for i in range(0, len(specs), 7):
        e, f, n = specs[i]
        assert (host(Cs[i]) == oracle.matmul(hosts[i][0], hosts[i][1], e, f)).all(), i
    assert srv.stats()["completed"] == len(specs)
    srv.close()
    ctx.close()


def _serving_inputs(g, specs, tag):
    """Device pools per field and, per request, views of its leading n x n
    windows and a distinct output tensor (as the benchmark lays them out)."""
    pools = workload.serve_pools(specs, tag=tag)
    dpools = {e: (to_dev(g, a, e), to_dev(g, b, e)) for e, (a, b) in pools.items()}
    As, Bs, Cs = [], [], []
    for e, f, n in specs:
        A, B = dpools[e]
        As.append(A[:n, :n])
        Bs.append(B[:n, :n])
        Cs.append(torch.empty((n, n), dtype=g.elem_dtype(e), device="cuda"))
    return pools, As, Bs, Cs


def test_served_workload_alone_mix_and_freivalds(g):
    """500 requests of the served workload (e ~ U{2..10}, n log-uniform in
    [64, 4096]) under a memory budget that binds, with bounded bypass: every
    result equals the product computed alone, byte for byte, and passes
    Freivalds' check over F_{2^e} with ceil(64/e) trials; a seeded sample is
    compared with the oracle's whole product."""
    specs = workload.serve_specs(500, lo=64, hi=4096, tag=14)
    pools, As, Bs, Cs = _serving_inputs(g, specs, tag=14)
    ctx = g.Context(0)
    budget = 256 << 20   # the largest request (n = 4096, e = 10) needs 207 MiB
    srv = g.Server(ctx, memory_budget=budget, max_inflight=48, bypass_limit=8)
    arrivals = workload.poisson_arrivals(len(specs), 4000.0, tag=14)
    print("serving 500 requests", flush=True)
    times = srv.run_trace(As, Bs, Cs, [s[0] for s in specs], [s[1] for s in specs], arrivals)
    st = srv.stats()
    srv.close()
    print(f"server counters {st}", flush=True)
    assert all(t["status"] == 0 for t in times)
    assert st["completed"] == len(specs)
    assert st["peak_inflight"] > 1
    assert st["shared_iterations"] >= 1 and st["max_iteration_requests"] >= 2
    assert st["peak_arena_bytes"] <= budget
    print("alone vs mix", flush=True)
    for i, (e, f, n) in enumerate(specs):
        alone = ctx.mul(As[i], Bs[i], e, f)
        assert torch.equal(alone, Cs[i]), (i, e, n)
    print("Freivalds on every result", flush=True)
    gen = workload.rng(14, 5)
    for i, (e, f, n) in enumerate(specs):
        a, b = pools[e]
        R = workload.freivalds_vectors(gen, n, e)
        assert oracle.freivalds(a[:n, :n], b[:n, :n], Cs[i].cpu().numpy(), e, f, R) == 0, (i, e, n)
    print("oracle on a seeded sample", flush=True)
    small = [i for i, (_, _, n) in enumerate(specs) if n <= 768]
    for i in np.random.default_rng(14).choice(small, 12, replace=False):
        e, f, n = specs[i]
        a, b = pools[e]
        assert (Cs[i].cpu().numpy() == oracle.matmul(a[:n, :n], b[:n, :n], e, f)).all(), i
    ctx.close()


@pytest.mark.parametrize("bypass", [0, 4])
def test_memory_budget_orders_admission(g, bypass):
    """Two large requests whose planes do not fit the budget together, then a
    small one: the second large request is admitted only after the first has
    completed; the small one goes ahead of it when bypass is allowed and
    behind it in strict arrival order."""
    e, f, n = 10, workload.DEFAULT_POLY[10], 4096  # about 0.5 ms of products each
    geo = g.plane_geometry(e, f, n, n, n)
    big_fp = sum((x + 255) // 256 * 256 for x in (geo.a_bytes, geo.b_bytes, geo.p_bytes))
    gen = np.random.default_rng(31)
    big = [(to_dev(g, workload.field_matrix(gen, n, n, e), e), to_dev(g, workload.field_matrix(gen, n, n, e), e))
           for _ in range(2)]
    small = to_dev(g, workload.field_matrix(gen, 64, 64, e), e)
    torch.cuda.synchronize()
    ctx = g.Context(0)
    srv = g.Server(ctx, memory_budget=big_fp + big_fp // 2, max_inflight=8, bypass_limit=bypass)
    t1 = srv.submit(*big[0], e, f)
    t2 = srv.submit(*big[1], e, f)
    t3 = srv.submit(small, small, e, f)
    (c1, r1), (c2, r2), (c3, r3) = srv.wait(t1), srv.wait(t2), srv.wait(t3)
    st = srv.stats()
    assert st["memory_waits"] >= 1
    assert r2["t_admit_ns"] >= r1["t_done_ns"]
    if bypass:
        assert st["bypass_admissions"] >= 1 and r3["t_admit_ns"] < r2["t_admit_ns"]
    else:
        assert st["bypass_admissions"] == 0 and r3["t_admit_ns"] >= r2["t_admit_ns"]
    for (A, B), C in zip(big + [(small, small)], (c1, c2, c3)):
        assert torch.equal(C, ctx.mul(A, B, e, f))
    srv.close()
    ctx.close()


def test_submit_waits_for_the_producer_stream(g):
    """Inputs written on a side stream and submitted with that stream and no
    host synchronisation: the server reads them only after the writes."""
    e, f, n = 8, 0x11D, 512
    gen = np.random.default_rng(77)
    a = workload.field_matrix(gen, n, n, e)
    b = workload.field_matrix(gen, n, n, e)
    src_a, src_b = to_dev(g, a, e), to_dev(g, b, e)
    A = torch.zeros_like(src_a)
    B = torch.zeros_like(src_b)
    torch.cuda.synchronize()
    ctx = g.Context(0)
    srv = g.Server(ctx, memory_budget=256 << 20, max_inflight=4)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        torch.cuda._sleep(20_000_000)  # holds the side stream for several ms
        A.copy_(src_a)
        B.copy_(src_b)
        t = srv.submit(A, B, e, f, stream=side)
    out, tm = srv.wait(t)
    assert tm["status"] == 0
    assert (host(out) == oracle.matmul(a, b, e, f)).all()
    srv.close()
    ctx.close()


def test_server_errors(g):
    ctx = g.Context(0)
    srv = g.Server(ctx, memory_budget=1 << 20, max_inflight=2)
    big = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")
    with pytest.raises(g.GF2EError) as ei:   # can never fit 1 MiB
        srv.submit(big, big, 8, 0x11D)
    assert ei.value.code == g.EBUSY
    a = to_dev(g, np.full((8, 8), 3), 2)
    bad = a.clone()
    bad[1, 1] = 4
    t_bad = srv.submit(bad, a, 2, 0x7)
    t_ok = srv.submit(a, a, 2, 0x7)
    with pytest.raises(g.GF2EError) as ei:
        srv.wait(t_bad)
    assert ei.value.code == g.ERANGE
    out, tm = srv.wait(t_ok)
    assert tm["status"] == 0
    assert (host(out) == oracle.matmul(np.full((8, 8), 3), np.full((8, 8), 3), 2, 0x7)).all()
    with pytest.raises(g.GF2EError):
        srv.submit(a, a, 2, 0x5)            # reducible f
    srv.close()
    ctx.close()
