"""Benchmark: dense C = A*B over F_256 (f = 0x11D), 8192 x 8192 x 8192, on one MI355X.

One step is the whole product pipeline on device-resident uint8 inputs: slice
A and B into the operand planes of the field's product schedule, the 24
GF(2) plane products (fp4 MFMA on 0/1 operands, exact counts), and the fused
recombination / reduction mod f / clinging into C.  The line printed also
carries the roofline of the dominant kernel (the plane products), the CPU
oracle timed on the same product (its rows compared with the timed C), the
batched-vs-plain speedup on 512 mixed products and the served p50/p99
latency with every served result verified (see --no-batched, --no-serve).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0     # MI355X HBM3E, 8 TB/s

# Roofline of each product kernel: (bound, peak, unit, ops counted per GF(2)
# multiply-add).  MFMA peaks are MI355X's published dense figures for the
# kernel's operand type; the VALU kernel's peak is derived from the unit
# counts: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 3-input bitwise op
# (acc ^= a & b) per 32 bit-products -> 1258.3 T bit-products/s.
KERNEL_ROOFLINE = {
    "mfma_i8": ("mfma", 5000.0, "TOP/s", 2.0),       # int8 dense, 5.0 POP/s
    "mfma_fp4": ("mfma", 10100.0, "TFLOP/s", 2.0),   # fp4 dense, 10.1 PFLOP/s
    "valu_xor": ("alu", 1258.3, "Tbit-MAC/s", 1.0),
}


def kernel_roofline(name):
    for prefix, spec in KERNEL_ROOFLINE.items():
        if name.startswith(prefix):
            return spec
    raise KeyError(name)


def measured_counters(workload_name, kernel_name, planes):
    """The committed rocprofv3 figures for this product kernel (HBM bytes per
    launch, MFMA busy fraction, traced mean over the timed steps), or None if
    there are none, the kernel source changed since, or the launch then
    covered a different number of plane products."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        entry = json.load(open(path))[workload_name][kernel_name]
        src = open(os.path.join(ROOT, entry["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != entry["source_sha256"] or entry.get("planes") != planes:
        return None
    return entry


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="f256_8192")
    ap.add_argument("--kernel", type=int, default=-1, help="force a product kernel (-1 = autotuned)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU oracle budget (the whole 8192^3 product takes about 12 s on 16 threads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-trsm", action="store_true")
    ap.add_argument("--no-echelon", action="store_true")
    ap.add_argument("--no-wide", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-budget-mib", type=int, default=256,
                    help="device memory for resident planes of admitted requests")
    ap.add_argument("--serve-inflight", type=int, default=256)
    ap.add_argument("--serve-bypass", type=int, default=16,
                    help="admissions allowed past an oldest request waiting for memory")
    ap.add_argument("--no-serve-verify", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for rocprofv3: a calibration copy of --copy-mib MiB, then "
                         "the timed steps only (no CPU, batched or serving legs)")
    ap.add_argument("--copy-mib", type=int, default=256)
    return ap.parse_args()


def log(args, *msg):
    if not args.quiet:
        print("[bench]", *msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, B, C_gpu, e, f, budget_s, workload_mod=None, echelon=False, no_trsm=False):
    """The oracle on whole rows of the same product until the budget is used
    (all of them when it allows), each row compared with the timed GPU C."""
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    m = A.shape[0]
    k, n = B.shape
    rows, spent, chunk, mismatched = 0, 0.0, 16, 0
    while spent < budget_s and rows < m:
        chunk = min(chunk, m - rows)
        t0 = time.perf_counter()
        part = oracle.matmul(A[rows:rows + chunk], B, e, f, nthreads=threads)
        dt = time.perf_counter() - t0
        mismatched += int(np.count_nonzero(np.any(part != C_gpu[rows:rows + chunk], axis=1)))
        spent += dt
        rows += chunk
        if dt < budget_s / 8:
            chunk *= 2
    macs = rows * k * n
    out = {"value": macs / spent, "unit": "element-MAC/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{rows} of {m} rows of C ({rows}x{k}x{n} element-MAC), "
                     f"{spent:.1f} s on {threads} threads",
           "rows_compared_with_gpu": rows, "rows_mismatched": mismatched}
    if workload_mod is not None and not no_trsm:
        # The oracle's triangular solve (Section 4.3 row algorithm) on a
        # column sample of the TRSM leg's smallest system.
        m, cols = TRSM_SIZES[0], min(64 * threads, TRSM_SIZES[0])  # 64-column chunks per thread
        U, Bt = trsm_system(workload_mod, m, TRSM_E)
        t0 = time.perf_counter()
        oracle.trsm(U, Bt[:, :cols], TRSM_E, TRSM_F, nthreads=threads)
        dt = time.perf_counter() - t0
        out["trsm"] = {"value": m * m * cols / 2 / dt, "unit": "element-MAC/s",
                       "sample": f"{cols} of {m} columns of the {m}x{m} solve, {dt:.2f} s on {threads} threads"}
    # One thread on the two smaller plain workloads (the whole 256^3 product
    # over F_4, a 64-row sample of the 4096^3 product over F_16).
    one = {}
    for name, rows in (("f4_256", None), ("f16_4096", 64)):
        e1, f1, A1, B1 = workload_mod.plain_inputs(name) if workload_mod is not None else (None,) * 4
        if e1 is None:
            break
        r = A1.shape[0] if rows is None else rows
        t0 = time.perf_counter()
        oracle.matmul(A1[:r], B1, e1, f1, nthreads=1)
        dt = time.perf_counter() - t0
        one[name] = {"value": r * A1.shape[1] * B1.shape[1] / dt, "unit": "element-MAC/s",
                     "sample": f"{r} of {A1.shape[0]} rows, {dt:.2f} s on 1 thread"}
    if one:
        out["one_thread"] = one
    if echelon:
        # The oracle's elimination loop (single-threaded) on a 2048^2 matrix
        # over F_256 drawn like the echelon leg's.
        import numpy as np
        m, e8, f8 = 2048, 8, 0x11D
        A8 = workload_mod.field_matrix(np.random.default_rng(90000 + m + e8), m, m, e8)
        t0 = time.perf_counter()
        _, r8, _ = oracle.echelon(A8, e8, f8)
        dt = time.perf_counter() - t0
        out["echelon"] = {"value": m * m * r8 / dt, "unit": "element-MAC/s",
                          "sample": f"RREF of a {m}x{m} matrix over F_256 (rank {r8}), {dt:.2f} s on 1 thread"}
    return out


def batched_leg(g, torch, workload, log, reps=5):
    """512 mixed products: one graph replay vs 512 plain calls on one stream."""
    specs = workload.batch_specs(512)
    mats = workload.batch_inputs(specs)
    As = [torch.from_numpy(a).to(g.elem_dtype(e)).cuda() for (e, *_), (a, b) in zip(specs, mats)]
    Bs = [torch.from_numpy(b).to(g.elem_dtype(e)).cuda() for (e, *_), (a, b) in zip(specs, mats)]
    outs = [torch.empty((a.size(0), b.size(1)), dtype=a.dtype, device="cuda") for a, b in zip(As, Bs)]
    es = [s[0] for s in specs]
    fs = [s[1] for s in specs]
    ctx = g.Context(0)

    def plain():
        for a, b, o, e, f in zip(As, Bs, outs, es, fs):
            ctx.mul_async(a, b, e, f, out=o)

    prepared = None

    def batched():
        prepared.launch()

    def timed(fn):
        fn()
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    log("batched leg: tuning the tile-class threshold")
    ctx.tune_batched(As, Bs, es, fs, outs)
    # The descriptors are marshalled once: a replay is one library call.
    prepared = ctx.prepare_batched(As, Bs, es, fs, outs)
    plain_ms = timed(plain)
    batched_ms = timed(batched)
    ctx.sync()
    info = ctx.batch_info()
    emacs = sum(m * k * n for (_, _, m, k, n) in specs)
    bmacs = sum(g.num_products(e, f) * m * k * n for (e, f, m, k, n) in specs)
    ctx.close()
    return {"products": len(specs), "element_macs": emacs, "bit_macs": bmacs,
            "plain_ms": round(plain_ms, 4), "batched_ms": round(batched_ms, 4),
            "speedup": round(plain_ms / batched_ms, 3),
            "batched_element_mac_per_s": emacs / (batched_ms / 1e3),
            "plain_element_mac_per_s": emacs / (plain_ms / 1e3),
            "work_items": info["items_large"] + info["items_small"] + info["items_fused"],
            "fused_items": info["items_fused"],
            "fused_recombination": bool(info["fusion"]),
            "tile_threshold": info["threshold"],
            "plane_arena_bytes": info["arena_bytes"]}


def forms_leg(g, torch, workload, log, reps=10):
    """Both forms of the plain product (schedule products vs one alpha-power
    product) on the three plain workloads, each with its tuned kernel."""
    res = {}
    for name, (e, f, m, k, n) in workload.PLAIN_CONFIGS.items():
        _, _, A, B = workload.plain_inputs(name)
        Ad = torch.from_numpy(A).to(g.elem_dtype(e)).cuda()
        Bd = torch.from_numpy(B).to(g.elem_dtype(e)).cuda()
        C = torch.empty((m, n), dtype=g.elem_dtype(e), device="cuda")
        ctx = g.Context(0, autotune=True)
        ctx.tune(e, f, m, k, n)
        row = {"e": e, "m": m, "k": k, "n": n,
               "chosen": ["schedule", "alpha"][ctx.chosen_form(e, f, m, k, n)]}
        for form, label in [(g.FORM_SCHEDULE, "schedule"), (g.FORM_ALPHA, "alpha")]:
            ctx.set_form(form)
            for _ in range(2):
                ctx.mul_async(Ad, Bd, e, f, out=C)
            ctx.sync()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                ctx.mul_async(Ad, Bd, e, f, out=C)
            e1.record()
            ctx.sync()
            row[f"{label}_ms"] = round(e0.elapsed_time(e1) / reps, 4)
            row[f"{label}_kernel"] = g.kernel_names()[ctx.chosen_kernel(e, f, m, k, n)]
        log(f"forms {name}: {row}")
        res[name] = row
        ctx.close()
        del Ad, Bd, C
    return res


WIDE_CASES = ((12, 4096), (16, 4096))


def wide_leg(g, torch, workload, log, reps=10):
    """Products over fields past the paper's range (e = 12 and 16, 4096^3),
    autotuned: ms per product and element-MAC/s."""
    import numpy as np
    res = {}
    ctx = g.Context(0, autotune=True)
    for e, m in WIDE_CASES:
        f = workload.WIDE_POLY[e]
        gen = np.random.default_rng(50000 + e)
        Ad = torch.from_numpy(workload.field_matrix(gen, m, m, e).astype(np.int64)).to(g.elem_dtype(e)).cuda()
        Bd = torch.from_numpy(workload.field_matrix(gen, m, m, e).astype(np.int64)).to(g.elem_dtype(e)).cuda()
        C = torch.empty((m, m), dtype=g.elem_dtype(e), device="cuda")
        for _ in range(2):
            ctx.mul_async(Ad, Bd, e, f, out=C)
        ctx.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.mul_async(Ad, Bd, e, f, out=C)
        e1.record()
        ctx.sync()
        ms = e0.elapsed_time(e1) / reps
        row = {"e": e, "m": m, "k": m, "n": m, "products": g.num_products(e, f), "ms": round(ms, 3),
               "element_mac_per_s": m ** 3 / (ms / 1e3),
               "kernel": g.kernel_names()[ctx.chosen_kernel(e, f, m, m, m)]}
        log(f"wide {row}")
        res[f"e{e}_{m}"] = row
        del Ad, Bd, C
    ctx.close()
    return res


def trsm_system(workload, m, e):
    """The seeded upper triangular system of the TRSM leg: U (m x m, nonzero
    diagonal) and B (m x m) over F_2^e."""
    import numpy as np
    gen = np.random.default_rng(70000 + m)
    U = np.triu(workload.field_matrix(gen, m, m, e))
    np.fill_diagonal(U, gen.integers(1, 1 << e, m))
    B = workload.field_matrix(gen, m, m, e)
    return U, B


TRSM_SIZES, TRSM_E, TRSM_F = (4096, 8192), 8, 0x11D


def trsm_leg(g, torch, workload, log, reps=5):
    """Triangular solves X = U^{-1} B (U upper, m x m; B m x m) over F_256:
    time per solve and element-MAC/s counting m*m*n/2 multiply-adds."""
    import numpy as np
    res = {}
    e, f = TRSM_E, TRSM_F
    ctx = g.Context(0, autotune=True)
    for m in TRSM_SIZES:
        U, B = trsm_system(workload, m, e)
        Ud = torch.from_numpy(U).to(g.elem_dtype(e)).cuda()
        B0 = torch.from_numpy(B).to(g.elem_dtype(e)).cuda()
        X = B0.clone()
        ctx.trsm(Ud, X, e, f)  # tunes the product sizes it meets
        times = []
        for _ in range(reps):
            X.copy_(B0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.trsm_async(Ud, X, e, f)
            e1.record()
            ctx.sync()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        row = {"m": m, "n": m, "e": e, "ms": round(ms, 3), "element_mac_per_s": m * m * m / 2 / (ms / 1e3)}
        log(f"trsm {row}")
        res[f"{m}"] = row
        del Ud, B0, X
    ctx.close()
    return res


ECHELON_CASES = ((4096, 2, 0x7), (4096, 8, 0x11D), (8192, 2, 0x7), (8192, 8, 0x11D))


def echelon_leg(g, torch, workload, log, reps=3):
    """Reduced row echelon forms of random square matrices (full rank with
    high probability): ms per form and element-MAC/s counting m*n*rank
    multiply-adds (the cost of the elimination loop of Section 4.1)."""
    import numpy as np
    res = {}
    ctx = g.Context(0, autotune=True)
    for m, e, f in ECHELON_CASES:
        A = workload.field_matrix(np.random.default_rng(90000 + m + e), m, m, e)
        A0 = torch.from_numpy(A).to(g.elem_dtype(e)).cuda()
        Ad = A0.clone()
        r, _ = ctx.echelonize(Ad, e, f)  # tunes the product sizes it meets
        times = []
        for _ in range(reps):
            Ad.copy_(A0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r, _ = ctx.echelonize(Ad, e, f)
            times.append((time.perf_counter() - t0) * 1e3)
        ms = float(np.median(times))
        row = {"m": m, "n": m, "e": e, "rank": r, "ms": round(ms, 2),
               "element_mac_per_s": m * m * r / (ms / 1e3)}
        # The PLE decomposition (Section 4.2) of the same matrix.
        L = torch.empty((m, m), dtype=A0.dtype, device="cuda")
        ptimes = []
        for _ in range(reps):
            Ad.copy_(A0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.ple(Ad, e, f, L=L)
            ptimes.append((time.perf_counter() - t0) * 1e3)
        row["ple_ms"] = round(float(np.median(ptimes)), 2)
        log(f"echelon {row}")
        res[f"{m}_e{e}"] = row
        del A0, Ad, L
    ctx.close()
    return res


def serve_leg(g, torch, workload, log, count=10000, budget=256 << 20, max_inflight=256, bypass=16,
              load=0.7, verify=True):
    """Served requests: n log-uniform in [64, 4096], e ~ U{2..10}.  A closed-loop
    run (all requests at t=0) gives the saturated rate; an open-loop Poisson
    run at `load` times that rate gives the latencies.  Afterwards every
    served result is compared, byte for byte, with the same product computed
    alone by gf2e_mul.  Returns the result block and what the oracle's check
    of every result needs (see serving_freivalds)."""
    import numpy as np
    specs = workload.serve_specs(count)
    # Inputs: one pool per field, each request reads its leading n x n window.
    pools = workload.serve_pools(specs)
    dpools = {e: (torch.from_numpy(a).to(g.elem_dtype(e)).cuda(),
                  torch.from_numpy(b).to(g.elem_dtype(e)).cuda()) for e, (a, b) in pools.items()}
    # Outputs: a distinct region per request.
    tot = {1: 0, 2: 0}
    for e, _, n in specs:
        tot[1 if e <= 8 else 2] += n * n
    out8 = torch.empty(max(tot[1], 1), dtype=torch.uint8, device="cuda")
    out16 = torch.empty(max(tot[2], 1), dtype=torch.int16, device="cuda")
    As, Bs, Cs, es, fs = [], [], [], [], []
    off = {1: 0, 2: 0}
    for e, f, n in specs:
        A, B = dpools[e]
        As.append(A[:n, :n])
        Bs.append(B[:n, :n])
        w = 1 if e <= 8 else 2
        buf = out8 if w == 1 else out16
        Cs.append(buf[off[w]:off[w] + n * n].view(n, n))
        off[w] += n * n
        es.append(e)
        fs.append(f)
    emacs = sum(n ** 3 for _, _, n in specs)
    ctx = g.Context(0)
    srv = g.Server(ctx, memory_budget=budget, max_inflight=max_inflight, bypass_limit=bypass)
    # warm-up on a prefix (first use of every kernel)
    srv.run_trace(As[:64], Bs[:64], Cs[:64], es[:64], fs[:64], [0.0] * 64)
    st0 = srv.stats()
    log(f"serving: closed-loop run of {count} requests")
    t0 = time.perf_counter()
    closed = srv.run_trace(As, Bs, Cs, es, fs, [0.0] * count)
    closed_s = time.perf_counter() - t0
    st1 = srv.stats()
    sat_rate = count / closed_s
    rate = load * sat_rate
    arrivals = workload.poisson_arrivals(count, rate)
    log(f"serving: open-loop Poisson run at {rate:.0f} req/s")
    for c in Cs:  # the open-loop run must write every result afresh
        c.fill_(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    opened = srv.run_trace(As, Bs, Cs, es, fs, arrivals)
    open_s = time.perf_counter() - t0
    lat = np.array([t["t_done_ns"] for t in opened]) / 1e9 - np.asarray(arrivals)
    st = srv.stats()
    srv.close()

    def delta(key, a, b):
        return b[key] - a[key]

    res = {"requests": count, "memory_budget_bytes": budget, "max_inflight": max_inflight,
           "bypass_limit": bypass, "element_macs": emacs,
           "saturated_req_per_s": round(sat_rate, 1),
           "saturated_element_mac_per_s": emacs / closed_s,
           "offered_req_per_s": round(rate, 1), "load": load,
           "throughput_req_per_s": round(count / open_s, 1),
           "throughput_element_mac_per_s": emacs / open_s,
           "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
           "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
           "max_ms": round(float(lat.max()) * 1e3, 3),
           "open_loop": {"memory_waits": delta("memory_waits", st1, st),
                         "bypass_admissions": delta("bypass_admissions", st1, st),
                         "iterations": delta("iterations", st1, st),
                         "shared_iterations": delta("shared_iterations", st1, st)},
           "closed_loop": {"memory_waits": delta("memory_waits", st0, st1),
                           "bypass_admissions": delta("bypass_admissions", st0, st1),
                           "iterations": delta("iterations", st0, st1),
                           "shared_iterations": delta("shared_iterations", st0, st1)},
           "peak_inflight": st["peak_inflight"], "max_iteration_requests": st["max_iteration_requests"],
           "peak_arena_bytes": st["peak_arena_bytes"],
           "status_errors": sum(1 for t in opened if t["status"] != 0)}
    if verify:
        # Every open-loop result against the same product computed alone
        # (one stream, a flag per request, one synchronisation at the end).
        log("serving: comparing every served result with the product computed alone")
        scratch = {1: torch.empty(4096 * 4096, dtype=torch.uint8, device="cuda"),
                   2: torch.empty(4096 * 4096, dtype=torch.int16, device="cuda")}
        diff = torch.zeros(count, dtype=torch.int32, device="cuda")
        for i, (e, f, n) in enumerate(specs):
            alone = scratch[1 if e <= 8 else 2][:n * n].view(n, n)
            ctx.mul_async(As[i], Bs[i], e, f, out=alone)
            diff[i] = (alone != Cs[i]).any().to(torch.int32)
        ctx.sync()
        res["alone_vs_mix_mismatches"] = int(diff.sum().item())
    ctx.close()
    state = {"specs": specs, "pools": pools, "Cs": Cs} if verify else None
    return res, state


def serving_freivalds(state, log):
    """The oracle's Freivalds check over F_{2^e} on every served result, with
    ceil(64/e) random vectors each (a wrong result passes with probability at
    at most 2^-64), plus the oracle's whole product on a seeded sample of
    requests.  Returns (failures, sample mismatches, seconds)."""
    import numpy as np
    import oracle
    import workload
    t0 = time.perf_counter()
    gen = workload.rng(4, 5)
    bad = 0
    for i, (e, f, n) in enumerate(state["specs"]):
        a, b = state["pools"][e]
        R = workload.freivalds_vectors(gen, n, e)
        bad += int(oracle.freivalds(a[:n, :n], b[:n, :n], state["Cs"][i].cpu().numpy(), e, f, R) != 0)
        if i % 2000 == 1999:
            log(f"serving: Freivalds checked {i + 1} results")
    small = [i for i, (_, _, n) in enumerate(state["specs"]) if n <= 512]
    sample = np.random.default_rng(4).choice(small, min(32, len(small)), replace=False)
    sample_bad = 0
    for i in sample:
        e, f, n = state["specs"][i]
        a, b = state["pools"][e]
        sample_bad += int(not np.array_equal(state["Cs"][i].cpu().numpy(),
                                             oracle.matmul(a[:n, :n], b[:n, :n], e, f)))
    return bad, len(sample), sample_bad, time.perf_counter() - t0


def main():
    args = parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; multi-GPU runs are not "
                                   "supported by this benchmark",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import workload
    import paper_1111_6900_amd as g

    e, f, m, k, n = workload.PLAIN_CONFIGS[args.workload]
    log(args, f"workload {args.workload}: e={e} f={f:#x} {m}x{k}x{n}")
    _, _, A, B = workload.plain_inputs(args.workload)
    Ad = torch.from_numpy(A).to(g.elem_dtype(e)).cuda()
    Bd = torch.from_numpy(B).to(g.elem_dtype(e)).cuda()
    C = torch.empty((m, n), dtype=g.elem_dtype(e), device="cuda")

    if args.profile_run:
        args.no_cpu = args.no_batched = args.no_serve = args.no_forms = args.no_trsm = args.no_echelon = True
        args.no_wide = True
        # A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
        # counters calibrate the byte counts read for the product kernels.
        src = torch.ones(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = g.Context(0, kernel=args.kernel, autotune=args.kernel < 0)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.mul_async(Ad, Bd, e, f, out=C)
    ctx.sync()
    kind = ctx.chosen_kernel(e, f, m, k, n)
    form = ctx.chosen_form(e, f, m, k, n)
    log(args, f"form {form}, product kernel: {g.kernel_names()[kind]}")

    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.mul_async(Ad, Bd, e, f, out=C)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.sync()
    stages = {}
    for st, name in [(g.STAGE_SLICE_A, "slice_a"), (g.STAGE_SLICE_B, "slice_b"),
                     (g.STAGE_PRODUCTS, "products"), (g.STAGE_COMBINE, "combine")]:
        ms, cnt = ctx.profile_read(st)
        stages[name] = ms / max(cnt, 1)
    ctx.profile(False)
    ms_per_step = elapsed * 1e3 / args.steps
    value = m * k * n / (ms_per_step / 1e3)
    C_timed = None if args.no_cpu else C.cpu().numpy()  # the timed steps' result

    # GF(2) products of m x k x n per element product: t(e) for the schedule
    # form, e^2 (as one product of m x ek x en) for the alpha form.
    T = g.num_products(e, f) if form == g.FORM_SCHEDULE else e * e
    prod_ms = stages["products"]
    kname = g.kernel_names()[kind]
    bound, peak, unit, ops_per_mac = kernel_roofline(kname)
    ops = ops_per_mac * T * m * n * k  # algorithmic: T GF(2) products of m x k x n
    # Operand planes read once and product planes written once.
    kwa, nwa = -(-k // 64), -(-n // 64)
    if form == g.FORM_SCHEDULE:
        plane_bytes = 8 * T * (kwa * (m + n) + m * nwa)
    else:
        plane_bytes = 8 * (e * kwa * m + e * e * kwa * n + e * m * nwa)
    achieved = ops / (prod_ms / 1e3) / 1e12
    prof = measured_counters(args.workload, kname, T if form == g.FORM_SCHEDULE else 1)
    roofline = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4),
                "traffic": prof["traffic_bytes"] if prof else None,
                "kernel": kname, "form": ["schedule", "alpha"][form], "avg_launch_ms": round(prod_ms, 4),
                "timer": "HIP events around every product launch on its own stream, mean over the "
                         f"{args.steps} timed steps",
                "algorithmic_ops_per_launch": ops,
                "algorithmic_bytes_per_launch": plane_bytes}
    if prof and "mfma_busy" in prof:
        # From the committed profile of the same kernel source: rocprofv3's
        # mean over the timed steps, and the matrix cores' busy share.
        roofline["profile"] = {k: prof[k] for k in ("trace_timed_mean_ms", "mfma_busy", "clock_ghz", "summary")
                               if k in prof}
    # HBM-bound stages: algorithmic bytes (elements in/out + planes written/read).
    esz = 1 if e <= 8 else 2
    kw = -(-k // 64)
    stage_bytes = {
        "slice_a": m * k * esz + T * kw * m * 8,
        "slice_b": k * n * esz + T * kw * n * 8,
        "combine": T * m * (-(-n // 64)) * 8 + m * n * esz,
    }
    hbm = {s: round(b / (stages[s] / 1e3) / 1e9, 1) for s, b in stage_bytes.items()}

    out = {
        "metric": "GF(2^e) element-MAC/s at 8192^3 e=8",
        "value": value,
        "unit": "element-MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: C=A*B over F_2^{e} (f={f:#x}), {m}x{k}x{n}, "
                               "uint8 entries uniform in the field, device-resident",
                   "e": e, "f": hex(f), "m": m, "k": k, "n": n, "products": T,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "stages_ms": {s: round(v, 4) for s, v in stages.items()},
        "stages_hbm_GBs": hbm,
    }

    # The XOR/popcount VALU kernel on the same product, for comparison.
    if args.kernel < 0 and not args.profile_run:
        vctx = g.Context(0, kernel=g.KERNEL_VALU_128)
        vctx.mul_async(Ad, Bd, e, f, out=C)
        vctx.profile(True)
        vctx.profile_reset()
        for _ in range(3):
            vctx.mul_async(Ad, Bd, e, f, out=C)
        vctx.sync()
        ms, cnt = vctx.profile_read(g.STAGE_PRODUCTS)
        out["valu_products_ms"] = round(ms / max(cnt, 1), 4)
        vctx.close()

    if not args.no_forms:
        out["forms"] = forms_leg(g, torch, workload, lambda *a: log(args, *a))
    if not args.no_wide:
        out["wide"] = wide_leg(g, torch, workload, lambda *a: log(args, *a))
    if not args.no_trsm:
        out["trsm"] = trsm_leg(g, torch, workload, lambda *a: log(args, *a))
    if not args.no_echelon:
        out["echelon"] = echelon_leg(g, torch, workload, lambda *a: log(args, *a))
    if not args.no_batched:
        out["batched"] = batched_leg(g, torch, workload, lambda *a: log(args, *a))
    serve_state = None
    if not args.no_serve:
        out["serving"], serve_state = serve_leg(
            g, torch, workload, lambda *a: log(args, *a), budget=args.serve_budget_mib << 20,
            max_inflight=args.serve_inflight, bypass=args.serve_bypass,
            verify=not args.no_serve_verify)

    if not args.no_cpu:
        log(args, "timing the CPU oracle on the benchmark product")
        out["cpu_baseline"] = cpu_baseline(A, B, C_timed, e, f, args.cpu_seconds, workload,
                                           echelon=not args.no_echelon, no_trsm=args.no_trsm)
        if serve_state is not None:
            log(args, "serving: the oracle's Freivalds check on every served result")
            bad, nsample, sample_bad, secs = serving_freivalds(serve_state, lambda *a: log(args, *a))
            out["serving"]["freivalds_failures"] = bad
            out["serving"]["freivalds_trials"] = "ceil(64/e) per result"
            out["serving"]["oracle_sample"] = {"requests": nsample, "mismatched": sample_bad}
            out["serving"]["verified"] = (bad == 0 and sample_bad == 0 and
                                          out["serving"].get("alone_vs_mix_mismatches") == 0)
            out["serving"]["verify_s"] = round(secs, 1)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
