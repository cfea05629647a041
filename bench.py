"""Benchmark: dense C = A*B over F_256 (f = 0x11D), 8192 x 8192 x 8192, on one MI355X.

One step is the whole product pipeline on device-resident uint8 inputs: slice
A and B into Karatsuba operand planes, the 27 GF(2) plane products, and the
fused recombination / reduction mod f / clinging into C.  The line printed
also carries the roofline of the dominant kernel (the plane products, int8
MFMA), the CPU oracle timed on a bounded sample, the batched-vs-plain speedup
on 512 mixed products and the served p50/p99 latency (see --no-batched,
--no-serve).
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

PEAK_INT8_TOPS = 5000.0   # MI355X dense int8 MFMA, 5.0 POP/s
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E, 8 TB/s


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="f256_8192")
    ap.add_argument("--kernel", type=int, default=-1, help="force a product kernel (-1 = autotuned)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU oracle sample budget")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *msg):
    if not args.quiet:
        print("[bench]", *msg, file=sys.stderr, flush=True)


def cpu_baseline(A, B, e, f, budget_s):
    """The oracle on whole rows of the same product until the budget is used."""
    import oracle
    threads = oracle.max_threads()
    k, n = B.shape
    rows, spent, chunk = 0, 0.0, 16
    while spent < budget_s and rows + chunk <= A.shape[0]:
        t0 = time.perf_counter()
        oracle.matmul(A[rows:rows + chunk], B, e, f, nthreads=threads)
        dt = time.perf_counter() - t0
        spent += dt
        rows += chunk
        if dt < budget_s / 8:
            chunk *= 2
    macs = rows * k * n
    return {"value": macs / spent, "unit": "element-MAC/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows} of {A.shape[0]} rows of C ({rows}x{k}x{n} element-MAC), "
                      f"{spent:.1f} s on {threads} threads"}


def main():
    args = parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; multi-GPU runs are not "
                                   "supported (products shard by output rows, see DESIGN.md)",
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

    ctx = g.Context(0, kernel=args.kernel, autotune=args.kernel < 0)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.mul_async(Ad, Bd, e, f, out=C)
    ctx.sync()
    kind = ctx.chosen_kernel(e, m, k, n)
    log(args, f"product kernel: {g.kernel_names()[kind]}")

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

    T = g.num_products(e)
    prod_ms = stages["products"]
    ops = 2.0 * T * m * n * k  # int8 MFMA ops: one 0/1 multiply-add = 2 ops
    achieved = ops / (prod_ms / 1e3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_INT8_TOPS,
                "unit": "TOP/s", "frac": round(achieved / PEAK_INT8_TOPS, 4), "traffic": None,
                "kernel": g.kernel_names()[kind], "avg_launch_ms": round(prod_ms, 4),
                "algorithmic_ops_per_launch": ops}
    # HBM-bound stages: algorithmic bytes (elements in/out + planes written/read).
    esz = 1 if e <= 8 else 2
    kw = 2 * -(-k // 128)
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
    if args.kernel < 0:
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

    if not args.no_batched and hasattr(g, "batched_bench"):
        out["batched"] = g.batched_bench(ctx, log=lambda *a: log(args, *a))
    if not args.no_serve and hasattr(g, "serve_bench"):
        out["serving"] = g.serve_bench(ctx, log=lambda *a: log(args, *a))

    if not args.no_cpu:
        log(args, "timing the CPU oracle on a row sample")
        out["cpu_baseline"] = cpu_baseline(A, B, e, f, args.cpu_seconds)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
