#!/usr/bin/env python3
"""Throughput of forward CSR SpMM (C = A B) on one MI355X.

Workload (default): the power-law matrix - m = k = 1,000,000, Zipf-2.1 row
lengths with mean 16 capped at 100,000, uniform random columns, values N(0,1)
- times B with n = 64 columns, uniform[-1, 1), all float32, synthetic and
seeded. The plan (kernel choice by timing, merge-path partition) is built
once before the timed region, as A's structure is fixed across steps; each
step is one full product (main kernel plus, for merge-based plans, the
carry-out fix-up pass).

Prints one JSON line: GFLOP/s = 2 nnz n / t over K timed steps, the roofline
of the main kernel (algorithmic bytes per launch over its event-timed
duration against 8 TB/s HBM), HBM traffic from committed rocprofv3 counters
when they match the current kernel sources, and the FP64 CPU oracle timed on
this host's cores as a baseline.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters.json")


def kernel_source_hash(files):
    """Hash of the sources a kernel is built from (counters taken on another
    version of them do not describe the current kernel)."""
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1803_08601_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


class HipEvents:
    """Raw hipEvents from the HIP runtime, so that the library can record them
    around its main kernel on the stream it launches on."""

    def __init__(self):
        self.L = ctypes.CDLL("libamdhip64.so")
        self.L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.L.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        assert self.L.hipEventCreate(ctypes.byref(e)) == 0
        return e

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        assert self.L.hipEventElapsedTime(ctypes.byref(ms), a, b) == 0
        return ms.value

    def destroy(self, e):
        self.L.hipEventDestroy(e)


def bytes_min(m, k, nnz, n, sv, sb):
    """Compulsory traffic: row offsets, column indices and values of A once,
    B once, C written once."""
    return 4 * (m + 1) + (4 + sv) * nnz + sb * k * n + 4 * m * n


def make_workload(name, n):
    from paper_1803_08601_amd import workloads as wl
    if name == "powerlaw":
        A = wl.power_law(seed=1002)
        desc = f"power-law CSR 1M x 1M, Zipf 2.1 row lengths mean 16 cap 1e5, n={n}"
    elif name == "stencil":
        A = wl.stencil27(seed=1003)
        desc = f"27-point stencil CSR on 128^3 grid, n={n}"
    elif name == "plain":
        A = wl.plain(seed=1001)
        desc = f"uniform CSR 4096 x 4096, 16 per row, n={n}"
    else:
        raise SystemExit(f"unknown workload {name}")
    B = wl.dense({"powerlaw": 1002, "stencil": 1003, "plain": 1001}[name], A.k, n)
    return A, B, desc


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def gcn_fwd_bwd(steps=20, warmup=3):
    """Differentiable SpMM on the GCN adjacency (500k nodes, mean degree 32,
    n = 128): one step = forward C = A B, then dB = A^T dC and dvals =
    SDDMM(dC, B). BF16 storage of vals and B against float32 storage, both
    with float32 accumulation; accuracy of both is checked by the test suite
    against the FP64 oracle at full size."""
    import torch
    from paper_1803_08601_amd import native as nv
    from paper_1803_08601_amd import workloads as wl
    A = wl.gcn_adjacency(seed=1004)
    n = 128
    B = wl.dense(1004, A.k, n)
    dC = torch.from_numpy(wl.dense(1004, A.m, n, kind="normal", stream=2)).cuda()
    rp, ci = torch.from_numpy(A.rowptr).cuda(), torch.from_numpy(A.colind).cuda()
    out = {"workload": "GCN normalised adjacency, 500k nodes, mean degree 32, n=128",
           "nnz": A.nnz}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        vals = torch.from_numpy(A.vals.astype(np.float32)).to(dt).cuda()
        Bt = torch.from_numpy(B).to(dt).cuda()
        sv = torch.tensor([], dtype=dt).element_size()
        plan = nv.Plan(rp, ci, A.m, A.k, n, dtype=nv.dtype_code(dt), mode="autotune", nnz=A.nnz)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.transpose_build()
        torch.cuda.synchronize()
        tr_ms = (time.perf_counter() - t0) * 1e3
        C = torch.empty(A.m, n, device="cuda")
        dB = torch.empty(A.k, n, device="cuda")
        dv = torch.empty(A.nnz, device="cuda")
        fwd = _timed(lambda: plan.execute(vals, Bt, C), steps, warmup)
        bwd_b = _timed(lambda: plan.execute_t(vals, dC, dB), steps, warmup)
        bwd_v = _timed(lambda: plan.sddmm(dC, Bt, dv), steps, warmup)

        def step():
            plan.execute(vals, Bt, C)
            plan.execute_t(vals, dC, dB)
            plan.sddmm(dC, Bt, dv)
        total = _timed(step, steps, warmup)
        # compulsory bytes of each product (A, the dense inputs and outputs once)
        b_fwd = bytes_min(A.m, A.k, A.nnz, n, sv, sv)
        b_db = 4 * (A.k + 1) + (4 + 4) * A.nnz + (4 + 4 + sv) * A.nnz + 4 * A.m * n + 4 * A.k * n
        b_dv = 4 * (A.m + 1) + 4 * A.nnz + 4 * A.m * n + sv * A.k * n + 4 * A.nnz

        def gbs(b, ms_):
            return round(b / (ms_ * 1e-3) / 1e9, 1)
        out[name] = {"fwd_ms": round(fwd, 4), "dB_ms": round(bwd_b, 4), "dvals_ms": round(bwd_v, 4),
                     "fwd_bwd_ms": round(total, 4), "transpose_build_ms": round(tr_ms, 2),
                     "fwd_gflops": round(2.0 * A.nnz * n / (fwd * 1e-3) / 1e9, 1),
                     "algorithmic_GBs": {"fwd": gbs(b_fwd, fwd), "dB": gbs(b_db, bwd_b),
                                         "dvals": gbs(b_dv, bwd_v)},
                     "kernel": "merge" if plan.info().config.kernel else "rowsplit"}
        plan.close()
    out["bf16_speedup_fwd_bwd"] = round(out["f32"]["fwd_bwd_ms"] / out["bf16"]["fwd_bwd_ms"], 3)
    out["bf16_speedup_fwd"] = round(out["f32"]["fwd_ms"] / out["bf16"]["fwd_ms"], 3)
    return out


def batched(steps=10, warmup=2):
    """512 uneven products (m = k log-uniform in [1e3, 2e5], half U{8..64}
    rows and half Zipf-2.1 rows, n from {8, 32, 128}) in one persistent
    launch replayed from a hipGraph, against the plain float32 kernel called
    once per problem; float32 and BF16 storage, float32 accumulation."""
    import torch
    from paper_1803_08601_amd import native as nv
    from paper_1803_08601_amd import workloads as wl
    probs = wl.batch_parallel(seed=1005)
    flops = sum(2.0 * p.A.nnz * p.n for p in probs)
    out = {"workload": "512 uneven CSR products, m=k in [1e3, 2e5], n in {8, 32, 128}",
           "problems": len(probs), "nnz": int(sum(p.A.nnz for p in probs)), "gflop": round(flops / 1e9, 2)}
    dev = {}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        tensors, specs = [], []
        for b, P in enumerate(probs):
            A, n = P.A, P.n
            key = (b, "struct")
            if key not in dev:
                dev[key] = (torch.from_numpy(A.rowptr).cuda(), torch.from_numpy(A.colind).cuda())
            rp, ci = dev[key]
            vt = torch.from_numpy(A.vals).to(dt).cuda()
            Bt = torch.from_numpy(wl.dense(1005 + b, A.k, n)).to(dt).cuda()
            C = torch.empty(A.m, n, device="cuda")
            tensors.append((vt, Bt, C))
            specs.append(nv.spmm_problem(rp.data_ptr(), ci.data_ptr(), vt.data_ptr(), Bt.data_ptr(),
                                         C.data_ptr(), A.m, A.k, A.nnz, n, n))
        t0 = time.perf_counter()
        h = nv.spmm_batch_plan(specs, nv.dtype_code(dt), nv.SPMM_MODE_AUTOTUNE)
        plan_s = time.perf_counter() - t0
        ms = _timed(lambda: nv.spmm_batch_run(h), steps, warmup)
        cfgs = [nv.spmm_batch_problem_config(h, b) for b in range(len(probs))]
        nv.spmm_batch_destroy(h)
        sv = torch.tensor([], dtype=dt).element_size()
        bmin = sum(bytes_min(P.A.m, P.A.k, P.A.nnz, P.n, sv, sv) for P in probs)
        rec = {"graph_ms": round(ms, 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
               "algorithmic_GBs": round(bmin / (ms * 1e-3) / 1e9, 1),
               "plan_s": round(plan_s, 2), "merge_problems": int(sum(c.kernel for c in cfgs))}
        if name == "f32":
            # the plain kernel called once per problem: with the batch's own
            # shapes (isolates batching), and with the Sec. 5.4 rule's choice
            for label, mk in (("plain_same_shapes_ms", lambda b, P: dict(config=cfgs[b])),
                              ("plain_paper_rule_ms", lambda b, P: dict(mode="paper"))):
                plans = [nv.Plan(dev[(b, "struct")][0], dev[(b, "struct")][1], P.A.m, P.A.k, P.n,
                                 nnz=P.A.nnz, **mk(b, P)) for b, P in enumerate(probs)]

                def per_problem():
                    for pl, (vt, Bt, C) in zip(plans, tensors):
                        pl.execute(vt, Bt, C)
                rec[label] = round(_timed(per_problem, 3, 1), 4)
                for pl in plans:
                    pl.close()
        out[name] = rec
        del tensors, specs
    base = out["f32"]["plain_same_shapes_ms"]
    out["batched_speedup_vs_plain_f32_same_shapes"] = round(base / out["f32"]["graph_ms"], 3)
    out["bf16_batched_speedup_vs_plain_f32_same_shapes"] = round(base / out["bf16"]["graph_ms"], 3)
    out["batched_speedup_vs_plain_f32_paper_rule"] = round(
        out["f32"]["plain_paper_rule_ms"] / out["f32"]["graph_ms"], 3)
    return out


def cpu_baseline(A, B, n, budget_s=10.0, max_reps=8):
    import numpy as np
    import oracle
    threads = len(os.sched_getaffinity(0))
    times = []
    t_start = time.perf_counter()
    while len(times) < max_reps and (time.perf_counter() - t_start < budget_s or len(times) < 2):
        t0 = time.perf_counter()
        oracle.spmm(A.rowptr, A.colind, A.vals, B, n=n, nthreads=threads)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return {"value": 2.0 * A.nnz * n / t / 1e9, "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"full workload, {len(times)} passes of the FP64 oracle (OpenMP over rows, "
                      f"{threads} threads), median {t * 1e3:.1f} ms per pass"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="powerlaw", choices=["powerlaw", "stencil", "plain"])
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--mode", default="autotune", choices=["autotune", "paper", "rowsplit", "merge"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="only the headline product (skip the GCN fwd+bwd and batched extras)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1803_08601_amd import native as nv

    if args.copy_calibration:
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": a.numel() * 4}))
        return

    dt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[args.dtype]
    A, B, desc = make_workload(args.workload, args.n)
    n = args.n
    rp = torch.from_numpy(A.rowptr).cuda()
    ci = torch.from_numpy(A.colind).cuda()
    vals = torch.from_numpy(A.vals).to(dt).cuda()
    Bt = torch.from_numpy(B).to(dt).cuda()
    C = torch.empty(A.m, n, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    plan = nv.Plan(rp, ci, A.m, A.k, n, ld=n, dtype=nv.dtype_code(dt), mode=args.mode, nnz=A.nnz)
    plan_s = time.perf_counter() - t0
    info = plan.info()
    kernel = "merge" if info.config.kernel == nv.SPMM_KERNEL_MERGE else "rowsplit"

    ev = HipEvents()
    evb = [ev.create() for _ in range(args.steps)]
    eva = [ev.create() for _ in range(args.steps)]
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.execute(vals, Bt, C)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        nv.spmm_execute_events(plan.handle, vals, Bt, C, evb[i], eva[i], stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms = [ev.elapsed_ms(evb[i], eva[i]) for i in range(args.steps)]
    for e in evb + eva:
        ev.destroy(e)

    ms = (t1 - t0) * 1e3 / args.steps
    flops = 2.0 * A.nnz * n
    gflops = flops / (ms * 1e-3) / 1e9
    sv = sb = torch.tensor([], dtype=dt).element_size()
    bmin = bytes_min(A.m, A.k, A.nnz, n, sv, sb)
    kavg = float(np.mean(kern_ms))
    achieved = bmin / (kavg * 1e-3) / 1e9

    traffic = None
    if os.path.exists(COUNTERS):
        rec = json.load(open(COUNTERS))
        key = f"{args.workload}-n{n}-{args.dtype}-{kernel}"
        r = rec.get(key)
        if (r and r.get("kernel_source_sha") == kernel_source_hash(r["files"])
                and r.get("config") in (None, info.config.as_dict())):
            traffic = round(r["fetch_kib"] * 1024.0 * r["fetch_scale"]
                            + r["write_kib"] * 1024.0 * r["write_scale"])

    out = {
        "metric": "SpMM GFLOP/s (2*nnz*n/t)",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": desc, "m": A.m, "k": A.k, "nnz": A.nnz, "n": n,
                   "kernel": kernel, "mode": args.mode, "shape": info.config.as_dict(),
                   "paper_rule_kernel": "merge" if info.paper_choice else "rowsplit",
                   "plan_build_s": round(plan_s, 3), "input_sha": A.digest()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_merge" if kernel == "merge" else "k_rowsplit",
                     "kernel_ms": round(kavg, 4), "algorithmic_bytes": bmin},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, n)
    if not args.quick:
        del C, Bt, vals
        plan.close()
        torch.cuda.empty_cache()
        out["extra"] = {"gcn_fwd_bwd": gcn_fwd_bwd(), "batched": batched()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
