#!/usr/bin/env python3
"""Throughput of forward CSR SpMM (C = A B) on one MI355X.

Workload (default): the power-law matrix - m = k = 1,000,000, Zipf-2.1 row
lengths with mean 16 capped at 100,000, uniform random columns, values N(0,1)
- times B with n = 64 columns, uniform[-1, 1), all float32, synthetic and
seeded. The plan (kernel choice by timing, merge-path partition) is built
once before the timed region, as A's structure is fixed across steps; each
step is one full product (main kernel plus, for merge-based plans, the
carry-out fix-up pass).

Timing: each timed step starts from cold caches - 1 GiB written just before
it (outside its hipEvents) evicts L2 and the Infinity Cache - and its time
is the hipEvent interval around the whole product. The warm rate (steps back
to back, wall clock) is reported beside it.

Prints one JSON line: GFLOP/s = 2 nnz n / t, the roofline of the main kernel
(algorithmic bytes per launch over its event-timed duration against 8 TB/s
HBM), the L2-to-fabric traffic from committed rocprofv3 counters when they
were taken on the current kernel sources, and the FP64 CPU oracle timed on
this host's cores as a baseline; the other workloads follow under "extra".
"""
import argparse
import ctypes
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters.json")
# the autotuner's choices from the traced runs the counter records were taken
# on (one line per matrix key); loaded by default so that every row plans the
# shapes its counters describe
BENCH_TUNE_CACHE = os.path.join(ROOT, "profiles", "bench_tune_cache.txt")
TRAFFIC_SOURCE = ("rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, scaled by a 1 GiB copy: "
                  "bytes between the L2 caches and the fabric, which include Infinity Cache "
                  "(MALL) hits - an upper bound on DRAM traffic, not DRAM traffic itself")


# device sources no product launches (the gather calibration kernel)
NOT_PRODUCT_SOURCES = {"calib.hip"}


def kernel_source_hash():
    """Hash of the device sources of the products (every .hip and .hpp file of
    the library but the calibration kernel): counters taken on another version
    of them do not describe the kernels."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_08601_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        if os.path.basename(f) in NOT_PRODUCT_SOURCES:
            continue
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def load_counters():
    return json.load(open(COUNTERS)) if os.path.exists(COUNTERS) else {}


def counter_record(records, key, config):
    """The counter record of row `key` taken for exactly this launch shape on
    the current kernel sources, else None."""
    sha = kernel_source_hash()
    for r in records.get(key, []):
        rc = r.get("config", {})
        same = (all(config.get(k) == v for k, v in rc.items())
                and all(v == 0 for k, v in config.items() if k not in rc))
        if same and r.get("kernel_source_sha") == sha:
            return r
    return None


def traffic_fields(records, key, config, bmin, bgat, ms):
    """Counter traffic of one row per launch, its rate over the row's
    event-timed `ms`, and its ratio to the compulsory bytes (null fields
    when no current record exists)."""
    r = counter_record(records, key, config)
    t = None if r is None else int(round(r["traffic_bytes"]))
    return {"traffic": t,
            "traffic_GBs": None if t is None else round(t / (ms * 1e-3) / 1e9, 1),
            "traffic_over_bytes_min": None if t is None else round(t / bmin, 3),
            "l2_hit_rate": None if r is None else r.get("l2_hit_rate"),
            "ta_busy": None if r is None else r.get("ta_busy"),
            "counter_profile": None if r is None else r.get("profile"),
            "bytes_min": bmin,
            "bytes_min_frac": round(bmin / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "gather_model_bytes": bgat,
            "gather_model_frac": None if bgat is None
            else round(bgat / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


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


def spread(ms):
    """Mean, median, 10th and 90th percentile of a list of times (ms)."""
    a = np.asarray(ms, dtype=np.float64)
    return {"mean": round(float(a.mean()), 4), "median": round(float(np.median(a)), 4),
            "p10": round(float(np.percentile(a, 10)), 4),
            "p90": round(float(np.percentile(a, 90)), 4)}


_SCRUB = None


def scrub():
    """1 GiB of writes: evicts L2 (4 MB per XCD) and the 256 MB Infinity Cache."""
    import torch
    global _SCRUB
    if _SCRUB is None:
        _SCRUB = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    _SCRUB.fill_(1.0)


def time_steps(run, steps, warmup, library_events=True):
    """Time `run(ev_before, ev_after)` (one product on torch's current stream;
    the library may record the two hipEvents around its main kernel, or
    ignore them): `warmup` untimed runs; `steps` warm runs back to back
    (wall clock between two device synchronisations); then `steps` cold runs,
    each after scrub() and bracketed by torch events, with the device
    synchronised before the first and after the last. Cold launches come
    last, so a profiler's last `steps` dispatches of a kernel are the cold
    ones."""
    import torch
    ev = HipEvents()
    evb = [ev.create() for _ in range(2 * steps)]
    eva = [ev.create() for _ in range(2 * steps)]
    t_start = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t_end = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for _ in range(warmup):
        run(None, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        run(evb[i], eva[i])
    torch.cuda.synchronize()
    warm_wall = (time.perf_counter() - t0) * 1e3 / steps
    scrub()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        scrub()
        t_start[i].record()
        run(evb[steps + i], eva[steps + i])
        t_end[i].record()
    torch.cuda.synchronize()
    cold_wall = (time.perf_counter() - t0) * 1e3 / steps

    def kern(lo):
        return [ev.elapsed_ms(evb[i], eva[i]) for i in range(lo, lo + steps)]
    # (events the run did not record are never queried: a failed query would
    # leave an error for the next runtime call to report)
    warm_k, cold_k = (kern(0), kern(steps)) if library_events else (None, None)
    cold_step = [t_start[i].elapsed_time(t_end[i]) for i in range(steps)]
    for e in evb + eva:
        ev.destroy(e)
    return {"cold_step": cold_step, "cold_kernel": cold_k or cold_step, "cold_wall": cold_wall,
            "warm_wall": warm_wall, "warm_kernel": warm_k}


def bytes_min(m, k, nnz, n, sv, sb):
    """Compulsory traffic: row offsets, column indices and values of A once,
    B once, C written once."""
    return 4 * (m + 1) + (4 + sv) * nnz + sb * k * n + 4 * m * n


def bytes_gather(m, nnz, n, sv, sb):
    """Traffic of the gather model of Table 1: as bytes_min, but every entry
    fetches its B row (no reuse of B rows on chip)."""
    return 4 * (m + 1) + (4 + sv) * nnz + sb * nnz * n + 4 * m * n


def main_kernel_patterns(kernel):
    """Regular expressions of the kernels one product launches (for the
    profiler's dispatch records), by plan kernel."""
    if kernel in ("merge", "nzsplit"):
        return [r"\bk_merge<", r"\bk_merge_fixup<"]
    return [{"rowsplit": r"\bk_rowsplit<", "rowblock": r"\bk_rowblock<"}[kernel]]


WORKLOADS = {
    "powerlaw": ("power-law CSR 1M x 1M, Zipf 2.1 row lengths mean 16 cap 1e5", 1002),
    "stencil": ("27-point stencil CSR on 128^3 grid", 1003),
    "plain": ("uniform CSR 4096 x 4096, 16 per row", 1001),
}


def make_workload(name, n):
    from paper_1803_08601_amd import workloads as wl
    if name == "powerlaw":
        A = wl.power_law(seed=1002)
    elif name == "stencil":
        A = wl.stencil27(seed=1003)
    elif name == "plain":
        A = wl.plain(seed=1001)
    else:
        raise SystemExit(f"unknown workload {name}")
    B = wl.dense(WORKLOADS[name][1], A.k, n)
    return A, B, f"{WORKLOADS[name][0]}, n={n}"


def single_product(A, B, n, dt, mode="autotune", cfg=None, steps=20, warmup=3, key=None,
                   records=None, manifest=None):
    """One planned product timed by time_steps; returns its row (times,
    GFLOP/s, compulsory and gather-model fractions, counter traffic) and the
    plan facts."""
    import torch
    from paper_1803_08601_amd import native as nv
    rp, ci = torch.from_numpy(A.rowptr).cuda(), torch.from_numpy(A.colind).cuda()
    vals = torch.from_numpy(A.vals).to(dt).cuda()
    Bt = torch.from_numpy(B).to(dt).cuda()
    C = torch.empty(A.m, n, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = nv.Plan(rp, ci, A.m, A.k, n, ld=n, dtype=nv.dtype_code(dt), mode=mode, config=cfg,
                   nnz=A.nnz)
    plan_s = time.perf_counter() - t0
    info = plan.info()
    kernel = nv.KERNEL_NAMES[info.config.kernel]
    stream = torch.cuda.current_stream()

    def run(eb, ea):
        nv.spmm_execute_events(plan.handle, vals, Bt, C, eb, ea, stream)
    t = time_steps(run, steps, warmup)
    sz = torch.tensor([], dtype=dt).element_size()
    bmin = bytes_min(A.m, A.k, A.nnz, n, sz, sz)
    bgat = bytes_gather(A.m, A.nnz, n, sz, sz)
    flops = 2.0 * A.nnz * n
    step = float(np.mean(t["cold_step"]))
    kms = float(np.mean(t["cold_kernel"]))
    cfgd = info.config.as_dict()
    row = {"n": n, "dtype": str(dt).replace("torch.", ""), "nnz": A.nnz, "kernel": kernel,
           "shape": cfgd, "plan_build_s": round(plan_s, 3),
           "paper_rule_kernel": "merge" if info.paper_choice else "rowsplit",
           "ms_per_step": round(step, 4), "gflops": round(flops / (step * 1e-3) / 1e9, 1),
           "kernel_ms": {"cold": spread(t["cold_kernel"]), "warm": spread(t["warm_kernel"])},
           "warm": {"ms_per_step": round(t["warm_wall"], 4),
                    "gflops": round(flops / (t["warm_wall"] * 1e-3) / 1e9, 1)},
           "tile_order": {"plane_rows": info.plane_rows, "strip_rows": info.strip_rows}}
    if key is not None:
        row.update(traffic_fields(records or {}, key, cfgd, bmin, bgat, kms))
    if manifest is not None:
        manifest.append({"row": key, "config": cfgd, "steps": steps,
                         "patterns": main_kernel_patterns(kernel),
                         "bytes_min": bmin, "bytes_gather": bgat,
                         "kernel_ms_cold_mean": round(kms, 4)})
    plan.close()
    return row, info, t


def other_configs(A_pl, records, steps=20, warmup=3, only=None, manifest=None):
    """The remaining single-product workloads, each planned by timing: the
    uniform 4096 x 4096 matrix with 16 entries per row at n = 32 (a
    launch-bound size), the power-law matrix at n = 8, the same at n = 64
    with BF16 storage, and the 27-point stencil on 128^3 at n = 16 and
    n = 128 (float32); timed as the headline (cold steps, warm beside)."""
    import torch
    from paper_1803_08601_amd import workloads as wl
    out = {}
    rows = [("plain-n32-f32", "plain", 32, torch.float32),
            ("powerlaw-n8-f32", "powerlaw", 8, torch.float32),
            ("powerlaw-n64-bf16", "powerlaw", 64, torch.bfloat16),
            ("stencil-n16-f32", "stencil", 16, torch.float32),
            ("stencil-n128-f32", "stencil", 128, torch.float32)]
    S = None
    for key, wname, n, dt in rows:
        if only is not None and key != only:
            continue
        if wname == "powerlaw":
            A = A_pl if A_pl is not None else wl.power_law(seed=1002)
        elif wname == "stencil":
            S = S if S is not None else wl.stencil27(seed=1003)
            A = S
        else:
            A = wl.plain(seed=1001)
        B = wl.dense(WORKLOADS[wname][1], A.k, n)
        row, _, _ = single_product(A, B, n, dt, steps=steps, warmup=warmup, key=key,
                                   records=records, manifest=manifest)
        row["workload"] = f"{WORKLOADS[wname][0]}, n={n}"
        out[key] = row
        torch.cuda.empty_cache()
    return out


def gcn_fwd_bwd(records, steps=20, warmup=3, only=None, manifest=None):
    """Differentiable SpMM on the GCN adjacency (500k nodes, mean degree 32,
    n = 128): forward C = A B, then dB = A^T dC and dvals = SDDMM(dC, B).
    BF16 storage of vals and B against float32 storage, both with float32
    accumulation; accuracy of both is checked by the test suite against the
    FP64 oracle at full size. Each of the three products is timed like the
    headline (cold steps, warm beside); fwd_bwd is the three back to back
    (warm). `only` = "f32-fwd", "bf16-dB", ... times just that product."""
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
    stream = torch.cuda.current_stream()
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        if only is not None and not only.startswith(name + "-"):
            continue
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
        fcfg = plan.info().config.as_dict()
        fkern = nv.KERNEL_NAMES[fcfg["kernel"]]
        # the A^T product's plan (same mode) is internal; its kernel shows in
        # the profile; the record is keyed by the forward plan's shape
        prods = {
            "fwd": (lambda eb, ea: nv.spmm_execute_events(plan.handle, vals, Bt, C, eb, ea, stream),
                    bytes_min(A.m, A.k, A.nnz, n, sv, sv), bytes_gather(A.m, A.nnz, n, sv, sv),
                    main_kernel_patterns(fkern)),
            # dB = A^T dC: the value gather (perm: 4, vals: s_v read, float32
            # written, read again) and the product over A^T with dC float32
            "dB": (lambda eb, ea: plan.execute_t(vals, dC, dB),
                   4 * (A.k + 1) + 4 * A.nnz + (4 + sv + 4 + 4) * A.nnz + 4 * A.m * n
                   + 4 * A.k * n,
                   4 * (A.k + 1) + 4 * A.nnz + (4 + sv + 4 + 4) * A.nnz + 4 * A.nnz * n
                   + 4 * A.k * n,
                   [r"\bk_gather_widen", r"\bk_merge<|\bk_rowsplit<|\bk_rowblock<",
                    r"\bk_merge_fixup<"]),
            # dvals: row offsets, column indices, dC once, B, dvals written
            "dvals": (lambda eb, ea: plan.sddmm(dC, Bt, dv),
                      4 * (A.m + 1) + 4 * A.nnz + 4 * A.m * n + sv * A.k * n + 4 * A.nnz,
                      4 * (A.m + 1) + 4 * A.nnz + 4 * A.m * n + sv * A.nnz * n + 4 * A.nnz,
                      [r"\bk_sddmm<"]),
        }
        rec = {"transpose_build_ms": round(tr_ms, 2), "kernel": fkern, "shape": fcfg}
        for pname, (run, bmin, bgat, pats) in prods.items():
            key = f"gcn-n128-{name}-{pname}"
            if only is not None and only != f"{name}-{pname}":
                continue
            t = time_steps(run, steps, warmup, library_events=pname == "fwd")
            ms = float(np.mean(t["cold_step"]))
            rec[pname] = {"ms_per_step": round(ms, 4),
                          "gflops": round(2.0 * A.nnz * n / (ms * 1e-3) / 1e9, 1),
                          "cold_ms": spread(t["cold_step"]),
                          "warm_ms_per_step": round(t["warm_wall"], 4)}
            rec[pname].update(traffic_fields(records, key, fcfg, bmin, bgat, ms))
            if manifest is not None:
                manifest.append({"row": key, "config": fcfg, "steps": steps, "patterns": pats,
                                 "bytes_min": bmin, "bytes_gather": bgat,
                                 "kernel_ms_cold_mean": round(ms, 4)})
        if only is None:
            def step():
                plan.execute(vals, Bt, C)
                plan.execute_t(vals, dC, dB)
                plan.sddmm(dC, Bt, dv)
            t = time_steps(lambda eb, ea: step(), steps, warmup, library_events=False)
            rec["fwd_bwd_ms"] = round(float(np.mean(t["cold_step"])), 4)
            rec["fwd_bwd_warm_ms"] = round(t["warm_wall"], 4)
            rec["dB_scatter_ms"] = round(float(np.mean(time_steps(
                lambda eb, ea: plan.execute_t_scatter(vals, dC, dB), 5, 1,
                library_events=False)["cold_step"])), 4)
        out[name] = rec
        plan.close()
    if only is None:
        out["bf16_speedup_fwd_bwd"] = round(out["f32"]["fwd_bwd_ms"] / out["bf16"]["fwd_bwd_ms"], 3)
        out["bf16_speedup_fwd"] = round(out["f32"]["fwd"]["ms_per_step"]
                                        / out["bf16"]["fwd"]["ms_per_step"], 3)
    return out


def batched(records, steps=10, warmup=2, only=None, manifest=None):
    """512 uneven products (m = k log-uniform in [1e3, 2e5], half U{8..64}
    rows and half Zipf-2.1 rows, n from {8, 32, 128}) in one persistent
    launch replayed from a hipGraph, against the plain float32 kernel called
    once per problem; float32 and BF16 storage, float32 accumulation. The
    graph replays are timed like the headline (cold steps, warm beside)."""
    import torch
    from paper_1803_08601_amd import native as nv
    from paper_1803_08601_amd import workloads as wl
    probs = wl.batch_parallel(seed=1005)
    flops = sum(2.0 * p.A.nnz * p.n for p in probs)
    out = {"workload": "512 uneven CSR products, m=k in [1e3, 2e5], n in {8, 32, 128}",
           "problems": len(probs), "nnz": int(sum(p.A.nnz for p in probs)), "gflop": round(flops / 1e9, 2)}
    dev = {}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        if only is not None and only != name:
            continue
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
        t = time_steps(lambda eb, ea: nv.spmm_batch_run(h), steps, warmup, library_events=False)
        ms = float(np.mean(t["cold_step"]))
        cfgs = [nv.spmm_batch_problem_config(h, b) for b in range(len(probs))]
        nv.spmm_batch_destroy(h)
        sv = torch.tensor([], dtype=dt).element_size()
        bmin = sum(bytes_min(P.A.m, P.A.k, P.A.nnz, P.n, sv, sv) for P in probs)
        bgat = sum(bytes_gather(P.A.m, P.A.nnz, P.n, sv, sv) for P in probs)
        rec = {"graph_ms": round(ms, 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
               "cold_ms": spread(t["cold_step"]), "warm_ms_per_step": round(t["warm_wall"], 4),
               "warm_gflops": round(flops / (t["warm_wall"] * 1e-3) / 1e9, 1),
               "plan_s": round(plan_s, 2), "merge_problems": int(sum(c.kernel for c in cfgs))}
        key = f"batch-{name}"
        rec.update(traffic_fields(records, key, {}, bmin, bgat, ms))
        if manifest is not None:
            manifest.append({"row": key, "config": {}, "steps": steps,
                             "patterns": [r"\bk_batch<", r"\bk_batch_fixup\b"],
                             "bytes_min": bmin, "bytes_gather": bgat,
                             "kernel_ms_cold_mean": round(ms, 4)})
        if name == "f32" and only is None:
            # the plain kernel called once per problem: with the batch's own
            # shapes (isolates batching), and with the Sec. 5.4 rule's choice
            for label, mk in (("plain_same_shapes_ms", lambda b, P: dict(config=cfgs[b])),
                              ("plain_paper_rule_ms", lambda b, P: dict(mode="paper"))):
                plans = [nv.Plan(dev[(b, "struct")][0], dev[(b, "struct")][1], P.A.m, P.A.k, P.n,
                                 nnz=P.A.nnz, **mk(b, P)) for b, P in enumerate(probs)]

                def per_problem():
                    for pl, (vt, Bt, C) in zip(plans, tensors):
                        pl.execute(vt, Bt, C)
                rec[label] = round(float(np.mean(time_steps(lambda eb, ea: per_problem(), 3, 1,
                                                            library_events=False)
                                                 ["cold_step"])), 4)
                for pl in plans:
                    pl.close()
        out[name] = rec
        del tensors, specs
    if only is None:
        base = out["f32"]["plain_same_shapes_ms"]
        out["batched_speedup_vs_plain_f32_same_shapes"] = round(base / out["f32"]["graph_ms"], 3)
        out["bf16_batched_speedup_vs_plain_f32_same_shapes"] = round(base / out["bf16"]["graph_ms"], 3)
        out["batched_speedup_vs_plain_f32_paper_rule"] = round(
            out["f32"]["plain_paper_rule_ms"] / out["f32"]["graph_ms"], 3)
    return out


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


def _plan_time(nv, rp, ci, m, k, nnz, n, vals, Bt, C, cfg=None, mode=None, steps=10):
    plan = nv.Plan(rp, ci, m, k, n, nnz=nnz, config=cfg, mode=mode or "paper")
    ms = _timed(lambda: plan.execute(vals, Bt, C), steps, 2)
    info = plan.info()
    plan.close()
    return ms, info


def _best_of(nv, rp, ci, m, k, nnz, n, vals, Bt, C, kernel):
    """Fastest time of one kernel over its shape candidates (the autotuner's
    candidate set restricted to that kernel)."""
    import torch
    best = None
    if kernel in ("merge", "nzsplit"):
        code = nv.SPMM_KERNEL_MERGE if kernel == "merge" else nv.SPMM_KERNEL_NZSPLIT
        shapes = [dict(kernel=code, items_per_wg=W, unroll=u) for W in (1024, 2048, 4096)
                  for u in (2, 4, 8)]
    elif kernel == "rowblock":
        shapes = [dict(kernel=nv.SPMM_KERNEL_ROWBLOCK, rows_per_block=R, lanes_per_row=l,
                       unroll=u) for R in (2, 4) for l in (0, 64, 32, 16) for u in (2, 4)]
    else:
        shapes = [dict(kernel=0, lanes_per_row=l, unroll=u) for l in (0, 64, 32, 16, 8)
                  for u in (2, 4, 8)]
    for cfg in shapes:
        try:
            ms, _ = _plan_time(nv, rp, ci, m, k, nnz, n, vals, Bt, C, cfg=cfg, steps=3)
        except nv.SpmmError:
            continue
        if best is None or ms < best[0]:
            best = (ms, cfg)
        torch.cuda.synchronize()
    return best


def rowblock_sweep():
    """Row blocks against row split and the merge path on matrices whose
    neighbouring rows share columns (2-D and 3-D stencils) and on controls
    without that sharing (a banded matrix with random columns, the uniform
    matrix), at n = 16, 32, 64, 128 in float32; each kernel at its fastest
    shape. Prints one JSON line per (matrix, n) with the union size of blocks
    of 4 rows relative to the entry count."""
    import torch
    from paper_1803_08601_amd import native as nv
    from paper_1803_08601_amd import workloads as wl
    mats = [("27-point 3-D 128^3", lambda: wl.grid_stencil(11, (128, 128, 128), 27)),
            ("7-point 3-D 128^3", lambda: wl.grid_stencil(12, (128, 128, 128), 7)),
            ("9-point 2-D 1448^2", lambda: wl.grid_stencil(13, (1448, 1448), 9)),
            ("5-point 2-D 1448^2", lambda: wl.grid_stencil(14, (1448, 1448), 5)),
            ("banded, 16 random in +-512, 2M rows", lambda: wl.banded(15, 2_097_152)),
            ("uniform 16 per row, 2M x 2M", lambda: wl.plain(seed=16, m=2_097_152,
                                                             k=2_097_152))]
    rb_shapes = [dict(kernel=nv.SPMM_KERNEL_ROWBLOCK, rows_per_block=R, lanes_per_row=l, unroll=u)
                 for R in (2, 4, 8) for l in (64, 32, 16, 8) for u in (2, 4)]
    recs = []
    for desc, make in mats:
        A = make()
        rows = np.repeat(np.arange(A.m, dtype=np.int64) // 4, A.row_lengths())
        ratio4 = np.unique(rows * A.k + A.colind).size / A.nnz
        del rows
        rp, ci = torch.from_numpy(A.rowptr).cuda(), torch.from_numpy(A.colind).cuda()
        vals = torch.from_numpy(A.vals.astype(np.float32)).cuda()
        for n in (16, 32, 64, 128):
            Bt = torch.from_numpy(wl.dense(17, A.k, n)).cuda()
            C = torch.empty(A.m, n, device="cuda")
            rs = _best_of(nv, rp, ci, A.m, A.k, A.nnz, n, vals, Bt, C, "rowsplit")
            mg = _best_of(nv, rp, ci, A.m, A.k, A.nnz, n, vals, Bt, C, "merge")
            rb = None
            for cfg in rb_shapes:
                try:
                    ms, _ = _plan_time(nv, rp, ci, A.m, A.k, A.nnz, n, vals, Bt, C, cfg=cfg,
                                       steps=3)
                except nv.SpmmError:
                    continue
                if rb is None or ms < rb[0]:
                    rb = (ms, cfg)
            best = min((rs[0], "rowsplit"), (mg[0], "merge"), (rb[0], "rowblock"))
            rec = {"matrix": desc, "n": n, "m": A.m, "nnz": A.nnz,
                   "union_ratio_4": round(ratio4, 3), "max_row": int(A.row_lengths().max()),
                   "rowsplit_ms": round(rs[0], 4), "merge_ms": round(mg[0], 4),
                   "rowblock_ms": round(rb[0], 4), "rowblock_shape": rb[1],
                   "fastest": best[1]}
            print(json.dumps(rec), flush=True)
            recs.append(rec)
            del Bt, C
            torch.cuda.empty_cache()
        del rp, ci, vals, A
        torch.cuda.empty_cache()
    return recs


def heuristic_sweep(n=64):
    """Both kernels on matrices whose mean row length spans the Sec. 5.4
    threshold: dense-as-CSR shapes from 2 x 8.4M to 8.4M x 2 (2^24 entries,
    as in Fig. 1 and Fig. 4) and power-law matrices of several exponents and
    means. Prints one JSON line per matrix and a summary line with the
    threshold on the mean row length that best separates the faster kernel,
    and the accuracy of the paper's 9.35 against best-of-two."""
    import torch
    from paper_1803_08601_amd import native as nv
    from paper_1803_08601_amd import workloads as wl
    recs = []
    cases = []
    for lg in range(1, 24, 2):  # row length 2^lg, m = 2^(24 - lg)
        L, m = 1 << lg, 1 << (24 - lg)
        cases.append(("dense", L, m))
    for shape, mean in ((1.1, 4.0), (1.1, 8.0), (1.1, 12.0), (1.1, 32.0), (1.5, 6.0), (2.0, 10.0),
                        (0.8, 8.0)):
        cases.append(("zipf", shape, mean))
    for kind, a, b in cases:
        if kind == "dense":
            L, m = a, b
            rp = torch.arange(0, (m + 1) * L, L, dtype=torch.int64, device="cuda").to(torch.int32)
            ci = torch.arange(L, dtype=torch.int32, device="cuda").repeat(m)
            k, nnz, desc = L, m * L, f"dense {m} x {L}"
            maxrow = L
            r2 = 0.5  # every pair of rows holds the same columns
        else:
            shape, mean = a, b
            rng = np.random.default_rng(int(shape * 100 + mean))
            lengths, _ = wl.power_law_lengths(rng, 1_000_000, mean=mean, cap=100_000, shape=shape)
            cols = wl.distinct_sorted_columns(rng, lengths, 1_000_000)
            rp = torch.from_numpy(wl.rowptr_from_lengths(lengths)).cuda()
            ci = torch.from_numpy(cols).cuda()
            m, k, nnz = 1_000_000, 1_000_000, int(lengths.sum())
            maxrow = int(lengths.max())
            pair = np.repeat(np.arange(m, dtype=np.int64) // 2, lengths)
            r2 = np.unique(pair * k + cols).size / nnz
            del pair
            desc = f"power law, tail exponent {shape + 1.0:.1f}, mean {mean:g}, 1M x 1M"
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        vals = torch.rand(nnz, generator=g, device="cuda") - 0.5
        Bt = torch.rand(k, n, generator=g, device="cuda") - 0.5
        C = torch.empty(m, n, device="cuda")
        rs = _best_of(nv, rp, ci, m, k, nnz, n, vals, Bt, C, "rowsplit")
        mg = _best_of(nv, rp, ci, m, k, nnz, n, vals, Bt, C, "merge")
        # row blocks only where the rule could take them (rows of at most 4096)
        rb = _best_of(nv, rp, ci, m, k, nnz, n, vals, Bt, C, "rowblock") if maxrow <= 4096 \
            else None
        d = nnz / m
        if nnz < 4 * m or maxrow >= 4096:
            rule = "merge"
        elif n >= 32 and r2 <= 0.9:
            rule = "rowblock"
        else:
            rule = "rowsplit"
        times = {"rowsplit": rs[0], "merge": mg[0], "rowblock": rb[0] if rb else float("inf")}
        rec = {"matrix": desc, "m": m, "k": k, "nnz": nnz, "mean_row": d, "max_row": maxrow,
               "r2": round(r2, 3),
               "rowsplit_ms": round(rs[0], 4), "merge_ms": round(mg[0], 4),
               "rowblock_ms": round(rb[0], 4) if rb else None,
               "rowsplit_shape": rs[1], "merge_shape": mg[1],
               "rowblock_shape": rb[1] if rb else None,
               "faster": "merge" if mg[0] < rs[0] else "rowsplit",
               "fastest_of_three": min(times, key=times.get),
               "paper_rule": "merge" if 100 * nnz < 935 * m else "rowsplit",
               "mi355x_rule": rule}
        print(json.dumps(rec), flush=True)
        recs.append(rec)
        del rp, ci, vals, Bt, C
        torch.cuda.empty_cache()

    def acc(th):
        ok = [(r["mean_row"] < th) == (r["faster"] == "merge") for r in recs]
        return sum(ok) / len(ok)
    cands = sorted({r["mean_row"] for r in recs} | {9.35})
    best_th = max(cands, key=lambda t: (acc(t), -abs(t - 9.35)))

    def loss(th):  # slowdown of following the rule instead of best-of-two
        tot = 0.0
        for r in recs:
            pick = r["merge_ms"] if r["mean_row"] < th else r["rowsplit_ms"]
            tot += np.log(pick / min(r["merge_ms"], r["rowsplit_ms"]))
        return float(np.exp(tot / len(recs)))
    def rule_stats(key):
        # against the fastest of the three kernels
        def t(r, kern):
            return r[kern + "_ms"] if r[kern + "_ms"] is not None else float("inf")
        ok = [r[key] == r["fastest_of_three"] for r in recs]
        tot = sum(np.log(t(r, r[key]) / min(t(r, q) for q in ("rowsplit", "merge", "rowblock")))
                  for r in recs)
        return round(sum(ok) / len(ok), 3), round(float(np.exp(tot / len(recs))), 3)
    mi_acc, mi_loss = rule_stats("mi355x_rule")
    summary = {"summary": "heuristic sweep", "n": n, "matrices": len(recs),
                      "mi355x_rule": "merge if mean < 4 or longest row >= 4096; else row blocks "
                                     "of 2 if n >= 32 and pairs of rows hold <= 0.9 distinct "
                                     "columns per entry; else row split",
                      "mi355x_rule_accuracy": mi_acc, "mi355x_rule_geomean_slowdown": mi_loss,
                      "paper_threshold": 9.35, "paper_rule_accuracy": round(acc(9.35), 3),
                      "paper_rule_geomean_slowdown": round(loss(9.35), 3),
                      "best_threshold": best_th, "best_threshold_accuracy": round(acc(best_th), 3),
                      "best_threshold_geomean_slowdown": round(loss(best_th), 3)}
    print(json.dumps(summary), flush=True)
    return recs + [summary]


def nz_compare(n=64):
    """The nonzero split (Sec. 4, scheme (a): equal nonzeros per piece, 1-D
    search on row offsets) against the diagonal merge-path split and row
    split, each at its fastest shape, on 1M x 1M matrices with 16M entries:
    uniform rows of 16 random columns (the same gathers without any
    irregularity), the power-law matrix of the headline, the same law on 10 % or 1 % of the
    rows with the others empty (scattered), and one run of 900k empty rows
    before 100k rows of 160 entries. Prints one JSON line per matrix."""
    import torch
    from paper_1803_08601_amd import native as nv
    from paper_1803_08601_amd import workloads as wl
    M = 1_000_000
    rng = np.random.default_rng(1006)
    cases = [("uniform rows of 16 (no irregularity)", "uniform"),
             ("power law, no empty rows", None), ("power law on 10% of rows, rest empty", 0.10),
             ("power law on 1% of rows, rest empty", 0.01),
             ("900k empty rows, then 100k rows of 160", "run")]
    recs = []
    for desc, frac in cases:
        if frac is None:
            A = wl.power_law(seed=1002)
            rowptr, colind = A.rowptr, A.colind
        else:
            lengths = np.zeros(M, np.int64)
            if frac == "uniform":
                lengths[:] = 16
            elif frac == "run":
                lengths[900_000:] = 160
            else:
                rows = np.sort(rng.choice(M, int(M * frac), replace=False))
                lens, _ = wl.power_law_lengths(rng, rows.shape[0], mean=16.0 / frac, cap=100_000)
                lengths[rows] = lens
            colind = wl.distinct_sorted_columns(rng, lengths, M)
            rowptr = wl.rowptr_from_lengths(lengths)
        nnz = int(rowptr[-1])
        rp = torch.from_numpy(rowptr).cuda()
        ci = torch.from_numpy(colind).cuda()
        g = torch.Generator(device="cuda")
        g.manual_seed(13)
        vals = torch.rand(nnz, generator=g, device="cuda") - 0.5
        Bt = torch.rand(M, n, generator=g, device="cuda") - 0.5
        C = torch.empty(M, n, device="cuda")
        rec = {"matrix": desc, "m": M, "nnz": nnz, "n": n,
               "empty_rows": int(np.count_nonzero(np.diff(rowptr) == 0))}
        for kern in ("rowsplit", "merge", "nzsplit"):
            best = _best_of(nv, rp, ci, M, M, nnz, n, vals, Bt, C, kern)
            rec[f"{kern}_ms"] = round(best[0], 4)
            rec[f"{kern}_shape"] = best[1]
        plan = nv.Plan(rp, ci, M, M, n, nnz=nnz, mode="autotune")
        rec["autotune_kernel"] = nv.KERNEL_NAMES[plan.info().config.kernel]
        plan.close()
        print(json.dumps(rec), flush=True)
        recs.append(rec)
        del rp, ci, vals, Bt, C
        torch.cuda.empty_cache()
    return recs


def table_size_sweep(n=64):
    """Where the gather time comes from: the same 16M power-law entries
    (1M rows, mean 16) against B tables of 1M, 500k, 250k, 64k and 16k rows
    (256 MB down to 4 MB at n = 64), each merge-walk kernel at W = 2048,
    U = 2. A table that fits one XCD's 4 MB L2 shows the on-chip gather rate;
    the larger ones show whether the 256 MB MALL changes it."""
    import torch
    from paper_1803_08601_amd import native as nv
    from paper_1803_08601_amd import workloads as wl
    rng = np.random.default_rng(5)
    M = 1_000_000
    lengths, _ = wl.power_law_lengths(rng, M, mean=16.0, cap=16_000)
    rp = torch.from_numpy(wl.rowptr_from_lengths(lengths)).cuda()
    nnz = int(lengths.sum())
    C = torch.empty(M, n, device="cuda")
    recs = []
    for k in (1_000_000, 500_000, 250_000, 64_000, 16_000):
        ci = torch.from_numpy(wl.distinct_sorted_columns(rng, lengths, k)).cuda()
        vals = torch.rand(nnz, device="cuda")
        B = torch.rand(k, n, device="cuda")
        rec = {"k": k, "B_MB": round(k * n * 4 / 1e6, 1), "nnz": nnz, "n": n}
        for name, code in (("merge_ms", nv.SPMM_KERNEL_MERGE), ("nzsplit_ms", nv.SPMM_KERNEL_NZSPLIT)):
            ms, _ = _plan_time(nv, rp, ci, M, k, nnz, n, vals, B, C,
                               cfg=dict(kernel=code, items_per_wg=2048, unroll=2), steps=20)
            rec[name] = round(ms, 4)
        rec["gather_TBs"] = round(nnz * n * 4 / (min(rec["merge_ms"], rec["nzsplit_ms"]) * 1e-3) / 1e12, 2)
        print(json.dumps(rec), flush=True)
        recs.append(rec)
        del ci, vals, B
        torch.cuda.empty_cache()
    return recs


def gather_ceiling():
    """The device's rate for the products' access to B alone: lanes read
    rows of 32, 64, 128, 256 and 512 bytes (n = 8, 16, 32, 64 and 128 in
    float32; 128 bytes is also n = 64 in bfloat16; 16 bytes a lane, eight
    rows in flight per lane group) at pseudo-random indices of a
    table of 16 KB (one CU's L1), 2 MB (within an XCD's 4 MB L2), 64 MB and
    256 MB (within and at the size of the 256 MB MALL), with no reads of A and
    no writes of C (the library's gather calibration kernel, 524,288 lanes,
    512 rows each, mean of 5 launches timed with events)."""
    import torch
    from paper_1803_08601_amd import native as nv
    threads, steps = 2048 * 256, 512
    table = torch.rand(64 << 20, device="cuda")  # 256 MB
    out = torch.empty(threads, device="cuda")
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    recs = []
    for row_bytes in (32, 64, 128, 256, 512):
        for table_bytes in (16 << 10, 2 << 20, 64 << 20, 256 << 20):
            rows = table_bytes // row_bytes
            for _ in range(2):
                nv.spmm_calibrate_gather(table, rows, row_bytes, steps, out, threads, st.cuda_stream)
            e0.record(st)
            for _ in range(5):
                nv.spmm_calibrate_gather(table, rows, row_bytes, steps, out, threads, st.cuda_stream)
            e1.record(st)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / 5
            nbytes = threads * steps * 16
            rec = {"row_bytes": row_bytes, "table_MB": round(table_bytes / 2**20, 3),
                   "ms": round(ms, 4), "TBs": round(nbytes / (ms * 1e-3) / 1e12, 2),
                   "G_rows_per_s": round(nbytes / row_bytes / (ms * 1e-3) / 1e9, 1),
                   "B_per_clk_per_CU": round(nbytes / (ms * 1e-3) / (256 * 2.4e9), 1)}
            print(json.dumps(rec), flush=True)
            recs.append(rec)
    return recs


def live_gather_ceiling(row_bytes, table_bytes):
    """The gather calibration kernel's rate (rows/s) for rows of row_bytes
    from a table of about table_bytes (the power of two of rows nearest in
    log scale), or None for a row size it does not take."""
    import math
    import torch
    from paper_1803_08601_amd import native as nv
    if row_bytes not in (32, 64, 128, 256, 512):
        return None
    rows = 1 << max(0, round(math.log2(max(1, table_bytes // row_bytes))))
    threads, steps = 2048 * 256, 512
    table = torch.rand(rows * row_bytes // 4, device="cuda")
    out = torch.empty(threads, device="cuda")
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        nv.spmm_calibrate_gather(table, rows, row_bytes, steps, out, threads, st.cuda_stream)
    e0.record(st)
    for _ in range(5):
        nv.spmm_calibrate_gather(table, rows, row_bytes, steps, out, threads, st.cuda_stream)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del table, out
    torch.cuda.empty_cache()
    return {"rows_per_s": threads * steps * 16 / row_bytes / (ms * 1e-3), "row_bytes": row_bytes,
            "table_bytes": rows * row_bytes}


def crossover(n=64, densities=(0.001, 0.0025, 0.005, 0.01, 0.02, 0.05, 0.1), panels=(4, 8, 16)):
    """Sparse versus dense (Fig. 7): a 100k x 100k matrix with a fixed share
    of distinct random columns in every row times a 100k x 64 B, SpMM (plan by
    timing, whose candidates include column panels) against the dense product
    of the same matrix stored densely (torch.mm, i.e. the vendor BLAS), in
    float32 and bfloat16. From 1 % density on, also the 2-D tiling question
    of Sec. 6 directly: row split without panels against P column panels
    (float32, one row-split pass per panel adding into C), B's panel slice
    then fitting one XCD's L2."""
    import torch
    from paper_1803_08601_amd import native as nv
    from paper_1803_08601_amd import workloads as wl
    N = 100_000
    recs = []
    for rho in densities:
        rp, ci, vals, L = wl.fixed_density_device(11, N, rho)
        nnz = N * L
        g = torch.Generator(device="cuda")
        g.manual_seed(12)
        Bt = torch.rand(N, n, generator=g, device="cuda") - 0.5
        C = torch.empty(N, n, device="cuda")
        rec = {"density": rho, "nnz": nnz, "n": n}
        for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
            v, b = vals.to(dt), Bt.to(dt)
            plan = nv.Plan(rp, ci, N, N, n, dtype=nv.dtype_code(dt), mode="autotune", nnz=nnz)
            rec[f"spmm_{name}_ms"] = round(_timed(lambda: plan.execute(v, b, C), 10, 2), 4)
            rec[f"spmm_{name}_kernel"] = nv.KERNEL_NAMES[plan.info().config.kernel]
            rec[f"spmm_{name}_panels"] = plan.info().config.col_panels
            plan.close()
            D = torch.zeros(N, N, dtype=dt, device="cuda")
            rows = torch.arange(N, device="cuda").repeat_interleave(L)
            D[rows, ci.long()] = v
            del rows
            rec[f"dense_{name}_ms"] = round(_timed(lambda: torch.mm(D, b), 5, 1), 4)
            del D
            torch.cuda.empty_cache()
        if rho >= 0.01:
            # the best row split without panels (whole and half-width column
            # tiles) against each panel count
            for P in (1,) + tuple(panels):
                best = None
                shapes = [(lpr, u, tc) for lpr in (64, 32, 16) for u in (2, 4, 8)
                          for tc in (0, n // 2)] if P == 1 else \
                    [(lpr, u, 0) for lpr in (64, 32) for u in (2, 4, 8)]
                for lpr, u, tc in shapes:
                    cfg = dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, lanes_per_row=lpr, unroll=u,
                               tile_cols=tc, col_panels=P)
                    plan = nv.Plan(rp, ci, N, N, n, nnz=nnz, config=cfg)
                    ms = _timed(lambda: plan.execute(vals, Bt, C), 10, 2)
                    plan.close()
                    best = ms if best is None else min(best, ms)
                rec["rowsplit_f32_ms" if P == 1 else f"panels{P}_f32_ms"] = round(best, 4)
            torch.cuda.empty_cache()
        print(json.dumps(rec), flush=True)
        recs.append(rec)
        del rp, ci, vals, Bt, C
        torch.cuda.empty_cache()
    return recs


def host_cpu():
    """CPU model, sockets, cores per socket and threads per core of this
    host (lscpu), and the threads this process may run on."""
    info = {"model": "", "sockets": None, "cores_per_socket": None, "threads_per_core": None}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            key, _, val = ln.partition(":")
            key, val = key.strip(), val.strip()
            if key == "Model name":
                info["model"] = val
            elif key == "Socket(s)":
                info["sockets"] = int(val)
            elif key == "Core(s) per socket":
                info["cores_per_socket"] = int(val)
            elif key == "Thread(s) per core":
                info["threads_per_core"] = int(val)
    except (OSError, ValueError):
        pass
    info["affinity_threads"] = len(os.sched_getaffinity(0))
    return info


def cpu_baseline(A, B, n, budget_s=10.0, max_reps=8):
    """The FP64 oracle on this host's cores: an -O3 -march=native build of
    oracle/spmm_oracle.c made here (bitwise the pinned test build), over the
    full workload - OpenMP over rows on every allowed thread (median of up to
    `max_reps` passes within `budget_s`) and one pass on one thread."""
    import tempfile
    import numpy as np
    import oracle
    threads = len(os.sched_getaffinity(0))
    build = "-O3 -march=native -ffp-contract=off, built on this host"
    try:
        lib = oracle.native_build(os.path.join(tempfile.mkdtemp(), "liboracle_native.so"))
    except Exception as e:  # no compiler on the host: the test build
        lib, build = None, f"test build -O2 (native build failed: {e})"
    times = []
    t_start = time.perf_counter()
    while len(times) < max_reps and (time.perf_counter() - t_start < budget_s or len(times) < 2):
        t0 = time.perf_counter()
        oracle.spmm(A.rowptr, A.colind, A.vals, B, n=n, nthreads=threads, library=lib)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    t0 = time.perf_counter()
    oracle.spmm(A.rowptr, A.colind, A.vals, B, n=n, nthreads=1, library=lib)
    t1 = time.perf_counter() - t0
    return {"value": 2.0 * A.nnz * n / t / 1e9, "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"full workload, {len(times)} passes of the FP64 oracle (OpenMP over rows, "
                      f"{threads} threads), median {t * 1e3:.1f} ms per pass; {build}",
            "one_thread": {"value": round(2.0 * A.nnz * n / t1 / 1e9, 3), "unit": "GFLOP/s",
                           "sample": f"full workload, one pass on one thread, {t1:.2f} s"},
            "host": host_cpu()}


# ---------------------------------------------------------------- counter records

ROW_FAMILIES = [  # (profile file, title, row-key prefix)
    ("spmm_powerlaw_1M.md", "Power-law 1M x 1M, mean 16 (k_merge / k_rowsplit)", "powerlaw-"),
    ("spmm_stencil27_128cube.md", "27-point stencil on 128^3 (k_rowsplit / k_rowblock)", "stencil-"),
    ("spmm_uniform_4096.md", "Uniform 4096 x 4096, 16 per row (launch-bound size)", "plain-"),
    ("gcn_500k_n128_fwd_dB_dvals.md", "GCN adjacency 500k nodes, n = 128: forward, dB, dvals",
     "gcn-"),
    ("batch_512_problems.md", "512 uneven products in one persistent launch (k_batch)", "batch-"),
]


def read_counter_csv(d):
    """Dispatches of a rocprofv3 counter run (every *counter_collection.csv
    under d) in dispatch order: [(kernel name, {counter: value})]."""
    import csv
    disp = {}
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                key = (f, int(r["Dispatch_Id"]))
                name, ctrs = disp.setdefault(key, (r["Kernel_Name"], {}))
                ctrs[r["Counter_Name"]] = ctrs.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [disp[k] for k in sorted(disp)]


def read_kernel_stats(d):
    """Rows of every *kernel_stats.csv under d: name -> (calls, average us,
    min us, max us)."""
    import csv
    out = {}
    for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                out[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                                  float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3)
    return out


def last_dispatches(disps, pattern, count):
    """The last `count` dispatches whose kernel name matches `pattern`."""
    rx = re.compile(pattern)
    hit = [c for name, c in disps if rx.search(name)]
    if len(hit) < count:
        raise SystemExit(f"record-counters: {len(hit)} dispatches match {pattern!r}, need {count}")
    return hit[-count:]


def mean_counter(dispatches, name):
    """Mean of one counter over the dispatches (None if the pass lacks it)."""
    if not dispatches or any(name not in c for c in dispatches):
        return None
    return float(np.mean([c[name] for c in dispatches]))


def copy_scale(d, name, bytes_per_copy):
    """Counter reading of the plain 1 GiB device copy: bytes moved divided by
    what `name` reports for one copy (median over its dispatches)."""
    disps = read_counter_csv(d)
    names = [n for n, _ in disps]
    top = max(set(names), key=names.count)
    vals = [c[name] for n, c in disps if n == top]
    return bytes_per_copy / (float(np.median(vals)) * 1024.0), top


def record_counters(run_dir, profiles=os.path.join(ROOT, "profiles")):
    """Turn the rocprofv3 runs under run_dir into counter records
    (profiles/hbm_counters.json) and one summary per workload family.
    Layout: run_dir/tune.txt: the autotuner's choices every pass loads and
    extends (seeded with profiles/bench_tune_cache.txt);
    run_dir/copy/{fetch,write}: `bench.py --copy-calibration` under
    `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE`; run_dir/<row>/: manifest.json
    and cmd.txt (the bench arguments) written by the profiled run,
    fetch/, write/, l2/ (--pmc TCC_HIT_sum TCC_MISS_sum TA_TA_BUSY_sum
    GRBM_GUI_ACTIVE) and trace/ (--kernel-trace --stats)."""
    copy_bytes = 256 * 1024 * 1024 * 4
    fs, fk = copy_scale(os.path.join(run_dir, "copy", "fetch"), "FETCH_SIZE", copy_bytes)
    ws, _ = copy_scale(os.path.join(run_dir, "copy", "write"), "WRITE_SIZE", copy_bytes)
    path = os.path.join(profiles, "hbm_counters.json")
    records = json.load(open(path)) if os.path.exists(path) else {}
    sha = kernel_source_hash()
    rows = []
    for mf in sorted(glob.glob(os.path.join(run_dir, "*", "manifest.json"))):
        rdir = os.path.dirname(mf)
        args = open(os.path.join(rdir, "cmd.txt")).read().strip()
        # the counter passes plan again (by timing): each must have picked
        # the shapes of the traced run, or its counters describe other kernels
        for sub in ("fetch", "write", "l2"):
            smf = os.path.join(rdir, sub + ".manifest.json")
            if os.path.exists(smf):
                got = [(x["row"], x["config"]) for x in json.load(open(smf))]
                want = [(x["row"], x["config"]) for x in json.load(open(mf))]
                if got != want:
                    raise SystemExit(f"record-counters: {rdir}/{sub} planned {got}, "
                                     f"the traced run {want}")
        fetch = read_counter_csv(os.path.join(rdir, "fetch"))
        write = read_counter_csv(os.path.join(rdir, "write"))
        l2 = read_counter_csv(os.path.join(rdir, "l2"))
        l2_names = " ".join(sorted({c for _, cs in l2 for c in cs}))
        stats = read_kernel_stats(os.path.join(rdir, "trace"))
        for m in json.load(open(mf)):
            k = m["steps"]
            per = []
            for pat in m["patterns"]:
                f_d = last_dispatches(fetch, pat, k)
                w_d = last_dispatches(write, pat, k)
                l_d = last_dispatches(l2, pat, k)
                rx = re.compile(pat)
                names = sorted(n for n in stats if rx.search(n))
                per.append({"pattern": pat, "kernels": names,
                            "trace_avg_us": [round(stats[n][1], 1) for n in names],
                            "fetch_kib": mean_counter(f_d, "FETCH_SIZE"),
                            "write_kib": mean_counter(w_d, "WRITE_SIZE"),
                            "hit": mean_counter(l_d, "TCC_HIT_sum"),
                            "miss": mean_counter(l_d, "TCC_MISS_sum"),
                            "ta": mean_counter(l_d, "TA_TA_BUSY_sum"),
                            "gui": mean_counter(l_d, "GRBM_GUI_ACTIVE")})
            fk_ = sum(p["fetch_kib"] for p in per)
            wk_ = sum(p["write_kib"] for p in per)
            traffic = fk_ * 1024.0 * fs + wk_ * 1024.0 * ws
            hits, miss = sum(p["hit"] for p in per), sum(p["miss"] for p in per)
            main = per[0] if "gather_widen" not in per[0]["pattern"] else per[1]
            # TA busy: TA_TA_BUSY_sum over 256 TAs against GRBM_GUI_ACTIVE over
            # 8 XCDs (the fraction of the kernel's cycles each TA was busy)
            ta = (main["ta"] / 256.0 / (main["gui"] / 8.0)
                  if main["ta"] is not None and main["gui"] else None)
            fam = next(f for f in ROW_FAMILIES if m["row"].startswith(f[2]))
            rec = {"config": m["config"], "kernel_source_sha": sha, "fetch_kib": fk_,
                   "write_kib": wk_, "fetch_scale": fs, "write_scale": ws,
                   "traffic_bytes": traffic,
                   "l2_hit_rate": round(hits / (hits + miss), 4) if hits + miss else None,
                   "ta_busy": None if ta is None else round(ta, 3),
                   "bytes_min": m["bytes_min"], "bytes_gather": m["bytes_gather"],
                   "kernel_ms_cold_mean": m["kernel_ms_cold_mean"], "profile": fam[0]}
            # records taken on other kernel sources describe other kernels: dropped
            lst = [r for r in records.get(m["row"], [])
                   if r.get("config") != m["config"] and r.get("kernel_source_sha") == sha]
            records[m["row"]] = [rec] + lst
            rows.append((fam, m, rec, per, (args, l2_names), stats))
    with open(path, "w") as fh:
        json.dump(records, fh, indent=1, sort_keys=True)
        fh.write("\n")
    # the traced runs' autotuner choices, one line per matrix key (the bench
    # loads them, so its rows plan the shapes recorded here)
    lines, header = {}, None
    for tf in sorted(glob.glob(os.path.join(run_dir, "*", "tune.txt")) +
                     glob.glob(os.path.join(run_dir, "tune.txt"))):
        rows_ = open(tf).read().splitlines()
        if not rows_:
            continue
        header = rows_[0]
        for ln in rows_[1:]:
            f_ = ln.split()
            if f_:
                lines[tuple(f_[:13])] = ln
    if header is not None:
        with open(os.path.join(profiles, "bench_tune_cache.txt"), "w") as fh:
            fh.write(header + "\n" + "\n".join(lines[k_] for k_ in sorted(lines)) + "\n")
    rp = "rocprofv3"
    for fam in ROW_FAMILIES:
        mine = [r for r in rows if r[0] is fam]
        if not mine:
            continue
        L = [f"# {fam[1]}", "",
             "Counters per row of `bench.py` (rocprofv3, one MI355X). Traffic = FETCH_SIZE and "
             "WRITE_SIZE per dispatch of the row's kernels over its last `steps` dispatches (the "
             "cold-cache steps), scaled by the same counters on a plain 1 GiB copy; it is measured "
             "between the L2 caches and the fabric, so it includes Infinity Cache hits. Bytes_min: "
             "A, B and C moved once; gather model: every entry fetching its B row.", "",
             "Commands (repository root):", "", "```",
             "cp profiles/bench_tune_cache.txt <run>/tune.txt"]
        for a_, l2n in sorted({r[4] for r in mine}):
            tc = "--tune-cache <run>/tune.txt"
            L += [f"{rp} --kernel-trace --stats --output-format csv -d <run>/<row>/trace -o r -- "
                  f"python3 bench.py {a_} {tc} --manifest <run>/<row>/manifest.json",
                  f"{rp} --pmc FETCH_SIZE --output-format csv -d <run>/<row>/fetch -o r -- "
                  f"python3 bench.py {a_} {tc} --manifest <run>/<row>/fetch.manifest.json",
                  f"{rp} --pmc WRITE_SIZE --output-format csv -d <run>/<row>/write -o r -- "
                  f"python3 bench.py {a_} {tc} --manifest <run>/<row>/write.manifest.json",
                  f"{rp} --pmc {l2n} "
                  f"--output-format csv -d <run>/<row>/l2 -o r -- python3 bench.py {a_} {tc} "
                  f"--manifest <run>/<row>/l2.manifest.json"]
        L += [f"{rp} --pmc FETCH_SIZE --output-format csv -d <run>/copy/fetch -o c -- "
              "python3 bench.py --copy-calibration",
              f"{rp} --pmc WRITE_SIZE --output-format csv -d <run>/copy/write -o c -- "
              "python3 bench.py --copy-calibration",
              "python3 bench.py --record-counters <run>", "```", "",
              f"Copy calibration (`{fk[:60]}`): FETCH_SIZE scale {fs:.4f}, WRITE_SIZE scale "
              f"{ws:.4f}. Kernel sources hash `{sha}`.", "",
              "| row | shape | cold ms (events) | FETCH KiB | WRITE KiB | traffic GB | "
              "Bytes_min GB | traffic / Bytes_min | gather model GB | L2 hit | TA busy |",
              "|---|---|---|---|---|---|---|---|---|---|---|"]
        for _, m, rec, per, _, _ in mine:
            L.append(f"| {m['row']} | `{json.dumps(m['config'])}` | {m['kernel_ms_cold_mean']} | "
                     f"{rec['fetch_kib']:.0f} | {rec['write_kib']:.0f} | "
                     f"{rec['traffic_bytes'] / 1e9:.3f} | {m['bytes_min'] / 1e9:.3f} | "
                     f"{rec['traffic_bytes'] / m['bytes_min']:.2f} | {m['bytes_gather'] / 1e9:.3f}"
                     f" | {rec['l2_hit_rate']} | {rec['ta_busy']} |")
        L += ["", "Kernels of each row (kernel trace of the same command; average over every "
              "dispatch of that name, autotuning candidates included):", "",
              "| row | kernel | calls | avg us | min us | max us | FETCH KiB / dispatch | "
              "WRITE KiB / dispatch |", "|---|---|---|---|---|---|---|---|"]
        for _, m, rec, per, _, stats in mine:
            for p_ in per:
                for nm in p_["kernels"]:
                    c, av, mn, mx = stats[nm]
                    L.append(f"| {m['row']} | `{nm[:110]}` | {c} | {av:.1f} | {mn:.1f} | "
                             f"{mx:.1f} | {p_['fetch_kib']:.0f} | {p_['write_kib']:.0f} |")
        with open(os.path.join(profiles, fam[0]), "w") as fh:
            fh.write("\n".join(L) + "\n")
    return records


def write_summary(path, title, about, recs):
    """Markdown record of a sweep: what it measures, the command that made
    it (this process's arguments, run from the repository root on one
    MI355X) and one table row per record (nested values as JSON)."""
    keys = []
    for r in recs:
        for k_ in r:
            if k_ not in keys:
                keys.append(k_)

    def cell(v):
        if isinstance(v, (dict, list)):
            return "`" + json.dumps(v, separators=(",", ":")) + "`"
        return "" if v is None else str(v)
    args = [a for a in sys.argv[1:]]
    L = [f"# {title}", "", about, "", "Command (repository root, one MI355X):", "", "```",
         "python3 bench.py " + " ".join(args), "```", "",
         "| " + " | ".join(keys) + " |", "|" + "---|" * len(keys)]
    for r in recs:
        L.append("| " + " | ".join(cell(r.get(k_)) for k_ in keys) + " |")
    with open(path, "w") as fh:
        fh.write("\n".join(L) + "\n")


ROWS = ["plain-n32-f32", "powerlaw-n8-f32", "powerlaw-n64-bf16", "stencil-n16-f32",
        "stencil-n128-f32"] + [f"gcn-{d}-{p}" for d in ("f32", "bf16") for p in ("fwd", "dB", "dvals")] \
    + ["batch-f32", "batch-bf16"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="powerlaw", choices=["powerlaw", "stencil", "plain"])
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--mode", default="autotune",
                    choices=["autotune", "paper", "rowsplit", "merge", "nzsplit", "rule",
                             "rowblock"])
    ap.add_argument("--config", default=None,
                    help="force a kernel shape, JSON of spmm_config fields, e.g. "
                         "'{\"kernel\": 1, \"items_per_wg\": 2048, \"unroll\": 2}'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="only the headline product (skip the other rows)")
    ap.add_argument("--row", choices=ROWS,
                    help="time just this row of the extra measurements and print its JSON")
    ap.add_argument("--manifest", default=None,
                    help="write the timed rows' kernels and byte counts here (for profiling)")
    ap.add_argument("--record-counters", default=None, metavar="RUN_DIR",
                    help="turn rocprofv3 runs under RUN_DIR into profiles/ records and summaries")
    ap.add_argument("--sweep", action="store_true",
                    help="kernel-choice sweep over mean row length (re-derives the Sec. 5.4 threshold)")
    ap.add_argument("--rowblock-sweep", action="store_true",
                    help="row blocks against row split and merge on stencils and controls")
    ap.add_argument("--nzsplit", action="store_true",
                    help="nonzero split against merge path and row split on matrices with "
                         "runs of empty rows")
    ap.add_argument("--table-size-sweep", action="store_true",
                    help="the same entries against B tables from 256 MB down to 4 MB")
    ap.add_argument("--gather-ceiling", action="store_true",
                    help="the device's rate for random row gathers alone, by row and table size")
    ap.add_argument("--crossover", action="store_true",
                    help="sparse versus dense product over density (100k x 100k, n = 64)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--retune", action="store_true",
                    help="time the autotuner's candidates afresh instead of loading the "
                         "choices kept in profiles/bench_tune_cache.txt")
    ap.add_argument("--summary", default=None, metavar="FILE",
                    help="with a sweep mode: also write its records as a markdown table")
    ap.add_argument("--tune-cache", default=None, metavar="FILE",
                    help="load the autotuner's choices from FILE if it exists and save them "
                         "there at exit (profiling passes then plan the shapes the traced "
                         "run timed)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library and this benchmark use one GPU; --gpus {args.gpus} is not "
              "supported (multi-GPU sharding is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.record_counters:
        record_counters(args.record_counters)
        return

    import torch
    from paper_1803_08601_amd import native as nv

    if args.tune_cache:
        import atexit
        if os.path.exists(args.tune_cache):
            nv.spmm_tune_cache_load(args.tune_cache)
        atexit.register(nv.spmm_tune_cache_save, args.tune_cache)
    elif not args.retune and os.path.exists(BENCH_TUNE_CACHE):
        nv.spmm_tune_cache_load(BENCH_TUNE_CACHE)
    manifest = [] if args.manifest else None

    def write_manifest():
        if manifest is not None:
            with open(args.manifest, "w") as fh:
                json.dump(manifest, fh, indent=1)

    def summarise(recs, title, about):
        if args.summary:
            write_summary(args.summary, title, about, recs)

    if args.sweep:
        summarise(heuristic_sweep(args.n), "Kernel choice over row-length regimes (Sec. 5.4)",
                  heuristic_sweep.__doc__.strip().replace("\n    ", " "))
        return
    records = load_counters()
    if args.row:
        r = args.row
        if r.startswith("gcn-"):
            rec = gcn_fwd_bwd(records, args.steps, args.warmup, only=r[4:], manifest=manifest)
        elif r.startswith("batch-"):
            rec = batched(records, args.steps, args.warmup, only=r[6:], manifest=manifest)
        else:
            rec = other_configs(None, records, args.steps, args.warmup, only=r, manifest=manifest)
        write_manifest()
        print(json.dumps(rec), flush=True)
        return
    if args.crossover:
        summarise(crossover(args.n), "Sparse versus dense, and column panels (Fig. 7, Sec. 6)",
                  crossover.__doc__.strip().replace("\n    ", " "))
        return
    if args.nzsplit:
        summarise(nz_compare(args.n), "Nonzero split against the merge-path split",
                  nz_compare.__doc__.strip().replace("\n    ", " "))
        return
    if args.rowblock_sweep:
        summarise(rowblock_sweep(), "Row blocks against row split and merge path",
                  rowblock_sweep.__doc__.strip().replace("\n    ", " "))
        return
    if args.gather_ceiling:
        summarise(gather_ceiling(), "Random row gathers alone: the ceiling of the B access",
                  gather_ceiling.__doc__.strip().replace("\n    ", " "))
        return
    if args.table_size_sweep:
        summarise(table_size_sweep(args.n), "Gather rate against the size of B",
                  table_size_sweep.__doc__.strip().replace("\n    ", " "))
        return
    if args.copy_calibration:
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / 20
        # a streaming device copy: the practical HBM rate (read + write)
        print(json.dumps({"copy_bytes_per_dispatch": a.numel() * 4,
                          "copy_ms": round(t * 1e3, 4),
                          "copy_read_write_GBs": round(2 * a.numel() * 4 / t / 1e9, 1)}))
        return

    dt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[args.dtype]
    A, B, desc = make_workload(args.workload, args.n)
    n = args.n
    cfg = json.loads(args.config) if args.config else None
    key = f"{args.workload}-n{n}-{args.dtype}"
    row, info, t = single_product(A, B, n, dt, mode=args.mode, cfg=cfg, steps=args.steps,
                                  warmup=args.warmup, key=key, records=records,
                                  manifest=manifest)
    write_manifest()
    flops = 2.0 * A.nnz * n
    ms = float(np.mean(t["cold_step"]))
    kavg = float(np.mean(t["cold_kernel"]))
    bmin = row["bytes_min"]
    achieved = bmin / (kavg * 1e-3) / 1e9
    out = {
        "metric": "SpMM GFLOP/s (2*nnz*n/t)",
        "value": round(flops / (ms * 1e-3) / 1e9, 2),
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
        "timing": "cold caches: 1 GiB written before each timed step (outside its hipEvents) "
                  "evicts L2 and the Infinity Cache; a step is the whole product (main kernel "
                  "and, for merge-based plans, the fix-up), timed by hipEvents around it",
        "config": {"workload": desc, "m": A.m, "k": A.k, "nnz": A.nnz, "n": n,
                   "kernel": row["kernel"], "mode": "config" if cfg else args.mode,
                   "shape": row["shape"], "paper_rule_kernel": row["paper_rule_kernel"],
                   "plan_build_s": row["plan_build_s"], "input_sha": A.digest(),
                   "tile_order": row["tile_order"]},
        "kernel_ms": row["kernel_ms"],
        "step_ms": {"cold": spread(t["cold_step"]), "cold_wall_incl_scrub": round(t["cold_wall"], 4)},
        "warm": {"value": row["warm"]["gflops"], "ms_per_step": row["warm"]["ms_per_step"],
                 "timing": "steps back to back, wall clock between two synchronisations"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": row["traffic"],
                     "traffic_GBs": row["traffic_GBs"],
                     "traffic_over_bytes_min": row["traffic_over_bytes_min"],
                     "traffic_source": TRAFFIC_SOURCE,
                     "counter_profile": row["counter_profile"],
                     "l2_hit_rate": row["l2_hit_rate"],
                     "kernel": {"rowsplit": "k_rowsplit", "rowblock": "k_rowblock"}.get(
                         row["kernel"], "k_merge"),
                     "kernel_ms": round(kavg, 4), "algorithmic_bytes": bmin,
                     "gather_model": {"bytes": row["gather_model_bytes"],
                                      "achieved": round(row["gather_model_bytes"] / (kavg * 1e-3)
                                                        / 1e9, 1),
                                      "frac": row["gather_model_frac"]}},
    }
    if not args.quick:
        # the same kernel against the measured ceiling of its access to B:
        # random rows of B's row size from a table of B's size, nothing else
        eb = {"f32": 4, "bf16": 2, "f16": 2}[args.dtype]
        ceil = live_gather_ceiling(n * eb, A.k * n * eb)
        if ceil:
            got = A.nnz / (kavg * 1e-3)
            out["roofline"]["gather_ceiling"] = {
                "achieved_rows_per_s": round(got / 1e9, 2), "ceiling_rows_per_s":
                round(ceil["rows_per_s"] / 1e9, 2), "unit": "G rows/s",
                "frac": round(got / ceil["rows_per_s"], 4), "row_bytes": ceil["row_bytes"],
                "table_bytes": ceil["table_bytes"],
                "source": "spmm_calibrate_gather measured in this run: random rows of B's row "
                          "size read from a table of about B's size, with no reads of A and "
                          "no writes of C"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, n)
    if not args.quick:
        torch.cuda.empty_cache()
        out["extra"] = {"other_configs": other_configs(A if args.workload == "powerlaw" else None,
                                                       records),
                        "gcn_fwd_bwd": gcn_fwd_bwd(records), "batched": batched(records)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
