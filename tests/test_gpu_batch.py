"""Batched SpMM on the GPU: one persistent launch for many uneven problems,
captured in a hipGraph. Each problem's result must equal, bit for bit, the
same plan run alone (same kernel shape, same summation order) and match the
FP64 oracle."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import DT, TOL_F32, dev, oracle_product, rel_err

pytestmark = pytest.mark.gpu


def build_batch(count, dtype, seed=1005, m_hi=6000, n_choices=(8, 32, 128), extra=()):
    specs = wl.batch_specs(seed=seed, count=count, m_lo=200, m_hi=m_hi, n_choices=n_choices)
    items = []
    for b, (m, n, kind) in enumerate(specs):
        A = wl.batch_problem(seed, b, m, kind)
        items.append((A, n))
    items.extend(extra)
    keep = []
    probs = []
    for b, (A, n) in enumerate(items):
        B = wl.dense(seed + b, A.k, n)
        rp, ci = dev(A.rowptr), dev(A.colind)
        vt, Bt = dev(A.vals, DT[dtype]), dev(B, DT[dtype])
        C = torch.full((A.m, n), float("nan"), device="cuda")
        keep.append((A, n, rp, ci, vt, Bt, C))
        probs.append(nv.spmm_problem(rp.data_ptr(), ci.data_ptr(), vt.data_ptr(), Bt.data_ptr(),
                                     C.data_ptr(), A.m, A.k, A.nnz, n, n))
    return keep, probs


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("mode", ["paper", "autotune", "merge", "rowsplit", "nzsplit"])
def test_batch_graph_matches_solo_and_oracle(dtype, mode):
    # one mostly empty matrix: nonzero-split pieces with more row ends than W
    sparse = wl.random_csr(23, 20_000, 3_000, density=0.003, empty_frac=0.9)
    keep, probs = build_batch(40, dtype, extra=[(sparse, 32)])
    h = nv.spmm_batch_plan(probs, nv.dtype_code(DT[dtype]), nv.MODES[mode])
    try:
        for C in (k[6] for k in keep):
            C.fill_(float("nan"))
        nv.spmm_batch_run(h)
        torch.cuda.synchronize()
        kinds = set()
        for b, (A, n, rp, ci, vt, Bt, C) in enumerate(keep):
            cfg = nv.spmm_batch_problem_config(h, b)
            kinds.add(cfg.kernel)
            solo = nv.Plan(rp, ci, A.m, A.k, n, dtype=nv.dtype_code(DT[dtype]), config=cfg,
                           nnz=A.nnz)
            Cs = torch.empty_like(C)
            solo.execute(vt, Bt, Cs)
            torch.cuda.synchronize()
            assert torch.equal(C, Cs), f"problem {b} differs from its solo run"
            Cref, N = oracle_product(A.rowptr, A.colind, vt, Bt, n)
            assert rel_err(C.cpu().numpy(), Cref, N) <= TOL_F32, f"problem {b}"
        if mode == "merge":
            assert kinds == {nv.SPMM_KERNEL_MERGE}
        if mode == "rowsplit":
            assert kinds == {nv.SPMM_KERNEL_ROWSPLIT}
        if mode == "nzsplit":
            assert kinds == {nv.SPMM_KERNEL_NZSPLIT}
    finally:
        nv.spmm_batch_destroy(h)


def test_batch_replays_and_direct_run():
    keep, probs = build_batch(30, "f32", seed=77)
    h = nv.spmm_batch_plan(probs, nv.SPMM_F32, nv.SPMM_MODE_AUTOTUNE)
    try:
        nv.spmm_batch_run(h)
        torch.cuda.synchronize()
        first = [k[6].clone() for k in keep]
        for rep in range(4):
            for k in keep:
                k[6].fill_(-1.0)  # eager work between replays
            torch.cuda.synchronize()
            if rep % 2:
                nv.spmm_batch_run_direct(h)
            else:
                nv.spmm_batch_run(h)
            torch.cuda.synchronize()
            for a, k in zip(first, keep):
                assert torch.equal(a, k[6])
    finally:
        nv.spmm_batch_destroy(h)


def test_batch_degenerate_and_unaligned_problems():
    empty_rows = wl.random_csr(1, 300, 200, density=0.0)
    zero_m = wl.CSR(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), 0, 50)
    giant = wl.CSR(np.array([0, 0, 30_000, 30_001], np.int32),
                   np.concatenate([np.arange(30_000), [7]]).astype(np.int32),
                   np.random.default_rng(3).uniform(-1, 1, 30_001).astype(np.float32), 3, 30_000)
    extra = [(empty_rows, 32), (zero_m, 8), (giant, 64), (wl.random_csr(2, 500, 400, 0.05), 12)]
    keep, probs = build_batch(6, "f32", seed=11, extra=extra)
    # one problem with B and C offset by one float: element access inside the batch
    A, n = keep[-1][0], keep[-1][1]
    Bflat = torch.zeros(A.k * n + 1, device="cuda")
    Bflat[1:] = keep[-1][5].reshape(-1)
    Cflat = torch.zeros(A.m * n + 1, device="cuda")
    probs[-1].B = Bflat.data_ptr() + 4
    probs[-1].C = Cflat.data_ptr() + 4
    h = nv.spmm_batch_plan(probs, nv.SPMM_F32, nv.SPMM_MODE_MERGE)
    try:
        nv.spmm_batch_run(h)
        torch.cuda.synchronize()
        for b, (A, n, rp, ci, vt, Bt, C) in enumerate(keep):
            if A.m == 0:
                continue
            out = Cflat[1:].reshape(A.m, n) if b == len(keep) - 1 else C
            Cref, N = oracle_product(A.rowptr, A.colind, vt, Bt, n)
            assert rel_err(out.cpu().numpy(), Cref, N) <= TOL_F32, f"problem {b}"
    finally:
        nv.spmm_batch_destroy(h)


def test_batch_errors():
    keep, probs = build_batch(3, "f32", seed=5)
    probs[1].C = None
    with pytest.raises(nv.SpmmError):
        nv.spmm_batch_plan(probs, nv.SPMM_F32, nv.SPMM_MODE_PAPER)
    h = nv.spmm_batch_plan([], nv.SPMM_F32, nv.SPMM_MODE_PAPER)  # empty batch runs
    nv.spmm_batch_run(h)
    torch.cuda.synchronize()
    nv.spmm_batch_destroy(h)
    with pytest.raises(nv.SpmmError):
        nv.spmm_batch_destroy(h)
    with pytest.raises(nv.SpmmError):
        nv.spmm_batch_problem_config(ctypes.c_void_p(12345), 0)
