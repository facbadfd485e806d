"""Column panels (spmm_config.col_panels; the 2-D tiling of Sec. 6 with one
row tile): the product as P row-split passes, each over the entries of one
column panel and adding into C. Checked against the FP64 oracle elementwise
at the float32 tolerance, bitwise on integer-valued inputs (every partial
sum exact, whatever the order), with BF16 storage, padded rows, empty rows
and panels, the one pass of P = 1, and refusals."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import DT, TOL_F32, dev, oracle_product, rel_err

pytestmark = pytest.mark.gpu

MATS = {
    # rows of 1..400 sorted distinct columns over 5000 columns, a fifth empty
    "wide": lambda: wl.random_csr(21, 3000, 5000, density=0.04, empty_frac=0.2),
    "power_law": lambda: wl.power_law(seed=22, m=20_000, cap=8_000),
    # one row holding every column, the others short
    "full_row": lambda: wl.CSR(np.array([0, 7000, 7003, 7003], np.int32),
                               np.concatenate([np.arange(7000), [5, 6000, 6999]]).astype(np.int32),
                               np.random.default_rng(3).uniform(-1, 1, 7003).astype(np.float32),
                               3, 7000),
}


def run(A, vals_t, B_t, n, cfg, ld=None):
    ld = ld or n
    rp, ci = dev(A.rowptr), dev(A.colind)
    plan = nv.Plan(rp, ci, A.m, A.k, n, ld=ld, dtype=nv.dtype_code(vals_t.dtype), config=cfg,
                   nnz=A.nnz)
    C = torch.full((A.m, ld), float("nan"), device="cuda")
    plan.execute(vals_t, B_t, C)
    torch.cuda.synchronize()
    info = plan.info()
    plan.close()
    return C[:, :n].cpu().numpy(), info


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("P", [2, 3, 8, 64])
@pytest.mark.parametrize("n", [8, 64])
def test_panels_match_oracle(name, P, n):
    A = MATS[name]()
    B = wl.dense(5, A.k, n)
    vt, Bt = dev(A.vals), dev(B)
    cfg = dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=P, lanes_per_row=32, unroll=4)
    got, info = run(A, vt, Bt, n, cfg)
    assert info.config.col_panels == P
    ref, N = oracle_product(A.rowptr, A.colind, vt, Bt, n)
    assert rel_err(got, ref, N) <= TOL_F32


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_panels_integer_exact(name, dtype):
    A = MATS[name]()
    rng = np.random.default_rng(7)
    vals = rng.integers(-8, 9, A.nnz).astype(np.float32)
    n = 32
    B = rng.integers(-8, 9, (A.k, n)).astype(np.float32)
    vt, Bt = dev(vals, DT[dtype]), dev(B, DT[dtype])
    for P, lpr, u in ((5, 64, 8), (16, 16, 2)):
        cfg = dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=P, lanes_per_row=lpr, unroll=u)
        got, _ = run(A, vt, Bt, n, cfg)
        ref = oracle.spmm(A.rowptr, A.colind, vals, B)
        assert np.array_equal(got.astype(np.float64), ref)


def test_panels_padded_rows_and_one_panel():
    """ld > n (padding left untouched by the product's columns) and P = 1,
    which is plain row split (bitwise)."""
    A = MATS["wide"]()
    n, ld = 24, 40
    B = np.zeros((A.k, ld), np.float32)
    B[:, :n] = wl.dense(9, A.k, n)
    vt, Bt = dev(A.vals), dev(B)
    got, _ = run(A, vt, Bt, n, dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=4), ld=ld)
    ref, N = oracle_product(A.rowptr, A.colind, vt, dev(B[:, :n].copy()), n)
    assert rel_err(got, ref, N) <= TOL_F32
    one, info1 = run(A, vt, Bt, n, dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=1), ld=ld)
    plain, _ = run(A, vt, Bt, n, dict(kernel=nv.SPMM_KERNEL_ROWSPLIT), ld=ld)
    assert info1.config.col_panels == 0
    assert np.array_equal(one, plain)


def test_panels_refusals():
    A = MATS["wide"]()
    rp, ci = dev(A.rowptr), dev(A.colind)
    for cfg in (dict(kernel=nv.SPMM_KERNEL_MERGE, col_panels=4),
                dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=65),
                dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=-2)):
        with pytest.raises(nv.SpmmError) as ei:
            nv.Plan(rp, ci, A.m, A.k, 16, config=cfg, nnz=A.nnz)
        assert ei.value.status == nv.SPMM_ERR_UNSUPPORTED
    # a row whose columns are not increasing
    rowptr = np.array([0, 3, 5], np.int32)
    colind = np.array([4, 2, 9, 1, 3], np.int32)
    with pytest.raises(nv.SpmmError) as ei:
        nv.Plan(dev(rowptr), dev(colind), 2, 10, 16,
                config=dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=2), nnz=5)
    assert ei.value.status == nv.SPMM_ERR_UNSUPPORTED


def test_panels_backward_and_autotune():
    """A panel plan's backward (dB over A^T, dvals) matches the oracle, and
    an autotuned plan of long sorted rows with a B larger than an L2 is
    correct whichever shape it picks."""
    A = wl.random_csr(23, 4000, 60_000, density=0.004)  # mean 240 per row, B 15 MB at n = 64
    n = 64
    B = wl.dense(24, A.k, n)
    dC = wl.dense(25, A.m, n, kind="normal")
    rp, ci = dev(A.rowptr), dev(A.colind)
    vt, Bt, dCt = dev(A.vals), dev(B), dev(dC)
    plan = nv.Plan(rp, ci, A.m, A.k, n, nnz=A.nnz,
                   config=dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=8))
    plan.transpose_build()
    dB = torch.empty(A.k, n, device="cuda")
    dv = torch.empty(A.nnz, device="cuda")
    plan.execute_t(vt, dCt, dB)
    plan.sddmm(dCt, Bt, dv)
    torch.cuda.synchronize()
    ref_dB = oracle.spmm_t(A.rowptr, A.colind, A.vals, dC, A.k)
    N_dB = oracle.spmm_t(A.rowptr, A.colind, A.vals, dC, A.k, absval=True)
    assert rel_err(dB.cpu().numpy(), ref_dB, N_dB) <= TOL_F32
    ref_dv = oracle.sddmm(A.rowptr, A.colind, dC, B)
    N_dv = oracle.sddmm(A.rowptr, A.colind, dC, B, absval=True)
    assert rel_err(dv.cpu().numpy(), ref_dv, N_dv) <= TOL_F32
    plan.close()
    tuned = nv.Plan(rp, ci, A.m, A.k, n, nnz=A.nnz, mode="autotune")
    C = torch.full((A.m, n), float("nan"), device="cuda")
    tuned.execute(vt, Bt, C)
    torch.cuda.synchronize()
    ref, N = oracle_product(A.rowptr, A.colind, vt, Bt, n)
    assert rel_err(C.cpu().numpy(), ref, N) <= TOL_F32
    print("autotuned shape", tuned.info().config.as_dict(), flush=True)
    tuned.close()


def test_panels_with_column_tiles_strips_and_more_panels_than_columns():
    """Panels combined with column tiles (grid y), with the strip order of a
    stencil, and with more panels than A has columns (empty panels): all
    integer-exact against the oracle."""
    rng = np.random.default_rng(11)
    cases = [
        (MATS["wide"](), 64, dict(col_panels=4, tile_cols=32, lanes_per_row=64, unroll=4)),
        (wl.stencil27(g=40), 32, dict(col_panels=2, tile_order=2, lanes_per_row=16, unroll=4)),
        (wl.random_csr(12, 500, 3, density=0.6), 16, dict(col_panels=8, unroll=2)),
    ]
    for A, n, extra in cases:
        vals = rng.integers(-8, 9, A.nnz).astype(np.float32)
        B = rng.integers(-8, 9, (A.k, n)).astype(np.float32)
        cfg = dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, **extra)
        got, info = run(A, dev(vals), dev(B), n, cfg)
        assert info.config.col_panels == extra["col_panels"]
        ref = oracle.spmm(A.rowptr, A.colind, vals, B)
        assert np.array_equal(got.astype(np.float64), ref), extra
