"""Strips across planes (spmm_config.tile_order): the plan finds a 3-D
stencil's plane distance, the kernels take their rows in strips through the
planes, and every result is bitwise the one of the row order."""
import numpy as np
import pytest
import torch

from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import TOL_F32, dev, oracle_product, rel_err

pytestmark = pytest.mark.gpu

RS = nv.SPMM_KERNEL_ROWSPLIT
RB = nv.SPMM_KERNEL_ROWBLOCK

SHAPES = [dict(kernel=RS), dict(kernel=RS, lanes_per_row=64, unroll=8),
          dict(kernel=RS, lanes_per_row=8, unroll=1), dict(kernel=RB, rows_per_block=2),
          dict(kernel=RB, rows_per_block=4, lanes_per_row=32, unroll=4),
          dict(kernel=RB, rows_per_block=8, lanes_per_row=64, unroll=2)]


def strip_for(D, row_bytes):
    """The strip the plan should pick: the largest power of two dividing D
    whose rows' B rows over three planes take at most 2 MB."""
    S = 1
    while S * 2 * 3 * row_bytes <= 2 << 20:
        S *= 2
    while S > 1 and D % S:
        S //= 2
    return S


@pytest.mark.parametrize("g,n", [(48, 128), (64, 128), (64, 16), (40, 32)])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_strips_bitwise_equal_to_row_order(g, n, shape):
    A = wl.stencil27(seed=3, g=g)
    B = wl.dense(4, A.k, n)
    rp, ci, v, Bt = dev(A.rowptr), dev(A.colind), dev(A.vals), dev(B)
    out = {}
    for order in (1, 2, 0):
        cfg = dict(SHAPES[shape], tile_order=order)
        plan = nv.Plan(rp, ci, A.m, A.k, n, nnz=A.nnz, config=cfg)
        info = plan.info()
        D = g * g
        S = strip_for(D, 4 * n)
        if order == 2 and 64 <= S < D:
            assert info.plane_rows == D
            assert info.strip_rows == S
        else:
            # row order: forced; automatic with a plane of B rows that fits an
            # L2; or strips as long as a plane
            assert order != 0 or D * 4 * n <= 4 << 20
            assert info.plane_rows == 0 and info.strip_rows == 0
        C = torch.full((A.m, n), float("nan"), device="cuda")
        plan.execute(v, Bt, C)
        torch.cuda.synchronize()
        out[order] = C
        plan.close()
    assert torch.equal(out[1], out[2])
    assert torch.equal(out[1], out[0])
    Cref, N = oracle_product(A.rowptr, A.colind, v, Bt, n)
    assert rel_err(out[2].cpu().numpy(), Cref, N) <= TOL_F32


def test_no_planes_found_elsewhere():
    """Matrices without far, narrow diagonal clusters keep the row order."""
    n = 128
    for A in (wl.power_law(seed=5, m=40_000, cap=20_000), wl.banded(6, 60_000),
              wl.grid_stencil(7, (300, 300), 5), wl.plain(m=5000, k=5000)):
        rp, ci = dev(A.rowptr), dev(A.colind)
        plan = nv.Plan(rp, ci, A.m, A.k, n, nnz=A.nnz, config=dict(kernel=RS, tile_order=2))
        info = plan.info()
        assert info.plane_rows == 0 and info.strip_rows == 0, A.m
        plan.close()


def test_tile_order_refusal():
    A = wl.stencil27(seed=3, g=12)
    rp, ci = dev(A.rowptr), dev(A.colind)
    with pytest.raises(nv.SpmmError):
        nv.Plan(rp, ci, A.m, A.k, 16, nnz=A.nnz, config=dict(kernel=RS, tile_order=3))
