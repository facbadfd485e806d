"""Every launch shape a plan can take, against the FP64 oracle.

The autotuner and the batch planner may pick any valid combination of kernel
(row split, merge path, nonzero split, row blocks), vector width, lanes per
row, unroll, merge items per workgroup, rows per block and column tile; each is a separate code path in
the kernels (template instantiations plus the runtime slot geometry). This
sweep runs all of them on one ragged matrix: empty rows, rows of every short
length, rows whose length is not a multiple of any slot count, and long rows
that span several merge pieces even at the largest piece size, for n from 1
to beyond one 64-lane pass."""
import numpy as np
import pytest
import torch

from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import TOL_F32, TOL_STORAGE_16, dev, oracle_product, rel_err

pytestmark = pytest.mark.gpu

RS, MG, NZ = nv.SPMM_KERNEL_ROWSPLIT, nv.SPMM_KERNEL_MERGE, nv.SPMM_KERNEL_NZSPLIT
RB = nv.SPMM_KERNEL_ROWBLOCK
VEC16 = {torch.float32: 4, torch.bfloat16: 8}


def ragged_matrix(seed=4242, m=700, k=1200):
    rng = np.random.default_rng(seed)
    lengths = np.concatenate([
        np.zeros(40, np.int64),                      # empty rows
        np.arange(1, 70, dtype=np.int64),            # every short length
        rng.integers(0, 24, m - 40 - 69 - 3),        # mostly short, ragged
        np.array([1100, 513, 9000 % k + 65]),        # long rows
    ])
    rng.shuffle(lengths)
    colind = wl.distinct_sorted_columns(rng, lengths, k)
    rowptr = wl.rowptr_from_lengths(lengths)
    vals = rng.uniform(-1, 1, colind.shape[0]).astype(np.float32)
    return wl.CSR(rowptr, colind, vals, m, k)


def configs(n, dtype):
    v16 = VEC16[dtype]
    vecs = [1] + ([v16] if n % v16 == 0 else [])
    for vec in vecs:
        tiles = [0] + ([2 * v16] if n > 2 * v16 else [])
        for tc in tiles:
            for u in (1, 2, 4, 8):
                for lanes in (1, 2, 4, 8, 16, 32, 64):
                    yield dict(kernel=RS, vec=vec, lanes_per_row=lanes, unroll=u, tile_cols=tc)
                for kern in (MG, NZ):
                    for W in (64, 100, 1000, 4096):
                        yield dict(kernel=kern, vec=vec, items_per_wg=W, unroll=u, tile_cols=tc)
                for R in (2, 4, 8):
                    for lanes in (1, 4, 16, 64):
                        yield dict(kernel=RB, vec=vec, lanes_per_row=lanes, unroll=u,
                                   tile_cols=tc, rows_per_block=R)


@pytest.fixture(scope="module")
def matrix():
    A = ragged_matrix()
    return A, dev(A.rowptr), dev(A.colind)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
@pytest.mark.parametrize("n", [1, 3, 8, 24, 64, 72, 136])
def test_every_launch_shape(matrix, dtype, n):
    A, rp, ci = matrix
    vals = dev(A.vals).to(dtype)
    B = dev(wl.dense(77, A.k, n)).to(dtype)
    Cref, N = oracle_product(A.rowptr, A.colind, vals, B, n)
    tol = TOL_F32 if dtype == torch.float32 else TOL_STORAGE_16
    code = nv.dtype_code(dtype)
    C = torch.empty(A.m, n, device="cuda")
    ran = 0
    for cfg in configs(n, dtype):
        plan = nv.Plan(rp, ci, A.m, A.k, n, dtype=code, config=cfg, nnz=A.nnz)
        try:
            C.fill_(float("nan"))
            plan.execute(vals, B, C)
            torch.cuda.synchronize()
            e = rel_err(C.cpu().numpy(), Cref, N)
            assert e <= tol, f"config {cfg}: max rel err {e}"
            ran += 1
        finally:
            plan.close()
    assert ran == len(list(configs(n, dtype)))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
@pytest.mark.parametrize("n", [1, 3, 8, 24, 64, 72, 136])
def test_sddmm_every_launch_shape(matrix, dtype, n):
    """SDDMM walks diagonal pieces of 1024 items: the plan's own when it is a
    merge plan of that piece size, else a partition built with the plan;
    every vector width and plan shape."""
    import oracle
    from spmm_check import host_bits

    A, rp, ci = matrix
    B = dev(wl.dense(78, A.k, n)).to(dtype)
    dC = wl.dense(79, A.m, n, kind="normal")
    dCt = dev(dC)
    b, btag = host_bits(B)
    ref = oracle.sddmm(A.rowptr, A.colind, dC, b, b_tag=btag)
    N = oracle.sddmm(A.rowptr, A.colind, dC, b, b_tag=btag, absval=True)
    v16 = VEC16[dtype]
    shapes = [dict(kernel=MG, items_per_wg=W) for W in (64, 100, 1000, 1024, 4096)]
    shapes += [dict(kernel=RS), dict(kernel=NZ, items_per_wg=1000), dict(kernel=RB)]
    dv = torch.empty(A.nnz, device="cuda")
    ran = 0
    for vec in [1] + ([v16] if n % v16 == 0 else []):
        for shape in shapes:
            plan = nv.Plan(rp, ci, A.m, A.k, n, dtype=nv.dtype_code(dtype),
                           config=dict(shape, vec=vec), nnz=A.nnz)
            try:
                dv.fill_(float("nan"))
                plan.sddmm(dCt, B, dv)
                torch.cuda.synchronize()
                e = rel_err(dv.cpu().numpy(), ref, N)
                assert e <= TOL_F32, f"vec {vec} {shape}: max rel err {e}"
                ran += 1
            finally:
                plan.close()
    assert ran == len(shapes) * (2 if n % v16 == 0 else 1)
