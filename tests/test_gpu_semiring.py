"""Products over the (min, +), (max, +) and (max, *) semirings on the GPU.
min and max are exact and order-free, and rounding is monotone, so each GPU
element must equal the float32 rounding of the FP64 oracle's element whenever
the oracle's own operations are exact (they are for these inputs: sums and
products of two float32 or bf16 values of moderate range are exact in
float64)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import DT, dev, host_bits

pytestmark = pytest.mark.gpu

SEMIRINGS = {"min_plus": (nv.SPMM_MIN_PLUS, oracle.MIN_PLUS),
             "max_plus": (nv.SPMM_MAX_PLUS, oracle.MAX_PLUS),
             "max_times": (nv.SPMM_MAX_TIMES, oracle.MAX_TIMES)}
CFGS = [dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, lanes_per_row=0, unroll=4),
        dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, lanes_per_row=64, unroll=2),
        dict(kernel=nv.SPMM_KERNEL_MERGE, items_per_wg=64, unroll=1),
        dict(kernel=nv.SPMM_KERNEL_MERGE, items_per_wg=1024, unroll=8),
        dict(kernel=nv.SPMM_KERNEL_NZSPLIT, items_per_wg=64, unroll=2),
        dict(kernel=nv.SPMM_KERNEL_ROWBLOCK, rows_per_block=4, unroll=4),
        dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, lanes_per_row=32, unroll=4, col_panels=3)]

MATS = {
    "power_law": lambda: wl.power_law(seed=41, m=20_000, cap=20_000, values="uniform"),
    "empty_rows": lambda: wl.random_csr(2, 600, 500, density=0.02, empty_frac=0.5),
    "giant_row": lambda: wl.CSR(np.array([0, 3, 3, 40_003, 40_010], np.int32),
                                np.concatenate([[1, 2, 3], np.arange(40_000), np.arange(7)]).astype(np.int32),
                                np.random.default_rng(1).uniform(-1, 1, 40_010).astype(np.float32), 4, 40_000),
}


def run(A, vals, B, n, sr, cfg):
    rp, ci = dev(A.rowptr), dev(A.colind)
    plan = nv.Plan(rp, ci, A.m, A.k, n, dtype=nv.dtype_code(vals.dtype), config=cfg, nnz=A.nnz)
    C = torch.full((A.m, n), float("nan"), device="cuda")
    plan.execute_semiring(sr, vals, B, C)
    torch.cuda.synchronize()
    return C.cpu().numpy()


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("sr", sorted(SEMIRINGS))
@pytest.mark.parametrize("cfg", CFGS, ids=["rs", "rs64", "mg64", "mg1024", "nz64", "rb4", "cp3"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_semiring_exact(name, sr, cfg, dtype):
    A = MATS[name]()
    n = 24 if dtype == "f32" else 32
    B = wl.dense(3, A.k, n)
    vt, Bt = dev(A.vals, DT[dtype]), dev(B, DT[dtype])
    got = run(A, vt, Bt, n, SEMIRINGS[sr][0], cfg)
    v, vtag = host_bits(vt)
    b, btag = host_bits(Bt)
    ref = oracle.spmm_semiring(A.rowptr, A.colind, v, b, SEMIRINGS[sr][1], vals_tag=vtag, b_tag=btag)
    assert np.array_equal(got, ref.astype(np.float32))


def test_plus_times_semiring_is_the_product():
    A = wl.power_law(seed=42, m=10_000, cap=5_000)
    n = 16
    B = dev(wl.dense(4, A.k, n))
    for cfg in CFGS:
        rp, ci = dev(A.rowptr), dev(A.colind)
        plan = nv.Plan(rp, ci, A.m, A.k, n, config=cfg, nnz=A.nnz)
        C1 = torch.empty(A.m, n, device="cuda")
        C2 = torch.empty(A.m, n, device="cuda")
        plan.execute(dev(A.vals), B, C1)
        plan.execute_semiring(nv.SPMM_PLUS_TIMES, dev(A.vals), B, C2)
        torch.cuda.synchronize()
        assert torch.equal(C1, C2)


def test_min_plus_shortest_paths_on_gpu():
    """Bellman-Ford with the GPU min-plus product on A^T reaches scipy's
    shortest-path distances."""
    from scipy.sparse.csgraph import shortest_path
    import scipy.sparse as sp
    N = 3000
    A = wl.random_csr(9, N, N, density=0.002)
    A.vals = np.random.default_rng(9).integers(1, 20, A.nnz).astype(np.float32)
    at_rp, at_ci, perm = oracle.transpose(A.rowptr, A.colind, N)
    T = wl.CSR(at_rp, at_ci, A.vals[perm], N, N)
    src = [0, 11, 2999, 1500]
    d = np.full((N, 4), np.inf, np.float32)
    d[src, np.arange(4)] = 0.0
    dd = dev(d)
    rp, ci, vt = dev(T.rowptr), dev(T.colind), dev(T.vals)
    plan = nv.Plan(rp, ci, N, N, 4, mode="merge", nnz=T.nnz)
    relax = torch.empty_like(dd)
    for _ in range(60):
        plan.execute_semiring(nv.SPMM_MIN_PLUS, vt, dd, relax)
        nd = torch.minimum(dd, relax)
        if torch.equal(nd, dd):
            break
        dd = nd
    torch.cuda.synchronize()
    ref = shortest_path(sp.csr_matrix((A.vals.astype(np.float64), A.colind, A.rowptr), shape=(N, N)),
                        method="D", directed=True, indices=src).T
    assert np.array_equal(dd.cpu().numpy().astype(np.float64), ref)


def test_semiring_bad_code():
    A = wl.random_csr(1, 10, 10, density=0.3)
    plan = nv.Plan(dev(A.rowptr), dev(A.colind), A.m, A.k, 4, nnz=A.nnz)
    with pytest.raises(nv.SpmmError):
        plan.execute_semiring(7, dev(A.vals), dev(np.zeros((10, 4), np.float32)),
                              torch.empty(10, 4, device="cuda"))
