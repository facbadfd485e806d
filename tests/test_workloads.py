"""Statistics and determinism of the seeded input generators."""
import numpy as np

from paper_1803_08601_amd import workloads as wl


def _check_csr(A):
    assert A.rowptr.dtype == np.int32 and A.colind.dtype == np.int32
    assert A.rowptr[0] == 0 and np.all(np.diff(A.rowptr) >= 0)
    assert A.colind.shape[0] == A.nnz == A.vals.shape[0]
    assert A.nnz == 0 or (A.colind.min() >= 0 and A.colind.max() < A.k)
    # distinct and sorted within each row
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    key = rows.astype(np.int64) * A.k + A.colind
    assert np.all(np.diff(key) > 0)


def test_plain():
    A = wl.plain()
    _check_csr(A)
    assert A.nnz == 4096 * 16 and np.all(A.row_lengths() == 16)
    assert -1 <= A.vals.min() and A.vals.max() < 1


def test_power_law_small_and_deterministic():
    A = wl.power_law(seed=1002, m=200_000, cap=100_000)
    _check_csr(A)
    L = A.row_lengths()
    assert abs(L.mean() - 16.0) < 0.05
    assert np.median(L) <= 5 and L.min() >= 1
    assert (L < 9.35).mean() > 0.7
    B = wl.power_law(seed=1002, m=200_000, cap=100_000)
    assert A.digest() == B.digest()
    C = wl.power_law(seed=1003, m=200_000, cap=100_000)
    assert A.digest() != C.digest()


def test_stencil_small():
    g = 9
    A = wl.stencil27(g=g)
    _check_csr(A)
    assert A.nnz == (3 * g - 2) ** 3
    L = A.row_lengths()
    assert L.min() == 8 and L.max() == 27
    rows = np.repeat(np.arange(A.m), L)
    diag = rows == A.colind
    assert np.all(A.vals[diag] == 26.0)
    off = A.vals[~diag]
    assert np.all(np.abs(off + 1.0) <= 1e-3 + 1e-7)


def test_gcn_small():
    A = wl.gcn_adjacency(N=5_000, mean_deg=32)
    _check_csr(A)
    deg = A.row_lengths() - 1
    assert abs(deg.mean() - 32.0) <= 0.5
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    assert np.all(np.isin(np.arange(A.m), A.colind[rows == A.colind]))  # self loops


def test_random_csr_dups():
    A = wl.random_csr(1, 50, 30, density=0.3, dup_frac=1.0)
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    key = rows.astype(np.int64) * A.k + A.colind
    assert np.unique(key).shape[0] < A.nnz


def test_batch_specs():
    specs = wl.batch_specs(count=512)
    ms = np.array([s[0] for s in specs])
    assert ms.min() >= 1000 and ms.max() <= 200_000
    assert set(s[1] for s in specs) <= {8, 32, 128}
    assert [s[2] for s in specs[:4]] == ["uniform", "zipf", "uniform", "zipf"]
    P = wl.batch_problem(1005, 1, 3000, "zipf")
    _check_csr(P)
    Q = wl.batch_problem(1005, 0, 3000, "uniform")
    _check_csr(Q)
    L = Q.row_lengths()
    assert L.min() >= 8 and L.max() <= 64


def test_grid_stencils_and_banded():
    # 7-point on 4^3: corners 4, edges 5, faces 6, interior 7 neighbours
    A = wl.grid_stencil(1, (4, 4, 4), 7)
    assert np.array_equal(np.bincount(A.row_lengths()), [0, 0, 0, 0, 8, 24, 24, 8])
    # the 27-point form has the structure of stencil27
    B, S = wl.grid_stencil(1, (6, 6, 6), 27), wl.stencil27(g=6)
    assert np.array_equal(B.rowptr, S.rowptr) and np.array_equal(B.colind, S.colind)
    # 5-point on a 5 x 5 grid: 4 * 5 * 4 horizontal and vertical neighbour pairs
    C = wl.grid_stencil(1, (5, 5), 5)
    assert C.nnz == 25 + 2 * 2 * 5 * 4
    D = wl.banded(2, 3000, per_row=16, half_band=100)
    assert np.all(D.row_lengths() == 16)
    rows = np.repeat(np.arange(D.m), 16)
    lo = np.clip(rows - 100, 0, D.m - 201)
    assert np.all((D.colind >= lo) & (D.colind <= lo + 200))
    for M in (A, C, D):
        for i in range(0, M.m, max(1, M.m // 50)):
            assert np.all(np.diff(M.colind[M.rowptr[i]:M.rowptr[i + 1]]) > 0)
