"""Kernel choice (Sec. 5.4) through the C ABI, compared with the oracle and
with row statistics computed in numpy; the one-call entry point's choice and
its handling of a structure that changes behind cached pointers."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import TOL_F32, dev, oracle_product, rel_err

pytestmark = pytest.mark.gpu

RS = nv.SPMM_KERNEL_ROWSPLIT
MG = nv.SPMM_KERNEL_MERGE
RB = nv.SPMM_KERNEL_ROWBLOCK


def csr_with(m, nnz, k=64, seed=0):
    """m rows holding nnz entries in total, spread as evenly as possible, at
    distinct sorted random columns of [0, k)."""
    rng = np.random.default_rng(seed)
    lengths = np.full(m, nnz // m if m else 0, np.int64)
    if m:
        lengths[rng.permutation(m)[: nnz - int(lengths.sum())]] += 1
    cols = wl.distinct_sorted_columns(rng, lengths, k)
    vals = rng.uniform(-1, 1, cols.shape[0]).astype(np.float32)
    return wl.CSR(wl.rowptr_from_lengths(lengths), cols, vals, m, k)


def check_product(A, C, vals_t, B_t, n):
    Cref, N = oracle_product(A.rowptr, A.colind, vals_t, B_t, n)
    assert rel_err(C[:, :n].cpu().numpy(), Cref, N) <= TOL_F32


# The table of Sec. 5.4 decisions: merge-based iff nnz / m < 9.35, so a mean
# of exactly 9.35 takes row split; nnz = 0 has mean 0 (merge-based); m = 0
# has no rows (row split, the kernel that launches nothing).
PAPER_TABLE = [(20, 187), (20, 186), (100, 935), (100, 934), (1, 9), (1, 10), (10, 0), (0, 0),
               (7, 65), (7, 66), (3, 28), (3, 29)]


@pytest.mark.parametrize("m,nnz", PAPER_TABLE)
def test_paper_mode_matches_oracle_rule(m, nnz):
    A = csr_with(m, nnz)
    n = 16
    want = MG if oracle.heuristic_merge(m, nnz) else RS
    rp, ci = dev(A.rowptr), dev(A.colind)
    plan = nv.Plan(rp, ci, m, A.k, n, mode="paper", nnz=nnz)
    info = plan.info()
    assert info.paper_choice == want
    assert info.config.kernel == want
    if m:
        v = dev(A.vals)
        Bt = dev(wl.dense(3, A.k, n))
        C = torch.full((m, n), float("nan"), device="cuda")
        plan.execute(v, Bt, C)
        torch.cuda.synchronize()
        check_product(A, C, v, Bt, n)
    plan.close()


def test_paper_rule_spot_values_from_the_oracle():
    # the oracle's own decisions at the threshold, as the table above assumes
    assert not oracle.heuristic_merge(20, 187) and oracle.heuristic_merge(20, 186)
    assert not oracle.heuristic_merge(100, 935) and oracle.heuristic_merge(100, 934)
    assert oracle.heuristic_merge(1, 9) and not oracle.heuristic_merge(1, 10)
    assert oracle.heuristic_merge(10, 0) and not oracle.heuristic_merge(0, 0)


def _stat_cases():
    pl = wl.power_law(seed=71, m=50_000, cap=20_000)
    giant = np.zeros(1000, np.int64)
    giant[500] = 5000
    rng = np.random.default_rng(72)
    G = wl.CSR(wl.rowptr_from_lengths(giant), wl.distinct_sorted_columns(rng, giant, 8000),
               np.ones(5000, np.float32), 1000, 8000)
    E = wl.CSR(np.zeros(101, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), 100, 50)
    one = np.array([3000], np.int64)
    O = wl.CSR(wl.rowptr_from_lengths(one), wl.distinct_sorted_columns(rng, one, 4000),
               np.ones(3000, np.float32), 1, 4000)
    edge = np.array([1023, 1024, 0, 1025, 4096, 4095], np.int64)
    X = wl.CSR(wl.rowptr_from_lengths(edge), wl.distinct_sorted_columns(rng, edge, 5000),
               np.ones(int(edge.sum()), np.float32), 6, 5000)
    return [("power law", pl), ("one giant row among empty rows", G), ("all rows empty", E),
            ("one row", O), ("lengths around 1024 and 4096", X)]


@pytest.mark.parametrize("case", range(5))
def test_device_row_statistics_match_numpy(case):
    """The device statistics that feed mode RULE and the tuner's cache key:
    the longest row and the number of rows with at least 1024 entries."""
    name, A = _stat_cases()[case]
    lengths = np.diff(A.rowptr.astype(np.int64))
    rp, ci = dev(A.rowptr), dev(A.colind)
    plan = nv.Plan(rp, ci, A.m, A.k, 8, mode="paper", nnz=A.nnz)
    info = plan.info()
    assert info.max_row_len == (int(lengths.max()) if A.m else 0), name
    assert info.long_rows == int(np.count_nonzero(lengths >= 1024)), name
    plan.close()


def rule_expected(A, n, rowblocks=True):
    """Mode RULE recomputed from numpy statistics of the matrix."""
    lengths = np.diff(A.rowptr.astype(np.int64))
    if A.m == 0:
        return RS
    maxrow = int(lengths.max())
    if A.nnz < 4 * A.m or maxrow >= 4096:
        return MG
    if not rowblocks or n < 32 or A.nnz == 0 or A.k >= 2**24 or maxrow > 4096:
        return RS
    rows = np.repeat(np.arange(A.m, dtype=np.int64), lengths)
    c = A.colind.astype(np.int64)
    if np.any((rows[1:] == rows[:-1]) & (c[1:] <= c[:-1])):
        return RS  # a row's columns do not strictly increase
    union2 = np.unique((rows // 2) * A.k + c).size
    return RB if union2 <= 0.9 * A.nnz else RS


def _rule_cases():
    S = wl.stencil27(g=20)
    ci = S.colind.copy()
    ci[S.rowptr[5]:S.rowptr[6]] = ci[S.rowptr[5]:S.rowptr[6]][::-1]
    S_uns = wl.CSR(S.rowptr, ci, S.vals, S.m, S.k)
    short = csr_with(5000, 19_999, k=3000, seed=4)   # mean just below 4
    short4 = csr_with(5000, 20_000, k=3000, seed=4)  # mean exactly 4
    edge = np.full(2000, 12, np.int64)
    edge[7] = 4095
    E4095 = wl.CSR(wl.rowptr_from_lengths(edge),
                   wl.distinct_sorted_columns(np.random.default_rng(9), edge, 6000),
                   np.ones(int(edge.sum()), np.float32), 2000, 6000)
    edge2 = edge.copy()
    edge2[7] = 4096
    E4096 = wl.CSR(wl.rowptr_from_lengths(edge2),
                   wl.distinct_sorted_columns(np.random.default_rng(9), edge2, 6000),
                   np.ones(int(edge2.sum()), np.float32), 2000, 6000)
    return [(wl.power_law(seed=51, m=40_000, cap=20_000), 16), (S, 16), (S, 32), (S, 64),
            (S_uns, 64), (wl.grid_stencil(3, (300, 300), 5), 32), (wl.plain(m=2000, k=2000), 64),
            (short, 64), (short4, 64), (E4095, 8), (E4096, 8), (E4095, 64)]


@pytest.mark.parametrize("case", range(12))
def test_rule_mode_from_numpy_statistics(case):
    A, n = _rule_cases()[case]
    want = rule_expected(A, n)
    rp, ci = dev(A.rowptr), dev(A.colind)
    plan = nv.Plan(rp, ci, A.m, A.k, n, mode="rule", nnz=A.nnz)
    assert plan.info().config.kernel == want, (A.m, A.nnz, n)
    plan.close()


@pytest.mark.parametrize("case", range(12))
def test_one_call_kernel_is_rule_over_the_two_kernels(case):
    """spmm_csr plans by mode RULE restricted to the paper's two kernels; its
    product matches the oracle."""
    A, n = _rule_cases()[case]
    want = rule_expected(A, n, rowblocks=False)
    rp, ci, v = dev(A.rowptr), dev(A.colind), dev(A.vals)
    Bt = dev(wl.dense(8, A.k, n))
    C = torch.full((A.m, n), float("nan"), device="cuda")
    nv.spmm_cache_clear()
    with pytest.raises(nv.SpmmError):
        nv.spmm_csr_plan_info(rp, ci, A.m, A.k, n, n)
    nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)
    torch.cuda.synchronize()
    info = nv.spmm_csr_plan_info(rp, ci, A.m, A.k, n, n)
    assert info.config.kernel == want
    assert info.mode == nv.SPMM_MODE_RULE and info.nnz == A.nnz
    check_product(A, C, v, Bt, n)
    nv.spmm_cache_clear()


def test_one_call_structure_changed_behind_cached_pointers():
    """A new matrix placed at the addresses of a cached one: with the same
    nnz the merge partition is re-searched on the device and the product is
    right; with another nnz the call fills C with NaN, the next call reports
    SPMM_ERR_STATE and the one after plans afresh."""
    A = wl.power_law(seed=81, m=30_000, cap=20_000)
    n = 32
    lengths = np.diff(A.rowptr.astype(np.int64))
    assert lengths.max() >= 4096  # the rule takes merge-based
    cap = A.nnz + 1000
    rp = torch.zeros(A.m + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(cap, dtype=torch.int32, device="cuda")
    v = torch.zeros(cap, dtype=torch.float32, device="cuda")
    Bt = dev(wl.dense(81, A.k, n))
    C = torch.empty(A.m, n, device="cuda")

    def place(M):
        rp.copy_(dev(M.rowptr))
        ci[: M.nnz].copy_(dev(M.colind))
        v[: M.nnz].copy_(dev(M.vals))
        torch.cuda.synchronize()

    def run_and_check(M):
        C.fill_(float("nan"))
        nv.spmm_csr(rp, ci, v, Bt, C, M.m, M.k, n, n)
        torch.cuda.synchronize()
        check_product(M, C, v[: M.nnz], Bt, n)

    nv.spmm_cache_clear()
    place(A)
    run_and_check(A)
    assert nv.spmm_csr_plan_info(rp, ci, A.m, A.k, n, n).config.kernel == MG
    # the same row lengths in another order, new columns: same nnz, new partition
    rng = np.random.default_rng(82)
    l2 = lengths[rng.permutation(A.m)]
    A2 = wl.CSR(wl.rowptr_from_lengths(l2), wl.distinct_sorted_columns(rng, l2, A.k),
                rng.standard_normal(A.nnz).astype(np.float32), A.m, A.k)
    place(A2)
    run_and_check(A2)
    # fewer entries: the cached partition cannot hold, C becomes NaN
    l3 = l2.copy()
    l3[np.argmax(l3)] -= 500
    A3 = wl.CSR(wl.rowptr_from_lengths(l3), wl.distinct_sorted_columns(rng, l3, A.k),
                rng.standard_normal(int(l3.sum())).astype(np.float32), A.m, A.k)
    place(A3)
    C.zero_()
    nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)
    torch.cuda.synchronize()
    assert torch.isnan(C).all()
    with pytest.raises(nv.SpmmError) as ei:
        nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)
    assert ei.value.status == nv.SPMM_ERR_STATE
    run_and_check(A3)
    assert nv.spmm_csr_plan_info(rp, ci, A.m, A.k, n, n).nnz == A3.nnz
    # more entries than the cached plan: the same path
    place(A2)
    C.zero_()
    nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)
    torch.cuda.synchronize()
    assert torch.isnan(C).all()
    with pytest.raises(nv.SpmmError):
        nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)
    run_and_check(A2)
    # a row-split plan re-reads the whole structure on every call
    P = wl.plain(m=3000, k=3000)
    rp2, ci2, v2 = dev(P.rowptr), dev(P.colind), dev(P.vals)
    B2 = dev(wl.dense(83, P.k, n))
    C2 = torch.empty(P.m, n, device="cuda")
    nv.spmm_csr(rp2, ci2, v2, B2, C2, P.m, P.k, n, n)
    assert nv.spmm_csr_plan_info(rp2, ci2, P.m, P.k, n, n).config.kernel == RS
    P2 = wl.plain(seed=99, m=3000, k=3000)
    ci2.copy_(dev(P2.colind))
    v2.copy_(dev(P2.vals))
    nv.spmm_csr(rp2, ci2, v2, B2, C2, P.m, P.k, n, n)
    torch.cuda.synchronize()
    check_product(P2, C2, v2, B2, n)
    nv.spmm_cache_clear()


def test_one_call_refuses_invalid_row_offsets():
    A = csr_with(50, 600, k=100, seed=5)
    bad = A.rowptr.copy()
    bad[10], bad[11] = bad[11], bad[10]  # decreasing
    rp, ci, v = dev(bad), dev(A.colind), dev(A.vals)
    Bt = dev(wl.dense(5, A.k, 8))
    C = torch.empty(A.m, 8, device="cuda")
    nv.spmm_cache_clear()
    with pytest.raises(nv.SpmmError) as ei:
        nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, 8, 8)
    assert ei.value.status == nv.SPMM_ERR_INVALID
