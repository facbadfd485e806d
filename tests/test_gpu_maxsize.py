"""The largest accepted entry count, nnz = 2^31 - 4097 (entry indices are
int32 in the kernels; their chunk loops step past an index below nnz by at
most 4096): row split, merge path, nonzero split, SDDMM, the transpose and
dB on rows whose entries reach the top of that range, and merge diagonals
past 2^31 (m + nnz exceeds int32). Integer values make every product exact: sampled rows (the
last non-empty row holds the largest indices) equal the oracle's bit for
bit, the three forward kernels agree on every row, the trailing empty rows
are zero, and the partitions equal the oracle's coordinates."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

MAX_NNZ = 2**31 - 4097
M, K, N = 2**21, 2**20, 8


@pytest.fixture(scope="module")
def big():
    # rows of 1024 entries, then one of 1023 and four empty rows: 2^31 - 4097
    lengths = np.full(M, 1024, np.int64)
    lengths[-5] = 1023
    lengths[-4:] = 0
    rowptr = wl.rowptr_from_lengths(lengths)
    assert int(rowptr[-1]) == MAX_NNZ
    g = torch.Generator(device="cuda").manual_seed(2031)
    ci = torch.randint(0, K, (MAX_NNZ,), generator=g, device="cuda", dtype=torch.int32)
    vals = torch.randint(-4, 5, (MAX_NNZ,), generator=g, device="cuda", dtype=torch.float32)
    B = wl.dense(2032, K, N, kind="int")
    dC = wl.dense(2033, M, N, kind="int")
    # sampled rows: the first, some in the middle and past 2^30, the last
    # non-empty ones and the empty tail
    rows = np.array([0, 1, 4097, M // 2, M // 2 + 1, M - 300, M - 7, M - 6, M - 5,
                     M - 4, M - 3, M - 2, M - 1], np.int64)
    sub_len = lengths[rows]
    sub_rp = wl.rowptr_from_lengths(sub_len)
    idx = np.concatenate([np.arange(rowptr[r], rowptr[r + 1], dtype=np.int64) for r in rows])
    it = torch.from_numpy(idx).cuda()
    sub_ci = ci[it].cpu().numpy()
    sub_v = vals[it].cpu().numpy()
    data = dict(rowptr=rowptr, ci=ci, vals=vals, B=B, dC=dC, rows=rows, sub_rp=sub_rp,
                sub_ci=sub_ci, sub_v=sub_v, idx=it)
    del ci, vals
    yield data
    data.clear()
    torch.cuda.empty_cache()


def _forward(d, **plan_kw):
    plan = nv.Plan(dev(d["rowptr"]), d["ci"], M, K, N, nnz=MAX_NNZ, **plan_kw)
    C = torch.full((M, N), float("nan"), device="cuda")
    plan.execute(d["vals"], dev(d["B"]), C)
    torch.cuda.synchronize()
    return plan, C


def test_forward_kernels_at_max_nnz(big):
    d = big
    ref = oracle.spmm(d["sub_rp"], d["sub_ci"], d["sub_v"], d["B"], k=K).astype(np.float32)
    assert np.abs(ref).max() < 2**24
    rows_t = torch.from_numpy(d["rows"]).cuda()
    first = None
    for name, kw in (("paper", dict(mode="paper")),
                     ("merge", dict(config=dict(kernel=nv.SPMM_KERNEL_MERGE,
                                                items_per_wg=1024))),
                     ("nzsplit", dict(config=dict(kernel=nv.SPMM_KERNEL_NZSPLIT,
                                                  items_per_wg=2048)))):
        plan, C = _forward(d, **kw)
        info = plan.info()
        if name == "paper":  # mean row length 1024: the Sec. 5.4 rule takes row split
            assert info.config.kernel == nv.SPMM_KERNEL_ROWSPLIT
        else:
            W = info.config.items_per_wg
            want = (oracle.merge_partition(d["rowptr"], W) if name == "merge"
                    else oracle.nz_partition(d["rowptr"], W))
            got = plan.partition()
            assert np.array_equal(got, want), name
        assert not torch.isnan(C).any(), name
        got_rows = C[rows_t].cpu().numpy()
        assert np.array_equal(got_rows, ref), f"{name}: {int((got_rows != ref).sum())} differ"
        assert torch.all(C[M - 4:] == 0), name
        if first is None:
            first = C
        else:
            assert torch.equal(C, first), f"{name}: differs from row split on some row"
            del C
        plan.close()
        torch.cuda.synchronize()


def test_sddmm_at_max_nnz(big):
    d = big
    plan = nv.Plan(dev(d["rowptr"]), d["ci"], M, K, N, nnz=MAX_NNZ, mode="paper")
    dv = torch.full((MAX_NNZ,), float("nan"), device="cuda")
    plan.sddmm(dev(d["dC"]), dev(d["B"]), dv)
    torch.cuda.synchronize()
    assert not torch.isnan(dv).any()
    ref = oracle.sddmm(d["sub_rp"], d["sub_ci"], d["dC"][d["rows"]], d["B"]).astype(np.float32)
    got = dv[d["idx"]].cpu().numpy()
    assert np.array_equal(got, ref), f"{int((got != ref).sum())} differ"
    # the very last entries of the index range
    assert got[-1023:].size == 1023 and np.array_equal(got[-1023:], ref[-1023:])
    plan.close()
    del dv
    torch.cuda.empty_cache()


def test_transpose_and_dB_at_max_nnz(big):
    """The radix-sort transpose at 2^31 - 4097 entries (digit histograms and
    scans at their largest) equals the oracle's counting sort bit for bit,
    and dB = A^T dC is exact on sampled columns, among them the column of
    the last entry."""
    d = big
    plan = nv.Plan(dev(d["rowptr"]), d["ci"], M, K, N, nnz=MAX_NNZ, mode="paper")
    plan.transpose_build()
    at_rp = torch.empty(K + 1, dtype=torch.int32, device="cuda")
    at_ci = torch.empty(MAX_NNZ, dtype=torch.int32, device="cuda")
    perm = torch.empty(MAX_NNZ, dtype=torch.int32, device="cuda")
    nv.spmm_transpose_get(plan.handle, at_rp, at_ci, perm)
    dB = torch.full((K, N), float("nan"), device="cuda")
    plan.execute_t(d["vals"], dev(d["dC"]), dB)
    torch.cuda.synchronize()
    e_rp, e_ci, e_perm = oracle.transpose(d["rowptr"], d["ci"].cpu().numpy(), K)
    assert np.array_equal(at_rp.cpu().numpy(), e_rp)
    assert np.array_equal(at_ci.cpu().numpy(), e_ci)
    assert np.array_equal(perm.cpu().numpy(), e_perm)
    del at_ci, perm
    assert not torch.isnan(dB).any()
    last_col = int(d["ci"][MAX_NNZ - 1])
    cols = np.unique(np.array([0, 1, K // 2, K - 1, last_col], np.int64))
    q = np.concatenate([np.arange(e_rp[c], e_rp[c + 1], dtype=np.int64) for c in cols])
    v = d["vals"][torch.from_numpy(e_perm[q].astype(np.int64)).cuda()].cpu().numpy()
    sub_rp = wl.rowptr_from_lengths(e_rp[cols + 1].astype(np.int64) - e_rp[cols])
    ref = oracle.spmm(sub_rp, e_ci[q], v, d["dC"], k=M).astype(np.float32)
    assert np.array_equal(dB[torch.from_numpy(cols).cuda()].cpu().numpy(), ref)
    plan.close()
    del dB, e_ci, e_perm
    torch.cuda.empty_cache()
