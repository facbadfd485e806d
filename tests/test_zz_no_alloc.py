"""The no-allocation one-call entry point spmm_csr_noalloc against the
one-call entry point spmm_csr on the same inputs, through the C ABI: both
within the float32 tolerance of the FP64 oracle and of each other, and
bitwise equal on integer-valued inputs (every partial sum exact). Two calls
in a row with a smaller second input, so the second runs on scratch that
still holds the first call's coordinates and carry-outs."""
import numpy as np
import pytest
import torch

from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import TOL_F32, dev, oracle_product, rel_err

pytestmark = pytest.mark.gpu


def _both(A, vals, B, n):
    rp, ci, v, Bt = dev(A.rowptr), dev(A.colind), dev(vals), dev(B)
    C1 = torch.full((A.m, n), float("nan"), device="cuda")
    C2 = torch.full((A.m, n), float("nan"), device="cuda")
    nv.spmm_csr(rp, ci, v, Bt, C1, A.m, A.k, n, n)
    nv.spmm_csr_noalloc(rp, ci, v, Bt, C2, A.m, A.k, A.nnz, n, n)
    torch.cuda.synchronize()
    return C1.cpu().numpy(), C2.cpu().numpy(), (rp, ci, v, Bt)


# (seed, m, mean row length, n): merge-based by the Sec. 5.4 rule (mean
# below 9.35), the second call of each pair smaller than the first; then row
# split (mean 16), which uses no scratch
CASES = [
    [(31, 120_000, 4.0, 64), (32, 20_000, 6.0, 32)],
    [(33, 60_000, 3.0, 128), (34, 5_000, 2.0, 8)],
    [(35, 40_000, 16.0, 32), (36, 3_000, 5.0, 16)],
]


@pytest.mark.parametrize("pair", CASES, ids=lambda p: "-".join(f"m{c[1]}n{c[3]}" for c in p))
def test_noalloc_matches_spmm_csr_two_calls(pair):
    for seed, m, mean, n in pair:
        print(f"noalloc case seed={seed} m={m} mean={mean} n={n}", flush=True)
        A = wl.power_law(seed=seed, m=m, mean=mean, cap=min(m, 20_000))
        B = wl.dense(seed, A.k, n)
        C1, C2, (rp, ci, v, Bt) = _both(A, A.vals, B, n)
        ref, N = oracle_product(A.rowptr, A.colind, v, Bt, n)
        assert rel_err(C2, ref, N) <= TOL_F32
        assert rel_err(C1, ref, N) <= TOL_F32
        assert rel_err(C2, C1.astype(np.float64), N) <= 2 * TOL_F32
        # integer-valued inputs: both exact, so bitwise equal
        rng = np.random.default_rng(seed)
        vi = rng.integers(-8, 9, A.nnz).astype(np.float32)
        Bi = rng.integers(-8, 9, (A.k, n)).astype(np.float32)
        D1, D2, _ = _both(A, vi, Bi, n)
        assert np.array_equal(D1, D2)
        refi, _ = oracle_product(A.rowptr, A.colind, dev(vi), dev(Bi), n)
        assert np.array_equal(D2.astype(np.float64), refi)


def test_noalloc_empty_rows_and_refusal_on_gpu():
    """All rows empty (nnz = 0, merge-based) gives exact zeros; a workspace
    above the static scratch is refused before any launch, and a normal call
    right after it still works."""
    m, n = 7_000, 16
    rp = torch.zeros(m + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    v = torch.zeros(1, device="cuda")
    B = torch.ones(5, n, device="cuda")
    C = torch.full((m, n), float("nan"), device="cuda")
    nv.spmm_csr_noalloc(rp, ci, v, B, C, m, 5, 0, n, n)
    torch.cuda.synchronize()
    assert torch.equal(C, torch.zeros_like(C))
    with pytest.raises(nv.SpmmError) as ei:
        nv.spmm_csr_noalloc(rp, ci, v, B, C, 5_000_000, 5, 0, 4096, 4096)
    assert ei.value.status == nv.SPMM_ERR_UNSUPPORTED
    C.fill_(float("nan"))
    nv.spmm_csr_noalloc(rp, ci, v, B, C, m, 5, 0, n, n)
    torch.cuda.synchronize()
    assert torch.equal(C, torch.zeros_like(C))
