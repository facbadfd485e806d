"""The sparse-versus-dense matrices (Fig. 7: 100k x 100k with a fixed number
of distinct random columns per row, n = 64) at 1 % and 10 % density, planned
by timing as the benchmark plans them, and with 8 and 16 column panels as
the benchmark's 2-D tiling measurement runs them: sampled rows of C against
the FP64 oracle on the same inputs."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import TOL_F32, rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N, n = 100_000, 64


def _oracle_rows(ci, vals, L, B, rows):
    """FP64 product and normaliser of the given rows (every row holds L
    entries, so row r is entries r L .. r L + L - 1)."""
    idx = (torch.as_tensor(rows, device="cuda")[:, None] * L
           + torch.arange(L, device="cuda")[None, :]).reshape(-1)
    c = ci[idx].cpu().numpy()
    v = vals[idx].cpu().numpy()
    rp = np.arange(0, (len(rows) + 1) * L, L, dtype=np.int32)
    ref = oracle.spmm(rp, c, v, B, n=n)
    N_ = oracle.spmm(rp, c, v, B, n=n, absval=True)
    return ref, N_


@pytest.mark.parametrize("density", [0.01, 0.1])
def test_crossover_matrix_sampled_rows(density):
    print(f"crossover density={density}", flush=True)
    rp, ci, vals, L = wl.fixed_density_device(11, N, density)
    B = wl.dense(12, N, n)
    Bt = torch.from_numpy(B).cuda()
    rng = np.random.default_rng(int(density * 1000))
    rows = np.unique(np.concatenate([[0, N - 1], rng.integers(0, N, 126)]))
    ref, Nrm = _oracle_rows(ci, vals, L, B, rows)
    C = torch.full((N, n), float("nan"), device="cuda")
    plan = nv.Plan(rp, ci, N, N, n, nnz=N * L, mode="autotune")
    plan.execute(vals, Bt, C)
    torch.cuda.synchronize()
    assert rel_err(C[torch.as_tensor(rows, device="cuda")].cpu().numpy(), ref, Nrm) <= TOL_F32
    print("autotuned shape", plan.info().config.as_dict(), flush=True)
    plan.close()
    # column panels as the benchmark times them (8 and 16 panels)
    for P in (8, 16):
        pl = nv.Plan(rp, ci, N, N, n, nnz=N * L,
                     config=dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, col_panels=P, lanes_per_row=64))
        C.fill_(float("nan"))
        pl.execute(vals, Bt, C)
        torch.cuda.synchronize()
        assert rel_err(C[torch.as_tensor(rows, device="cuda")].cpu().numpy(), ref, Nrm) <= TOL_F32
        pl.close()
