"""Autotuner results across processes: a shape loaded from a tune-cache file
is the one a later autotuned plan of the same matrix takes (no trials), and
its product still matches the FP64 oracle."""
import pytest
import torch

from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import TOL_F32, dev, oracle_product, rel_err

pytestmark = pytest.mark.gpu


def test_loaded_shape_is_used(tmp_path):
    A = wl.power_law(seed=71, m=20_000, cap=5_000)
    n = 32
    B = wl.dense(71, A.k, n)
    rp, ci, v, Bt = dev(A.rowptr), dev(A.colind), dev(A.vals), dev(B)
    first = nv.Plan(rp, ci, A.m, A.k, n, nnz=A.nnz, mode="autotune")
    tuned = first.info().config.as_dict()
    first.close()
    f = tmp_path / "tune.txt"
    nv.spmm_tune_cache_save(str(f))
    # replace this matrix's entry by another valid shape: row split, whole
    # wavefront per row, unroll 1
    rows = f.read_text().splitlines()
    key = [r for r in rows[1:] if r.split()[1:4] == [str(A.m), str(A.k), str(A.nnz)]]
    assert len(key) == 1
    parts = key[0].split()
    forced = {"kernel": nv.SPMM_KERNEL_ROWSPLIT, "vec": 4, "lanes_per_row": 64, "unroll": 1,
              "items_per_wg": 1024, "tile_cols": 0, "rows_per_block": 0, "tile_order": 0,
              "col_panels": 0}
    assert forced != tuned
    # 13 key fields, then the 9 config fields
    parts[13:22] = [str(forced[k]) for k in ("kernel", "vec", "lanes_per_row", "unroll",
                                             "items_per_wg", "tile_cols", "rows_per_block",
                                             "tile_order", "col_panels")]
    f.write_text(rows[0] + "\n" + " ".join(parts) + "\n")
    nv.spmm_tune_cache_load(str(f))
    plan = nv.Plan(rp, ci, A.m, A.k, n, nnz=A.nnz, mode="autotune")
    assert plan.info().config.as_dict() == forced
    C = torch.empty(A.m, n, device="cuda")
    plan.execute(v, Bt, C)
    torch.cuda.synchronize()
    ref, N = oracle_product(A.rowptr, A.colind, v, Bt, n)
    assert rel_err(C.cpu().numpy(), ref, N) <= TOL_F32
    plan.close()
