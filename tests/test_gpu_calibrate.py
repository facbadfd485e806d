"""The gather calibration kernel reads exactly the rows it is meant to: its
per-lane sums over an integer table equal a numpy replay of the same row
indices (a measurement aid; the products do not use it)."""
import numpy as np
import pytest
import torch

from paper_1803_08601_amd import native as nv

pytestmark = pytest.mark.gpu


def _mix(x):
    x = x.astype(np.uint64) & 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x7FEB352D) & 0xFFFFFFFF
    x ^= x >> 15
    x = (x * 0x846CA68B) & 0xFFFFFFFF
    x ^= x >> 16
    return x


@pytest.mark.parametrize("row_bytes", [32, 64, 128, 256, 512])
def test_calibrate_gather_reads_the_indexed_rows(row_bytes):
    rows, steps, threads = 64, 16, 512
    G = row_bytes // 16
    table = np.random.default_rng(row_bytes).integers(-8, 9, rows * row_bytes // 4).astype(np.float32)
    t = torch.from_numpy(table).cuda()
    out = torch.full((threads,), float("nan"), device="cuda")
    nv.spmm_calibrate_gather(t, rows, row_bytes, steps, out, threads)
    torch.cuda.synchronize()
    tid = np.arange(threads, dtype=np.uint64)
    grp, g = tid // G, tid % G
    quads = table.reshape(-1, 4).astype(np.float64)
    exp = np.zeros(threads)
    for it in range(steps):
        r = _mix(grp * 131 + (it * 0x9E3779B9 & 0xFFFFFFFF)) & (rows - 1)
        exp += quads[(r * G + g).astype(np.int64)].sum(axis=1)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), exp)
