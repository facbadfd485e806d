"""Execute calls captured into a graph: each enqueues only kernels (no
allocation, no memset, no host synchronisation), so a torch.cuda.CUDAGraph
capture of it replays the same work. Every replay - with other eager work
and host synchronisations in between, and C refilled with NaN first - must
equal the eager call bit for bit, and a replay after the values change in
place must equal the eager call on the new values. Integer-valued inputs
keep every sum exact, so kernels whose summation order is not fixed (the
atomic dB scatter) compare bitwise too."""
import numpy as np
import pytest
import torch

from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import dev

pytestmark = pytest.mark.gpu

RS, MG, NZ, RB = (nv.SPMM_KERNEL_ROWSPLIT, nv.SPMM_KERNEL_MERGE, nv.SPMM_KERNEL_NZSPLIT,
                  nv.SPMM_KERNEL_ROWBLOCK)


def _int_csr(A, seed):
    v = np.random.default_rng(seed).integers(-4, 5, A.nnz).astype(np.float32)
    return wl.CSR(A.rowptr, A.colind, v, A.m, A.k)


def _replays(run, outs, vals):
    """Eager result of run(), then a captured run() replayed three times and
    once more after vals doubles in place."""
    nan = float("nan")
    for o in outs:
        o.fill_(nan)
    run()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    for o in outs:
        o.fill_(nan)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    torch.cuda.synchronize()
    x = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        for o in outs:
            o.fill_(nan)
        y = x @ x  # other eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), f"replay {rep}"
    vals.mul_(2)
    for o in outs:
        o.fill_(nan)
    run()
    torch.cuda.synchronize()
    eager2 = [o.clone() for o in outs]
    for o in outs:
        o.fill_(nan)
    g.replay()
    torch.cuda.synchronize()
    for o, e in zip(outs, eager2):
        assert torch.equal(o, e), "replay after the values changed"
    vals.div_(2)
    del g


POWER = _int_csr(wl.power_law(seed=81, m=30_000, cap=8_000), 81)
SHORT = _int_csr(wl.power_law(seed=82, m=30_000, mean=4.0, cap=2_000), 82)
STENCIL = _int_csr(wl.stencil27(seed=83, g=24), 83)
LONG = _int_csr(wl.random_csr(84, 600, 40_000, density=0.05), 84)

FORWARD = [
    ("rowsplit", POWER, dict(kernel=RS)),
    ("merge", POWER, dict(kernel=MG, items_per_wg=512)),
    ("merge-short", SHORT, dict(kernel=MG, items_per_wg=1024)),
    ("nzsplit", SHORT, dict(kernel=NZ, items_per_wg=256)),
    ("rowblock", STENCIL, dict(kernel=RB, rows_per_block=4)),
    ("rowsplit-strips", STENCIL, dict(kernel=RS, tile_order=2)),
    ("panels", LONG, dict(kernel=RS, col_panels=4)),
    ("tiles", POWER, dict(kernel=MG, items_per_wg=512, tile_cols=16)),
]


@pytest.mark.parametrize("name,A,cfg", FORWARD, ids=[f[0] for f in FORWARD])
@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16])
def test_forward_replays(name, A, cfg, dt):
    n = 32
    B = dev(wl.dense(85, A.k, n, kind="int"), dt)
    vals = dev(A.vals, dt)
    C = torch.empty(A.m, n, device="cuda")
    plan = nv.Plan(dev(A.rowptr), dev(A.colind), A.m, A.k, n, dtype=nv.dtype_code(dt),
                   config=cfg, nnz=A.nnz)
    _replays(lambda: plan.execute(vals, B, C), [C], vals)
    plan.close()


@pytest.mark.parametrize("kernel", [RS, MG])
def test_semiring_backward_and_sddmm_replays(kernel):
    """(min,+) product, dB = A^T dC through the transpose, the atomic dB
    scatter and SDDMM, all four in one graph."""
    A = POWER
    n = 24
    B = dev(wl.dense(86, A.k, n, kind="int"))
    dC = dev(wl.dense(87, A.m, n, kind="int"))
    vals = dev(A.vals)
    plan = nv.Plan(dev(A.rowptr), dev(A.colind), A.m, A.k, n, config=dict(kernel=kernel),
                   nnz=A.nnz)
    plan.transpose_build()
    Cm = torch.empty(A.m, n, device="cuda")
    dB = torch.empty(A.k, n, device="cuda")
    dB2 = torch.empty(A.k, n, device="cuda")
    dv = torch.empty(A.nnz, device="cuda")

    def run():
        plan.execute_semiring(nv.SPMM_MIN_PLUS, vals, B, Cm)
        plan.execute_t(vals, dC, dB)
        plan.execute_t_scatter(vals, dC, dB2)
        plan.sddmm(dC, B, dv)

    _replays(run, [Cm, dB, dB2, dv], vals)
    assert torch.equal(dB, dB2)
    plan.close()


def test_noalloc_replays():
    """The one-call entry point that allocates nothing (merge-based here: its
    partition, carry-outs and fix-up all run from static scratch)."""
    A = SHORT
    n = 16
    rp, ci, vals = dev(A.rowptr), dev(A.colind), dev(A.vals)
    B = dev(wl.dense(88, A.k, n, kind="int"))
    C = torch.empty(A.m, n, device="cuda")
    _replays(lambda: nv.spmm_csr_noalloc(rp, ci, vals, B, C, A.m, A.k, A.nnz, n, n), [C], vals)


def test_sddmm_without_columns_replays():
    """SDDMM with n = 0 (every dot product empty) writes zeros by a kernel,
    so a captured call clears dvals again on every replay."""
    A = POWER
    rp, ci = dev(A.rowptr), dev(A.colind)
    plan = nv.Plan(rp, ci, A.m, A.k, 0, ld=1, nnz=A.nnz)
    dv = torch.empty(A.nnz, device="cuda")
    _replays(lambda: nv.spmm_sddmm(plan.handle, None, None, dv), [dv], torch.zeros(1, device="cuda"))
    assert torch.all(dv == 0)
    plan.close()
