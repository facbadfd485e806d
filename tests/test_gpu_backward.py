"""Backward pass on the GPU: CSR transpose (bit-exact), dB = A^T dC, SDDMM,
and the autograd Function, against the FP64 oracle, central differences and
the identities of the bilinear loss L = <dC, A B>."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from paper_1803_08601_amd.autograd import spmm
from spmm_check import DT, TOL_F32, TOL_STORAGE_16, dev, host_bits, rel_err

pytestmark = pytest.mark.gpu

RS, MG, NZ = nv.SPMM_KERNEL_ROWSPLIT, nv.SPMM_KERNEL_MERGE, nv.SPMM_KERNEL_NZSPLIT


def make_plan(A, n, dtype="f32", kernel=None, mode="paper"):
    rp, ci = dev(A.rowptr), dev(A.colind)
    cfg = None if kernel is None else dict(kernel=kernel)
    return nv.Plan(rp, ci, A.m, A.k, n, dtype=nv.dtype_code(DT[dtype]), mode=mode, config=cfg,
                   nnz=A.nnz)


MATS = {
    "random_empty": lambda: wl.random_csr(1, 700, 500, density=0.03, empty_frac=0.4),
    "power_law": lambda: wl.power_law(seed=21, m=30_000, cap=8_000),
    "k_is_1": lambda: wl.random_csr(2, 300, 1, density=0.6),
    "dups": lambda: wl.random_csr(3, 200, 150, density=0.1, dup_frac=0.6),
    "wide": lambda: wl.random_csr(4, 50, 70_000, density=0.01),
    "gcn": lambda: wl.gcn_adjacency(N=3_000, mean_deg=12),
    "empty": lambda: wl.random_csr(5, 40, 30, density=0.0),
}


@pytest.mark.parametrize("name", sorted(MATS))
def test_transpose_bit_exact(name):
    A = MATS[name]()
    plan = make_plan(A, 8)
    plan.transpose_build()
    assert plan.info().has_transpose
    at_rp = torch.empty(A.k + 1, dtype=torch.int32, device="cuda")
    at_ci = torch.empty(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    perm = torch.empty(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    nv.spmm_transpose_get(plan.handle, at_rp, at_ci, perm)
    torch.cuda.synchronize()
    e_rp, e_ci, e_perm = oracle.transpose(A.rowptr, A.colind, A.k)
    assert np.array_equal(at_rp.cpu().numpy(), e_rp)
    assert np.array_equal(at_ci.cpu().numpy()[:A.nnz], e_ci)
    assert np.array_equal(perm.cpu().numpy()[:A.nnz], e_perm)


@pytest.mark.parametrize("name", ["random_empty", "power_law", "gcn"])
def test_transpose_twice_is_identity(name):
    """The transpose of the transpose reproduces A's CSR bit for bit (columns
    are sorted within rows), and the two value permutations compose to the
    identity."""
    A = MATS[name]()
    plan = make_plan(A, 8)
    plan.transpose_build()
    at_rp = torch.empty(A.k + 1, dtype=torch.int32, device="cuda")
    at_ci = torch.empty(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    perm = torch.empty(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    nv.spmm_transpose_get(plan.handle, at_rp, at_ci, perm)
    plan2 = nv.Plan(at_rp, at_ci, A.k, A.m, 8, nnz=A.nnz, mode="paper")
    plan2.transpose_build()
    rp2 = torch.empty(A.m + 1, dtype=torch.int32, device="cuda")
    ci2 = torch.empty(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    perm2 = torch.empty(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    nv.spmm_transpose_get(plan2.handle, rp2, ci2, perm2)
    torch.cuda.synchronize()
    assert np.array_equal(rp2.cpu().numpy(), A.rowptr)
    assert np.array_equal(ci2.cpu().numpy()[:A.nnz], A.colind)
    p1, p2 = perm.cpu().numpy()[:A.nnz], perm2.cpu().numpy()[:A.nnz]
    assert np.array_equal(p1[p2], np.arange(A.nnz))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("name", ["random_empty", "power_law", "dups", "gcn", "wide"])
@pytest.mark.parametrize("n", [3, 16, 128, 300])
def test_grad_b_and_vals_vs_oracle(dtype, name, n):
    A = MATS[name]()
    rng = np.random.default_rng(n)
    B = rng.uniform(-1, 1, (A.k, n)).astype(np.float32)
    dC = rng.standard_normal((A.m, n)).astype(np.float32)
    vt, Bt, dCt = dev(A.vals.astype(np.float32), DT[dtype]), dev(B, DT[dtype]), dev(dC)
    plan = make_plan(A, n, dtype)
    plan.transpose_build()
    dB = torch.full((A.k, n), float("nan"), device="cuda")
    plan.execute_t(vt, dCt, dB)
    dv = torch.full((max(A.nnz, 1),), float("nan"), device="cuda")
    plan.sddmm(dCt, Bt, dv)
    torch.cuda.synchronize()
    v, vtag = host_bits(vt)
    b, btag = host_bits(Bt)
    ref_dB = oracle.spmm_t(A.rowptr, A.colind, v, dC, A.k, vals_tag=vtag)
    N_dB = oracle.spmm_t(A.rowptr, A.colind, v, dC, A.k, vals_tag=vtag, absval=True)
    assert rel_err(dB.cpu().numpy(), ref_dB, N_dB) <= TOL_F32
    # the transpose-free scatter form of the same product
    dBs = torch.full((A.k, n), float("nan"), device="cuda")
    plan.execute_t_scatter(vt, dCt, dBs)
    torch.cuda.synchronize()
    assert rel_err(dBs.cpu().numpy(), ref_dB, N_dB) <= TOL_F32
    ref_dv = oracle.sddmm(A.rowptr, A.colind, dC, b, b_tag=btag)
    N_dv = oracle.sddmm(A.rowptr, A.colind, dC, b, b_tag=btag, absval=True)
    assert rel_err(dv.cpu().numpy()[:A.nnz], ref_dv, N_dv) <= TOL_F32
    if dtype != "f32":  # storage error against the unrounded inputs
        r32 = oracle.sddmm(A.rowptr, A.colind, dC, B)
        n32 = oracle.sddmm(A.rowptr, A.colind, dC, B, absval=True)
        assert rel_err(dv.cpu().numpy()[:A.nnz], r32, n32) <= TOL_STORAGE_16


@pytest.mark.parametrize("kernel", [RS, MG, NZ])
@pytest.mark.parametrize("n", [5, 32, 300])
def test_scatter_transpose_free(kernel, n):
    """dB = A^T dC by atomic scatter on A's CSR, without spmm_transpose_build:
    integer data exact whatever the order of the additions; padding columns
    of dB untouched; repeated calls overwrite (dB is zeroed by the call)."""
    A = wl.power_law(seed=19, m=12_000, cap=6_000, values="int")
    dC = wl.dense(20, A.m, n, kind="int")
    ld = n + 3
    dCp = np.zeros((A.m, ld), np.float32)
    dCp[:, :n] = dC
    plan = nv.Plan(dev(A.rowptr), dev(A.colind), A.m, A.k, n, ld=ld, nnz=A.nnz,
                   config=dict(kernel=kernel))
    assert not plan.info().has_transpose
    dB = torch.full((A.k, ld), 7.0, device="cuda")
    ref = oracle.spmm_t(A.rowptr, A.colind, A.vals, dC, A.k)
    for _ in range(2):
        plan.execute_t_scatter(dev(A.vals), dev(dCp), dB)
        torch.cuda.synchronize()
        assert np.array_equal(dB[:, :n].cpu().numpy(), ref)
    assert torch.all(dB[:, n:] == 7.0)


@pytest.mark.parametrize("kernel,mode", [(RS, "paper"), (MG, "paper"), (NZ, "paper"),
                                         (None, "nzsplit"), (None, "rowblock")])
def test_backward_integer_exact(kernel, mode):
    """Integer data: dB and dvals bit for bit. With mode nzsplit the plan of
    A^T uses the nonzero split too; SDDMM walks diagonal pieces either way."""
    A = wl.power_law(seed=9, m=20_000, cap=20_000, values="int")
    n = 32
    B = wl.dense(9, A.k, n, kind="int")
    dC = wl.dense(10, A.m, n, kind="int")
    plan = make_plan(A, n, kernel=kernel, mode=mode)
    plan.transpose_build()
    dB = torch.empty(A.k, n, device="cuda")
    dv = torch.empty(A.nnz, device="cuda")
    plan.execute_t(dev(A.vals), dev(dC), dB)
    plan.sddmm(dev(dC), dev(B), dv)
    torch.cuda.synchronize()
    assert np.array_equal(dB.cpu().numpy(), oracle.spmm_t(A.rowptr, A.colind, A.vals, dC, A.k))
    assert np.array_equal(dv.cpu().numpy(), oracle.sddmm(A.rowptr, A.colind, dC, B))


def test_symmetric_adjacency_transpose_equals_forward():
    """For the symmetric normalised adjacency, A^T has A's CSR exactly, so
    A^T dC through the transpose equals the forward product on dC bit for bit."""
    A = wl.gcn_adjacency(N=20_000, mean_deg=16)
    A.vals = A.vals.astype(np.float32)
    n = 64
    dC = wl.dense(3, A.m, n, kind="normal")
    plan = make_plan(A, n)
    plan.transpose_build()
    dB = torch.empty(A.k, n, device="cuda")
    plan.execute_t(dev(A.vals), dev(dC), dB)
    C = torch.empty(A.m, n, device="cuda")
    plan.execute(dev(A.vals), dev(dC), C)
    torch.cuda.synchronize()
    assert torch.equal(dB, C)
    # D^1/2 1 is an eigenvector with eigenvalue 1
    x = np.repeat(np.sqrt(A.row_lengths().astype(np.float64))[:, None], n, axis=1)
    plan.execute(dev(A.vals), dev(x.astype(np.float32)), C)
    torch.cuda.synchronize()
    N = oracle.spmm(A.rowptr, A.colind, np.abs(A.vals), x.astype(np.float32))
    assert rel_err(C.cpu().numpy(), x.astype(np.float32).astype(np.float64), N) <= 1e-5 + 2**-23


def test_autograd_central_differences_64_nodes():
    """L is linear in vals and in B, so central differences with step 1 along
    +-1 directions equal the directional derivative exactly (up to fp32
    rounding of the two forward products)."""
    A = wl.gcn_adjacency(N=64, mean_deg=8)
    A.vals = A.vals.astype(np.float32)
    n = 16
    rng = np.random.default_rng(4)
    B = rng.uniform(-1, 1, (A.k, n)).astype(np.float32)
    dC = rng.standard_normal((A.m, n)).astype(np.float32)
    plan = make_plan(A, n)
    vt = dev(A.vals).requires_grad_(True)
    Bt = dev(B).requires_grad_(True)
    dCt = dev(dC)
    L = (spmm(plan, vt, Bt) * dCt).sum()
    L.backward()
    gv, gB = vt.grad.cpu().numpy().astype(np.float64), Bt.grad.cpu().numpy().astype(np.float64)
    # oracle gradients (FP64)
    assert np.allclose(gv, oracle.sddmm(A.rowptr, A.colind, dC, B), rtol=0, atol=1e-5 * n)
    assert np.allclose(gB, oracle.spmm_t(A.rowptr, A.colind, A.vals, dC, A.k), rtol=0, atol=1e-5 * 8)

    def Lgpu(v, b):
        C = torch.empty(A.m, n, device="cuda")
        plan.execute(dev(v), dev(b), C)
        return float((C.double() * dCt.double()).sum())

    scale = float(np.abs(dC).sum() * 8)
    for _ in range(3):
        d = rng.choice([-1.0, 1.0], size=A.nnz).astype(np.float32)
        fd = (Lgpu(A.vals + d, B) - Lgpu(A.vals - d, B)) / 2.0
        assert abs(fd - float(gv @ d)) <= 1e-5 * scale
        D = rng.choice([-1.0, 1.0], size=B.shape).astype(np.float32)
        fd = (Lgpu(A.vals, B + D) - Lgpu(A.vals, B - D)) / 2.0
        assert abs(fd - float((gB * D).sum())) <= 1e-5 * scale


def test_autograd_bf16_and_euler():
    A = wl.gcn_adjacency(N=5_000, mean_deg=16)
    n = 128
    rng = np.random.default_rng(6)
    B = rng.uniform(-1, 1, (A.k, n)).astype(np.float32)
    dC = rng.standard_normal((A.m, n)).astype(np.float32)
    plan = make_plan(A, n, "bf16")
    vt = dev(A.vals.astype(np.float32), torch.bfloat16).requires_grad_(True)
    Bt = dev(B, torch.bfloat16).requires_grad_(True)
    C = spmm(plan, vt, Bt)
    assert C.dtype == torch.float32
    (C * dev(dC)).sum().backward()
    assert vt.grad.dtype == torch.bfloat16 and Bt.grad.dtype == torch.bfloat16
    # Euler identities of the bilinear loss, in fp32 on the device results
    plan32 = plan
    dv = torch.empty(A.nnz, device="cuda")
    plan32.sddmm(dev(dC), Bt.detach(), dv)
    dB = torch.empty(A.k, n, device="cuda")
    plan32.execute_t(vt.detach(), dev(dC), dB)
    L = float((C.detach().double() * dev(dC).double()).sum())
    e1 = float((dB.double() * Bt.detach().double()).sum())
    e2 = float((dv.double() * vt.detach().double()).sum())
    scale = float((C.detach().abs().double() * dev(dC).abs().double()).sum())
    assert abs(e1 - L) <= 1e-5 * scale and abs(e2 - L) <= 1e-5 * scale
    # gradient values against the oracle on the bf16 inputs (storage error of the bf16 cast)
    v, vtag = host_bits(vt.detach())
    b, btag = host_bits(Bt.detach())
    ref = oracle.sddmm(A.rowptr, A.colind, dC, b, b_tag=btag)
    N = oracle.sddmm(A.rowptr, A.colind, dC, b, b_tag=btag, absval=True)
    assert rel_err(vt.grad.float().cpu().numpy(), ref, N) <= TOL_STORAGE_16
