"""Forward SpMM on the GPU (row split, merge-based, Sec. 5.4 choice, autotune)
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_08601_amd import native as nv
from paper_1803_08601_amd import workloads as wl
from spmm_check import DT, TOL_F32, TOL_STORAGE_16, dev, oracle_product, rel_err

pytestmark = pytest.mark.gpu

RS = nv.SPMM_KERNEL_ROWSPLIT
MG = nv.SPMM_KERNEL_MERGE
NZ = nv.SPMM_KERNEL_NZSPLIT
RB = nv.SPMM_KERNEL_ROWBLOCK


def _upload(A):
    return dev(A.rowptr), dev(A.colind)


def run(A, vals_t, B_t, n, ld=None, mode="paper", config=None, C=None):
    rp, ci = _upload(A)
    ld = n if ld is None else ld
    code = nv.dtype_code(B_t.dtype)
    plan = nv.Plan(rp, ci, A.m, A.k, n, ld=ld, dtype=code, mode=mode, config=config, nnz=A.nnz)
    if C is None:
        C = torch.full((A.m, ld), float("nan"), device="cuda")
    plan.execute(vals_t, B_t, C)
    torch.cuda.synchronize()
    return C, plan


def check(A, vals_t, B_t, n, C, tol=TOL_F32):
    Cref, N = oracle_product(A.rowptr, A.colind, vals_t, B_t, n)
    e = rel_err(C[:, :n].cpu().numpy(), Cref, N)
    assert e <= tol, f"max rel err {e}"
    return e


CONFIGS = [
    dict(kernel=RS, lanes_per_row=0, unroll=1),
    dict(kernel=RS, lanes_per_row=64, unroll=4),
    dict(kernel=RS, lanes_per_row=16, unroll=8),
    dict(kernel=MG, items_per_wg=64, unroll=1),
    dict(kernel=MG, items_per_wg=256, unroll=2),
    dict(kernel=MG, items_per_wg=1024, unroll=4),
    dict(kernel=MG, items_per_wg=4096, unroll=8),
    dict(kernel=RS, lanes_per_row=16, unroll=4, tile_cols=32),
    dict(kernel=MG, items_per_wg=512, unroll=4, tile_cols=32),
    dict(kernel=NZ, items_per_wg=64, unroll=1),
    dict(kernel=NZ, items_per_wg=256, unroll=2),
    dict(kernel=NZ, items_per_wg=2048, unroll=4),
    dict(kernel=NZ, items_per_wg=4096, unroll=8),
    dict(kernel=NZ, items_per_wg=512, unroll=4, tile_cols=32),
    dict(kernel=RB, rows_per_block=2, lanes_per_row=16, unroll=2),
    dict(kernel=RB, rows_per_block=4, unroll=4),
    dict(kernel=RB, rows_per_block=8, lanes_per_row=64, unroll=8),
    dict(kernel=RB, rows_per_block=4, lanes_per_row=8, unroll=1, tile_cols=32),
]


def cfg_id(c):
    return (f"{nv.KERNEL_NAMES[c['kernel']]}-{c.get('lanes_per_row', c.get('items_per_wg'))}"
            f"-u{c['unroll']}-t{c.get('tile_cols', 0)}-r{c.get('rows_per_block', 0)}")


@pytest.mark.parametrize("cfg", CONFIGS, ids=cfg_id)
@pytest.mark.parametrize("n", [1, 8, 32, 64, 100, 128, 512])
def test_plain_configs(cfg, n):
    A = wl.plain(m=1000, k=900)
    B = wl.dense(1001, A.k, n)
    C, plan = run(A, dev(A.vals), dev(B), n, config=cfg)
    check(A, dev(A.vals), dev(B), n, C)


@pytest.mark.parametrize("mode", ["autotune", "paper", "rule"])
def test_uniform_4096_workload_whole_output(mode):
    """The uniform 4096 x 4096 workload with 16 entries per row at n = 32 (the
    launch-bound case the benchmark times, planned the same way): the whole
    output against the oracle, and on integer values bit for bit."""
    A = wl.plain()
    assert (A.m, A.k, A.nnz) == (4096, 4096, 65536)
    n = 32
    B = wl.dense(1001, A.k, n)
    C, plan = run(A, dev(A.vals), dev(B), n, mode=mode)
    check(A, dev(A.vals), dev(B), n, C)
    Ai = wl.CSR(A.rowptr, A.colind,
                np.random.default_rng(5).integers(-8, 9, A.nnz).astype(np.float32), A.m, A.k)
    Bi = wl.dense(1002, A.k, n, kind="int")
    Ci = torch.full((A.m, n), float("nan"), device="cuda")
    plan.execute(dev(Ai.vals), dev(Bi), Ci)
    torch.cuda.synchronize()
    assert np.array_equal(Ci.cpu().numpy(), oracle.spmm(A.rowptr, A.colind, Ai.vals, Bi).astype(np.float32))
    plan.close()


@pytest.mark.parametrize("mode", ["paper", "rowsplit", "merge", "nzsplit", "rowblock", "autotune"])
def test_power_law_modes(mode):
    A = wl.power_law(seed=31, m=40_000, cap=20_000)
    for n in (8, 64):
        B = wl.dense(31, A.k, n)
        C, plan = run(A, dev(A.vals), dev(B), n, mode=mode)
        check(A, dev(A.vals), dev(B), n, C)
        info = plan.info()
        assert info.paper_choice == RS  # mean row length 16
        if mode == "merge":
            assert info.config.kernel == MG
        if mode == "nzsplit":
            assert info.config.kernel == NZ
        if mode == "rowblock":
            assert info.config.kernel == RB and info.config.rows_per_block == 2


@pytest.mark.parametrize("mode", ["rowsplit", "merge", "nzsplit", "rowblock", "autotune"])
def test_stencil_modes(mode):
    A = wl.stencil27(g=24)
    for n in (16, 128):
        B = wl.dense(1003, A.k, n)
        C, plan = run(A, dev(A.vals), dev(B), n, mode=mode)
        check(A, dev(A.vals), dev(B), n, C)
        if mode == "rowblock":
            assert plan.info().config.kernel == RB


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("cfg", CONFIGS, ids=cfg_id)
def test_integer_exact(dtype, cfg):
    """Integer values: every partial sum is exact, so any summation order must
    reproduce the oracle bit for bit (catches dropped or doubled partials)."""
    A = wl.power_law(seed=5, m=30_000, cap=30_000, values="int")
    n = 16
    B = wl.dense(5, A.k, n, kind="int")
    vt, Bt = dev(A.vals, DT[dtype]), dev(B, DT[dtype])
    C, _ = run(A, vt, Bt, n, config=cfg)
    Cref = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    assert np.array_equal(C.cpu().numpy().astype(np.float64), Cref)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("kernel", [RS, MG, NZ, RB])
def test_identity_permutation_diagonal_bitwise(kernel, dtype):
    """One product per output element, no additions: A = I gives B, a
    permutation gives B[pi], a diagonal gives diag * B, bit for bit (the
    16-bit inputs widen exactly)."""
    k, n = 3000, 32
    rng = np.random.default_rng(0)
    Bt = dev(rng.uniform(-1, 1, (k, n)).astype(np.float32), DT[dtype])
    B = Bt.float().cpu().numpy()
    I = np.arange(k + 1, dtype=np.int32)
    pi = rng.permutation(k).astype(np.int32)
    dt = dev(rng.uniform(-2, 2, k).astype(np.float32), DT[dtype])
    d = dt.float().cpu().numpy()
    ones = dev(np.ones(k, np.float32), DT[dtype])
    for cols, vt, expect in [(np.arange(k, dtype=np.int32), ones, B),
                             (pi, ones, B[pi]),
                             (np.arange(k, dtype=np.int32), dt, d[:, None] * B)]:
        A = wl.CSR(I, cols, np.ones(k, np.float32), k, k)
        C, _ = run(A, vt, Bt, n, config=dict(kernel=kernel))
        assert np.array_equal(C.cpu().numpy(), expect)


@pytest.mark.parametrize("kernel", [RS, MG, NZ, RB])
def test_power_of_two_scaling_and_empty_rows_bitwise(kernel):
    """(2^e A) B equals 2^e (A B) bit for bit (scaling by a power of two is
    exact and the plan fixes the summation order), and every empty row is
    +0.0 in every column."""
    A = wl.random_csr(31, 4000, 3000, density=0.01, empty_frac=0.4)
    n = 48
    B = wl.dense(31, A.k, n)
    C1, plan = run(A, dev(A.vals), dev(B), n, config=dict(kernel=kernel, items_per_wg=256))
    for e in (-3, 5):
        C2 = torch.empty_like(C1)
        plan.execute(dev(A.vals * np.float32(2.0 ** e)), dev(B), C2)
        torch.cuda.synchronize()
        assert torch.equal(C2, C1 * 2.0 ** e)
    empty = np.nonzero(A.row_lengths() == 0)[0]
    assert empty.size > 100
    bits = C1[torch.from_numpy(empty).cuda()].view(torch.int32)
    assert torch.all(bits == 0)  # +0.0, not -0.0


@pytest.mark.parametrize("W", [64, 100, 257, 1024, 4096])
def test_merge_partition_bit_exact(W):
    A = wl.power_law(seed=8, m=20_000, cap=10_000)
    _, plan = run(A, dev(A.vals), dev(wl.dense(8, A.k, 8)), 8, config=dict(kernel=MG, items_per_wg=W))
    got = plan.partition()
    assert np.array_equal(got, oracle.merge_partition(A.rowptr, W))


NZ_MATRICES = {
    "power_law": wl.power_law(seed=8, m=20_000, cap=10_000),
    "mostly_empty": wl.random_csr(21, 30_000, 5_000, density=0.002, empty_frac=0.95),
    "leading_trailing_empty": wl.CSR(np.array([0] * 700 + list(range(0, 3001, 3)) + [3000] * 900,
                                              np.int32),
                                     np.random.default_rng(3).integers(0, 400, 3000).astype(np.int32),
                                     np.random.default_rng(4).uniform(-1, 1, 3000).astype(np.float32),
                                     700 + 1000 + 900, 400),
    "no_entries": wl.random_csr(22, 5_000, 100, density=0.0),
}


@pytest.mark.parametrize("name", sorted(NZ_MATRICES))
@pytest.mark.parametrize("W", [64, 100, 1024, 4096])
def test_nz_partition_bit_exact_and_product(name, W):
    """Nonzero-split coordinates equal the oracle's bit for bit; the product
    is right also where a piece holds more than W row ends (runs of empty
    rows, whose ends the kernel reads from global memory instead of LDS)."""
    A = NZ_MATRICES[name]
    n = 24
    B = wl.dense(8, A.k, n)
    C, plan = run(A, dev(A.vals), dev(B), n, config=dict(kernel=NZ, items_per_wg=W))
    got = plan.partition()
    want = oracle.nz_partition(A.rowptr, W)
    assert np.array_equal(got, want)
    assert plan.info().num_parts == want.shape[0] - 1
    check(A, dev(A.vals), dev(B), n, C)


def test_row_sum_invariant_and_determinism():
    A = wl.power_law(seed=12, m=20_000, cap=20_000, values="uniform")
    ones = np.ones((A.k, 32), np.float32)
    for cfg in (dict(kernel=RS), dict(kernel=MG, items_per_wg=512), dict(kernel=NZ, items_per_wg=512),
                dict(kernel=RB, rows_per_block=8)):
        C1, plan = run(A, dev(A.vals), dev(ones), 32, config=cfg)
        C2 = torch.empty_like(C1)
        plan.execute(dev(A.vals), dev(ones), C2)
        assert torch.equal(C1, C2)
        c = C1.cpu().numpy()
        assert np.all(c == c[:, :1])  # every column is the same row sum
        rows = np.repeat(np.arange(A.m), A.row_lengths())
        s = np.bincount(rows, weights=A.vals.astype(np.float64), minlength=A.m)
        N = np.bincount(rows, weights=np.abs(A.vals.astype(np.float64)), minlength=A.m)
        assert rel_err(c[:, 0], s, N) <= TOL_F32


EDGE = {
    "empty_rows": wl.random_csr(1, 500, 300, density=0.05, empty_frac=0.7),
    "all_empty": wl.random_csr(2, 300, 50, density=0.0),
    "single_row": wl.CSR(np.array([0, 5000], np.int32),
                         np.sort(np.random.default_rng(0).choice(6000, 5000, replace=False)).astype(np.int32),
                         np.random.default_rng(1).uniform(-1, 1, 5000).astype(np.float32), 1, 6000),
    "giant_row_among_empty": wl.CSR(np.array([0, 0, 0, 20000, 20000, 20001], np.int32),
                                    np.concatenate([np.arange(20000), [3]]).astype(np.int32),
                                    np.random.default_rng(2).uniform(-1, 1, 20001).astype(np.float32),
                                    5, 20000),
    "k_is_1": wl.random_csr(3, 400, 1, density=0.5),
    "dups": wl.random_csr(4, 300, 200, density=0.1, dup_frac=0.5),
    "dense_rows": wl.random_csr(5, 40, 300, density=0.9),
}


@pytest.mark.parametrize("name", sorted(EDGE))
@pytest.mark.parametrize("kernel", [RS, MG, NZ, RB])
@pytest.mark.parametrize("n", [3, 16, 260])
def test_edge_cases(name, kernel, n):
    A = EDGE[name]
    B = wl.dense(9, max(A.k, 1), n)
    if kernel == RB and name == "dups":  # repeated columns in a row: refused
        with pytest.raises(nv.SpmmError) as ei:
            run(A, dev(A.vals), dev(B), n, config=dict(kernel=kernel))
        assert ei.value.status == nv.SPMM_ERR_UNSUPPORTED
        return
    C, _ = run(A, dev(A.vals), dev(B), n, config=dict(kernel=kernel, items_per_wg=128))
    check(A, dev(A.vals), dev(B), n, C)


def test_rowblock_terms_refusals_and_other_entry_points():
    """Row blocks: a row without a column takes no term for it (an infinite
    B row reaches only the rows that hold its column); rows whose columns do
    not strictly increase, or k >= 2^24, are refused, and timing then picks
    another kernel; semiring products, SDDMM and dB run on a row-block plan."""
    A = wl.stencil27(g=12)
    n = 16
    B = wl.dense(41, A.k, n)
    cstar = 5 + 12 * 6 + 144 * 6
    B[cstar, :] = np.inf
    for R in (2, 4, 8):
        C, plan = run(A, dev(A.vals), dev(B), n, config=dict(kernel=RB, rows_per_block=R))
        c = C.cpu().numpy()
        holds = np.zeros(A.m, bool)
        rows = np.repeat(np.arange(A.m), A.row_lengths())
        holds[rows[A.colind == cstar]] = True
        assert holds.sum() == 27 and np.all(np.isinf(c[holds]))
        Bf = B.copy()
        Bf[cstar, :] = 0.0
        Cref, N = oracle_product(A.rowptr, A.colind, dev(A.vals), dev(Bf), n)
        assert rel_err(c[~holds], Cref[~holds], N[~holds]) <= TOL_F32
        with pytest.raises(nv.SpmmError):
            plan.partition()
    # unsorted rows: refused when forced, another kernel when timed
    U = wl.random_csr(42, 800, 500, density=0.05)
    ci = U.colind.copy()
    r = int(np.argmax(U.row_lengths()))
    ci[U.rowptr[r]:U.rowptr[r + 1]] = ci[U.rowptr[r]:U.rowptr[r + 1]][::-1]
    Uu = wl.CSR(U.rowptr, ci, U.vals, U.m, U.k)
    Bu = wl.dense(43, U.k, 32)
    with pytest.raises(nv.SpmmError) as ei:
        run(Uu, dev(Uu.vals), dev(Bu), 32, mode="rowblock")
    assert ei.value.status == nv.SPMM_ERR_UNSUPPORTED
    C, plan = run(Uu, dev(Uu.vals), dev(Bu), 32, mode="autotune")
    assert plan.info().config.kernel != RB
    check(Uu, dev(Uu.vals), dev(Bu), 32, C)
    # k >= 2^24: refused before any launch
    big = wl.CSR(np.array([0, 1], np.int32), np.array([(1 << 24) + 5], np.int32),
                 np.ones(1, np.float32), 1, (1 << 24) + 10)
    with pytest.raises(nv.SpmmError) as ei:
        nv.Plan(dev(big.rowptr), dev(big.colind), 1, big.k, 4, config=dict(kernel=RB), nnz=1)
    assert ei.value.status == nv.SPMM_ERR_UNSUPPORTED
    # semiring, SDDMM and dB on a row-block plan
    S = wl.stencil27(g=10)
    n = 24
    Bs = wl.dense(44, S.k, n)
    dC = wl.dense(45, S.m, n, kind="normal")
    plan = nv.Plan(dev(S.rowptr), dev(S.colind), S.m, S.k, n, config=dict(kernel=RB), nnz=S.nnz)
    Cm = torch.empty(S.m, n, device="cuda")
    plan.execute_semiring(nv.SPMM_MIN_PLUS, dev(S.vals), dev(Bs), Cm)
    plan.transpose_build()
    dB = torch.empty(S.k, n, device="cuda")
    dv = torch.empty(S.nnz, device="cuda")
    plan.execute_t(dev(S.vals), dev(dC), dB)
    plan.sddmm(dev(dC), dev(Bs), dv)
    torch.cuda.synchronize()
    ref = oracle.spmm_semiring(S.rowptr, S.colind, S.vals, Bs, oracle.MIN_PLUS)
    assert np.array_equal(Cm.cpu().numpy(), ref.astype(np.float32))  # min and + are exact here
    rdB = oracle.spmm_t(S.rowptr, S.colind, S.vals, dC, S.k)
    NdB = oracle.spmm_t(S.rowptr, S.colind, S.vals, dC, S.k, absval=True)
    assert rel_err(dB.cpu().numpy(), rdB, NdB) <= TOL_F32
    rdv = oracle.sddmm(S.rowptr, S.colind, dC, Bs)
    Ndv = oracle.sddmm(S.rowptr, S.colind, dC, Bs, absval=True)
    assert rel_err(dv.cpu().numpy(), rdv, Ndv) <= TOL_F32


@pytest.mark.parametrize("kernel", [RS, MG, NZ])
def test_ld_padding_and_unaligned(kernel):
    A = wl.power_law(seed=13, m=5000, cap=2000)
    n, ld = 24, 40
    B = wl.dense(13, A.k, ld)
    Bt = dev(B)
    C = torch.full((A.m, ld), 7.0, device="cuda")
    rp, ci = _upload(A)
    plan = nv.Plan(rp, ci, A.m, A.k, n, ld=ld, config=dict(kernel=kernel))
    plan.execute(dev(A.vals), Bt, C)
    torch.cuda.synchronize()
    Cref, N = oracle_product(A.rowptr, A.colind, dev(A.vals), Bt, n)
    assert rel_err(C[:, :n].cpu().numpy(), Cref, N) <= TOL_F32
    assert torch.all(C[:, n:] == 7.0)  # padding untouched
    # B and C offset by one float: not 16-byte aligned, element access fallback
    Bflat = torch.zeros(A.k * ld + 1, device="cuda")
    Bflat[1:] = Bt.reshape(-1)
    Cflat = torch.zeros(A.m * ld + 1, device="cuda")
    plan.execute(dev(A.vals), Bflat[1:], Cflat[1:])
    torch.cuda.synchronize()
    C2 = Cflat[1:].reshape(A.m, ld)
    assert rel_err(C2[:, :n].cpu().numpy(), Cref, N) <= TOL_F32


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("kernel", [RS, MG, NZ])
def test_half_storage_errors(dtype, kernel):
    """Kernel error against the oracle on the rounded inputs (1e-5) and
    storage error against the original fp32 inputs (1e-2)."""
    A = wl.power_law(seed=14, m=30_000, cap=10_000, values="uniform")
    n = 64
    B = wl.dense(14, A.k, n)
    vt, Bt = dev(A.vals, DT[dtype]), dev(B, DT[dtype])
    C, _ = run(A, vt, Bt, n, config=dict(kernel=kernel))
    c = C.cpu().numpy()
    Cr, Nr = oracle_product(A.rowptr, A.colind, vt, Bt, n)
    assert rel_err(c, Cr, Nr) <= TOL_F32
    C32 = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    N32 = oracle.spmm(A.rowptr, A.colind, A.vals, B, absval=True)
    assert rel_err(c, C32, N32) <= TOL_STORAGE_16


def test_spmm_csr_one_call_and_cache():
    A = wl.power_law(seed=15, m=8000, cap=4000)
    n = 32
    B = wl.dense(15, A.k, n)
    rp, ci, v, Bt = dev(A.rowptr), dev(A.colind), dev(A.vals), dev(B)
    C = torch.empty(A.m, n, device="cuda")
    nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)
    nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)  # cached plan
    torch.cuda.synchronize()
    check(A, v, Bt, n, C)
    nv.spmm_cache_clear()
    with pytest.raises(nv.SpmmError):
        nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n - 1)


def test_streams_and_threads():
    """Plans run on two streams at once and the one-call entry point used from
    two host threads give the same results as serial runs (plan workspaces
    are per plan; the plan cache and registry are locked)."""
    import threading
    mats = [wl.power_law(seed=61, m=30_000, cap=10_000), wl.stencil27(g=24)]
    n = 32
    data = []
    for A in mats:
        B = wl.dense(62, A.k, n)
        rp, ci, v, Bt = dev(A.rowptr), dev(A.colind), dev(A.vals), dev(B)
        data.append((A, rp, ci, v, Bt))
    ref = []
    for A, rp, ci, v, Bt in data:
        C = torch.empty(A.m, n, device="cuda")
        nv.Plan(rp, ci, A.m, A.k, n, nnz=A.nnz, mode="rule").execute(v, Bt, C)
        torch.cuda.synchronize()
        ref.append(C)
    plans = [nv.Plan(rp, ci, A.m, A.k, n, nnz=A.nnz, mode="rule") for A, rp, ci, v, Bt in data]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(A.m, n, device="cuda") for A, *_ in data]
    for rep in range(3):
        for (A, rp, ci, v, Bt), plan, st, C in zip(data, plans, streams, outs):
            with torch.cuda.stream(st):
                plan.execute(v, Bt, C, stream=st.cuda_stream)
        torch.cuda.synchronize()
        for C, R in zip(outs, ref):
            assert torch.equal(C, R)
    # the one-call path plans without row blocks, so its serial result (not
    # mode RULE's) is the reference for the threaded calls
    ref1 = []
    for A, rp, ci, v, Bt in data:
        C = torch.empty(A.m, n, device="cuda")
        nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)
        torch.cuda.synchronize()
        ref1.append(C)
    nv.spmm_cache_clear()
    res = [None, None]
    def work(i):
        A, rp, ci, v, Bt = data[i]
        C = torch.empty(A.m, n, device="cuda")
        for _ in range(3):
            nv.spmm_csr(rp, ci, v, Bt, C, A.m, A.k, n, n)
        torch.cuda.synchronize()
        res[i] = C
    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for C, R in zip(res, ref1):
        assert torch.equal(C, R)


def test_shape_limits_and_degenerate_plans():
    """The largest merge pieces (8192 items: 108 KB of LDS in FP32, 116 KB
    with 16-bit storage, within gfx950's 160 KB per workgroup) give the right
    product; larger ones are refused with SPMM_ERR_UNSUPPORTED before any
    launch; plans with no rows, one column or no entries work for every
    kernel."""
    A = wl.power_law(seed=71, m=6000, cap=3000)
    n = 64
    B = wl.dense(71, A.k, n)
    for dt in ("f32", "bf16"):
        for kern in (MG, NZ):
            vt, Bt = dev(A.vals, DT[dt]), dev(B, DT[dt])
            C, _ = run(A, vt, Bt, n, config=dict(kernel=kern, items_per_wg=8192))
            check(A, vt, Bt, n, C)
    with pytest.raises(nv.SpmmError) as ei:
        run(A, dev(A.vals), dev(B), n, config=dict(kernel=MG, items_per_wg=16384))
    assert ei.value.status == nv.SPMM_ERR_UNSUPPORTED
    for kern in (RS, MG, NZ):
        empty = wl.CSR(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32), 0, 10)
        Ce = torch.empty(0, 8, device="cuda")
        run(empty, dev(np.zeros(1, np.float32)), dev(wl.dense(1, 10, 8)), 8, config=dict(kernel=kern),
            C=Ce)
        one_col = wl.random_csr(72, 500, 1, density=0.7)
        C1, _ = run(one_col, dev(one_col.vals), dev(wl.dense(2, 1, 1)), 1, config=dict(kernel=kern))
        check(one_col, dev(one_col.vals), dev(wl.dense(2, 1, 1)), 1, C1)


def test_validate():
    A = wl.random_csr(6, 100, 80, density=0.1)
    rp, ci = dev(A.rowptr), dev(A.colind)
    nv.spmm_csr_validate(rp, ci, A.m, A.k, A.nnz)
    with pytest.raises(nv.SpmmError):
        nv.spmm_csr_validate(rp, ci, A.m, A.k - 79, A.nnz)
    bad = A.rowptr.copy()
    bad[50] = bad[51] + 1
    with pytest.raises(nv.SpmmError):
        nv.spmm_csr_validate(dev(bad), ci, A.m, A.k, A.nnz)


def test_plan_methods_refuse_bad_tensors():
    """The Python plan checks dtype, device and extent before any launch: a
    tensor too short for rows of stride ld, a wrong dtype, a host tensor or a
    view with other strides raises ValueError and leaves C untouched."""
    A = wl.random_csr(7, 120, 90, density=0.1)
    n, ld = 6, 10
    plan = nv.Plan(dev(A.rowptr), dev(A.colind), A.m, A.k, n, ld=ld, nnz=A.nnz)
    vals, B = dev(A.vals), torch.ones(A.k, ld, device="cuda")
    C = torch.full((A.m, ld), 3.0, device="cuda")
    bad = [
        (vals[:-1], B, C),                                   # vals shorter than nnz
        (vals.to(torch.bfloat16), B, C),                     # dtype of another plan
        (vals, torch.ones(A.k, n, device="cuda"), C),        # B rows of stride n < ld
        (vals, B.to(torch.float16), C),
        (vals, B, torch.empty(A.m, n, device="cuda")),       # C too short for stride ld
        (vals, B, C.to(torch.float64)),
        (vals.cpu(), B, C),                                  # host memory
        (vals, B.t().contiguous().t(), C),                   # column-major view
    ]
    for v, b_, c in bad:
        with pytest.raises(ValueError):
            plan.execute(v, b_, c)
    dv = torch.empty(A.nnz, device="cuda")
    with pytest.raises(ValueError):
        plan.sddmm(torch.empty(A.m, n, device="cuda"), B, dv)
    with pytest.raises(ValueError):
        plan.sddmm(torch.empty(A.m, ld, device="cuda"), B, dv[:-1])
    torch.cuda.synchronize()
    assert torch.all(C == 3.0)
    # accepted: contiguous memory read as rows of stride ld, and (ld, 1) views
    plan.execute(vals, B.reshape(-1), C)
    plan.execute(vals, B, torch.empty(A.m, 2 * ld, device="cuda")[:, :ld].contiguous())
    big = torch.full((A.m, ld + 4), 5.0, device="cuda")
    with pytest.raises(ValueError):
        plan.execute(vals, B, big[:, :ld])                   # stride ld + 4, not ld


def test_rule_mode_choice():
    """The MI355X rule: merge-based for power-law rows (a row of >= 4096
    entries) or a mean below 4; row blocks of 2 rows for sorted rows whose
    pairs share columns (at most 0.9 distinct columns per entry) when
    n >= 32; row split otherwise."""
    S = wl.stencil27(g=20)
    ci = S.colind.copy()
    ci[S.rowptr[5]:S.rowptr[6]] = ci[S.rowptr[5]:S.rowptr[6]][::-1]  # one row out of order
    S_unsorted = wl.CSR(S.rowptr, ci, S.vals, S.m, S.k)
    cases = [(wl.power_law(seed=51, m=40_000, cap=20_000), 16, MG),
             (S, 16, RS),
             (S, 64, RB),
             (wl.grid_stencil(3, (300, 300), 5), 32, RB),
             (S_unsorted, 64, RS),
             (wl.plain(m=2000, k=2000), 64, RS),
             (wl.random_csr(8, 5000, 4000, density=0.0005), 64, MG)]
    for A, n, want in cases:
        B = wl.dense(5, A.k, n)
        C, plan = run(A, dev(A.vals), dev(B), n, mode="rule")
        info = plan.info()
        assert info.config.kernel == want, (A.m, n)
        if want == RB:
            assert info.config.rows_per_block == 2
        check(A, dev(A.vals), dev(B), n, C)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_rowsplit_infinite_b_row_reaches_only_its_rows(dtype):
    """Row split never lets a step past a row's last entry touch the sum: with
    B row 0 infinite, only the rows that hold column 0 are infinite, and every
    other row matches the oracle - for every team width and unroll (rows of
    8 to 27 entries leave partial blocks of U steps) and with column panels."""
    A = wl.stencil27(g=12)
    n = 16
    B = wl.dense(46, A.k, n)
    B[0, :] = np.inf
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    holds = np.zeros(A.m, bool)
    holds[rows[A.colind == 0]] = True
    Bf = B.copy()
    Bf[0, :] = 0.0
    vt, Bt, Bft = dev(A.vals, DT[dtype]), dev(B, DT[dtype]), dev(Bf, DT[dtype])
    Cref, N = oracle_product(A.rowptr, A.colind, vt, Bft, n)
    tol = TOL_F32
    for lpr in (4, 16, 64):
        for u in (2, 4, 8):
            for P in (0, 3):
                cfg = dict(kernel=nv.SPMM_KERNEL_ROWSPLIT, lanes_per_row=lpr, unroll=u,
                           col_panels=P)
                C, plan = run(A, vt, Bt, n, config=cfg)
                c = C.cpu().numpy()
                assert holds.sum() == 8 and np.all(np.isinf(c[holds]))
                assert np.all(np.isfinite(c[~holds]))
                assert rel_err(c[~holds], Cref[~holds], N[~holds]) <= tol, (lpr, u, P)
