"""Pins for the FP64 CPU oracle: each check compares it with something other
than itself (a hand-worked example, numpy/scipy/torch routines, closed forms,
exact integer arithmetic, brute force), so that a dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1803_08601_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_of(A: wl.CSR):
    """Dense copy of A with duplicate entries summed (numpy scatter-add)."""
    D = np.zeros((A.m, A.k), dtype=np.float64)
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    np.add.at(D, (rows, A.colind.astype(np.int64)), A.vals.astype(np.float64))
    return D


def scipy_of(A: wl.CSR, dtype=np.float64):
    return sp.csr_matrix((A.vals.astype(dtype), A.colind, A.rowptr), shape=(A.m, A.k))


# ---------------------------------------------------------------- worked example

def test_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    rp = np.array(g["rowptr"], np.int32)
    ci = np.array(g["colind"], np.int32)
    v = np.array(g["vals"], np.float64)
    B = np.array(g["B"], np.float64)
    dC = np.array(g["dC"], np.float64)
    assert np.array_equal(oracle.spmm(rp, ci, v, B), np.array(g["C"], float))
    assert np.array_equal(oracle.spmm(rp, ci, v, B, absval=True), np.array(g["absnorm"], float))
    assert np.array_equal(oracle.merge_walk(rp), np.array(g["merge_walk"]))
    assert np.array_equal(oracle.merge_partition(rp, g["W"]), np.array(g["merge_partition"]))
    assert np.array_equal(oracle.sddmm(rp, ci, dC, B), np.array(g["dvals"], float))
    assert np.array_equal(oracle.spmm_t(rp, ci, v, dC, g["k"]), np.array(g["dB"], float))
    at_rp, at_ci, perm = oracle.transpose(rp, ci, g["k"])
    assert at_rp.tolist() == g["at_rowptr"] and at_ci.tolist() == g["at_colind"]
    assert perm.tolist() == g["perm"]
    assert oracle.heuristic_merge(g["m"], len(g["colind"])) == g["heuristic_merge"]
    C = oracle.spmm(rp, ci, v, B)
    assert float((dC * C).sum()) == g["L"]


# ---------------------------------------------------------------- product

@pytest.mark.parametrize("seed", range(12))
def test_spmm_matches_dense_gemm(seed):
    rng = np.random.default_rng(seed)
    m, k, n = int(rng.integers(1, 65)), int(rng.integers(1, 65)), int(rng.integers(1, 40))
    dens = float(rng.choice([0.0, 0.05, 0.3, 0.7, 1.0]))
    A = wl.random_csr(seed, m, k, density=dens, empty_frac=0.2, dtype=np.float64,
                      dup_frac=0.3 if seed % 2 else 0.0)
    B = rng.uniform(-1, 1, (k, n))
    C = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    ref = dense_of(A) @ B
    N = np.abs(dense_of(A)) @ np.abs(B)
    assert np.all(np.abs(C - ref) <= 1e-13 * N + 1e-300)
    Nor = oracle.spmm(A.rowptr, A.colind, A.vals, B, absval=True)
    if seed % 2 == 0:  # without duplicates |A| has the same pattern as A
        assert np.allclose(Nor, N, rtol=1e-13, atol=0)


def test_spmm_ld_and_column_subset():
    A = wl.random_csr(3, 20, 30, density=0.2)
    B = np.random.default_rng(0).uniform(-1, 1, (30, 12))
    full = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    part = oracle.spmm(A.rowptr, A.colind, A.vals, B, n=7)  # ld = 12, n = 7
    assert np.array_equal(part, full[:, :7])


def test_spmm_vs_scipy_power_law():
    A = wl.power_law(seed=1002, m=60_000, cap=5_000)
    B = wl.dense(1002, A.k, 8)
    C = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    ref = scipy_of(A) @ B.astype(np.float64)
    N = oracle.spmm(A.rowptr, A.colind, A.vals, B, absval=True)
    assert np.all(np.abs(C - ref) <= 1e-12 * N)


def test_spmm_vs_scipy_stencil():
    A = wl.stencil27(seed=1003, g=20)
    assert A.nnz == (3 * 20 - 2) ** 3
    B = wl.dense(1003, A.k, 16)
    C = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    ref = scipy_of(A) @ B.astype(np.float64)
    N = oracle.spmm(A.rowptr, A.colind, A.vals, B, absval=True)
    assert np.all(np.abs(C - ref) <= 1e-12 * N)


def test_spmm_vs_scipy_plain():
    A = wl.plain()
    B = wl.dense(1001, A.k, 32)
    C = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    ref = scipy_of(A) @ B.astype(np.float64)
    N = oracle.spmm(A.rowptr, A.colind, A.vals, B, absval=True)
    assert np.all(np.abs(C - ref) <= 1e-12 * N)


def test_identity_permutation_diagonal_exact():
    rng = np.random.default_rng(5)
    k, n = 50, 9
    B = rng.uniform(-1, 1, (k, n)).astype(np.float32)
    I = np.arange(k + 1, dtype=np.int32)
    assert np.array_equal(oracle.spmm(I, np.arange(k, dtype=np.int32), np.ones(k, np.float32), B),
                          B.astype(np.float64))
    pi = rng.permutation(k).astype(np.int32)
    assert np.array_equal(oracle.spmm(I, pi, np.ones(k, np.float32), B), B[pi].astype(np.float64))
    d = rng.uniform(-2, 2, k).astype(np.float32)
    assert np.array_equal(oracle.spmm(I, np.arange(k, dtype=np.int32), d, B),
                          d[:, None].astype(np.float64) * B.astype(np.float64))


def test_row_sum_invariant():
    A = wl.random_csr(11, 200, 150, density=0.1, empty_frac=0.1, values="int")
    ones = np.ones((A.k, 5), np.float32)
    C = oracle.spmm(A.rowptr, A.colind, A.vals, ones)
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    expect = np.bincount(rows, weights=A.vals.astype(np.float64), minlength=A.m)
    assert np.array_equal(C, np.repeat(expect[:, None], 5, axis=1))


def test_integer_exact_against_int64_scipy():
    A = wl.power_law(seed=7, m=20_000, cap=2_000, values="int")
    B = wl.dense(7, A.k, 16, kind="int")
    C = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    Ai = sp.csr_matrix((A.vals.astype(np.int64), A.colind, A.rowptr), shape=(A.m, A.k))
    exact = Ai @ B.astype(np.int64)
    assert np.array_equal(C, exact.astype(np.float64))


def test_linearity():
    A = wl.random_csr(4, 80, 70, density=0.2)
    rng = np.random.default_rng(4)
    B1, B2 = rng.uniform(-1, 1, (70, 6)), rng.uniform(-1, 1, (70, 6))
    s = oracle.spmm(A.rowptr, A.colind, A.vals, B1 + B2)
    t = oracle.spmm(A.rowptr, A.colind, A.vals, B1) + oracle.spmm(A.rowptr, A.colind, A.vals, B2)
    N = oracle.spmm(A.rowptr, A.colind, A.vals, np.abs(B1) + np.abs(B2), absval=True)
    assert np.all(np.abs(s - t) <= 1e-13 * N)
    v4 = A.vals.astype(np.float64) * 4.0
    assert np.array_equal(oracle.spmm(A.rowptr, A.colind, v4, B1),
                          4.0 * oracle.spmm(A.rowptr, A.colind, A.vals.astype(np.float64), B1))


def test_rows_subset_and_thread_invariance():
    A = wl.power_law(seed=9, m=30_000, cap=3_000)
    B = wl.dense(9, A.k, 8)
    C1 = oracle.spmm(A.rowptr, A.colind, A.vals, B, nthreads=1)
    C8 = oracle.spmm(A.rowptr, A.colind, A.vals, B, nthreads=8)
    assert np.array_equal(C1, C8)
    rows = np.array([0, 17, 29_999, 5, 5], np.int64)
    assert np.array_equal(oracle.spmm_rows(A.rowptr, A.colind, A.vals, B, rows), C1[rows])


# ---------------------------------------------------------------- storage decoders

def test_bf16_and_f16_decoders_all_patterns():
    torch = pytest.importorskip("torch")
    bits = np.arange(65536, dtype=np.uint16)
    got16 = oracle.decode(bits, oracle.F16)
    ref16 = bits.view(np.float16).astype(np.float64)
    ok = ~np.isnan(ref16)
    assert np.array_equal(got16[ok], ref16[ok]) and np.all(np.isnan(got16[~ok]))
    gotb = oracle.decode(bits, oracle.BF16)
    refb = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).double().numpy()
    ok = ~np.isnan(refb)
    assert np.array_equal(gotb[ok], refb[ok]) and np.all(np.isnan(gotb[~ok]))


def test_bf16_inputs_widened_exactly():
    torch = pytest.importorskip("torch")
    A = wl.random_csr(21, 40, 30, density=0.3)
    B = np.random.default_rng(21).uniform(-1, 1, (30, 8)).astype(np.float32)
    vb = torch.from_numpy(A.vals).bfloat16()
    Bb = torch.from_numpy(B).bfloat16()
    got = oracle.spmm(A.rowptr, A.colind, vb.view(torch.int16).numpy().view(np.uint16),
                      Bb.view(torch.int16).numpy().view(np.uint16), vals_tag=oracle.BF16,
                      b_tag=oracle.BF16)
    ref = oracle.spmm(A.rowptr, A.colind, vb.double().numpy(), Bb.double().numpy())
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- backward

def test_spmm_t_and_sddmm_vs_dense():
    rng = np.random.default_rng(3)
    for seed in range(6):
        A = wl.random_csr(seed, 30 + seed, 25, density=0.25, empty_frac=0.1, dtype=np.float64)
        dC = rng.standard_normal((A.m, 7))
        B = rng.uniform(-1, 1, (A.k, 7))
        D = dense_of(A)
        dB = oracle.spmm_t(A.rowptr, A.colind, A.vals, dC, A.k)
        assert np.allclose(dB, D.T @ dC, rtol=0, atol=1e-13 * (np.abs(D.T) @ np.abs(dC)).max())
        dv = oracle.sddmm(A.rowptr, A.colind, dC, B)
        rows = np.repeat(np.arange(A.m), A.row_lengths())
        full = dC @ B.T
        assert np.allclose(dv, full[rows, A.colind], rtol=1e-13, atol=1e-13)


def test_gradients_euler_identities():
    """L(vals, B) = <dC, A B> is linear in vals and in B, so
    <dB, B> = <dvals, vals> = L."""
    A = wl.gcn_adjacency(seed=1004, N=300, mean_deg=8)
    rng = np.random.default_rng(1)
    B = rng.uniform(-1, 1, (A.k, 16))
    dC = rng.standard_normal((A.m, 16))
    C = oracle.spmm(A.rowptr, A.colind, A.vals, B)
    L = float((dC * C).sum())
    dB = oracle.spmm_t(A.rowptr, A.colind, A.vals, dC, A.k)
    dv = oracle.sddmm(A.rowptr, A.colind, dC, B)
    assert abs(float((dB * B).sum()) - L) <= 1e-12 * max(1.0, abs(L))
    assert abs(float((dv * A.vals).sum()) - L) <= 1e-12 * max(1.0, abs(L))


def test_gradients_central_differences_exact():
    """Bilinear loss: central differences with step 1 along +-1 directions are
    exact in real arithmetic, so they pin the gradient formulas."""
    A = wl.gcn_adjacency(seed=1004, N=64, mean_deg=8)
    rng = np.random.default_rng(2)
    B = rng.uniform(-1, 1, (A.k, 4))
    dC = rng.standard_normal((A.m, 4))

    def L(vals, BB):
        return float((dC * oracle.spmm(A.rowptr, A.colind, vals, BB)).sum())

    dB = oracle.spmm_t(A.rowptr, A.colind, A.vals, dC, A.k)
    dv = oracle.sddmm(A.rowptr, A.colind, dC, B)
    for _ in range(4):
        v = rng.choice([-1.0, 1.0], size=A.vals.shape)
        fd = (L(A.vals + v, B) - L(A.vals - v, B)) / 2.0
        assert abs(fd - float(dv @ v)) <= 1e-10
        V = rng.choice([-1.0, 1.0], size=B.shape)
        fd = (L(A.vals, B + V) - L(A.vals, B - V)) / 2.0
        assert abs(fd - float((dB * V).sum())) <= 1e-10


def test_gcn_normalised_adjacency_eigenvector():
    """D^-1/2 (A+I) D^-1/2 applied to D^1/2 1 gives D^1/2 1."""
    A = wl.gcn_adjacency(seed=1004, N=2_000, mean_deg=12)
    lens = A.row_lengths().astype(np.float64)
    x = np.sqrt(lens)[:, None] * np.ones((1, 3))
    C = oracle.spmm(A.rowptr, A.colind, A.vals, x)
    assert np.allclose(C, x, rtol=1e-12, atol=0)
    s = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.m, A.k))
    assert abs(s - s.T).max() == 0.0  # symmetric pattern and values


# ---------------------------------------------------------------- transpose

@pytest.mark.parametrize("seed", range(5))
def test_transpose_vs_scipy(seed):
    A = wl.random_csr(seed, 50 + 3 * seed, 40, density=0.15, empty_frac=0.2)
    A.vals = np.arange(1, A.nnz + 1, dtype=np.float64)  # distinct, identifies each entry
    at_rp, at_ci, perm = oracle.transpose(A.rowptr, A.colind, A.k)
    T = scipy_of(A).T.tocsr()
    T.sort_indices()
    assert np.array_equal(at_rp, T.indptr) and np.array_equal(at_ci, T.indices)
    assert np.array_equal(A.vals[perm], T.data)
    back_rp, back_ci, back_perm = oracle.transpose(at_rp, at_ci, A.m)
    assert np.array_equal(back_rp, A.rowptr) and np.array_equal(back_ci, A.colind)
    assert np.array_equal(perm[back_perm], np.arange(A.nnz))


# ---------------------------------------------------------------- merge path

def _adversarial():
    cases = {
        "empty_rows": np.zeros(9, np.int32),
        "one_giant_row": np.array([0, 0, 0, 500, 500, 500], np.int32),
        "single_row": np.array([0, 37], np.int32),
        "no_rows": np.array([0], np.int32),
        "all_len_1": np.arange(21, dtype=np.int32),
    }
    for s in range(6):
        A = wl.random_csr(s, 60, 80, density=[0.0, 0.02, 0.1, 0.5, 0.9, 0.3][s], empty_frac=0.3)
        cases[f"random{s}"] = A.rowptr
    A = wl.power_law(seed=3, m=2_000, cap=1_000)
    cases["power_law"] = A.rowptr
    return cases


@pytest.mark.parametrize("name,rowptr", list(_adversarial().items()))
def test_merge_walk_invariants_and_search(name, rowptr):
    m = rowptr.shape[0] - 1
    nnz = int(rowptr[-1])
    walk = oracle.merge_walk(rowptr)
    d = np.arange(m + nnz + 1)
    assert np.array_equal(walk[:, 0] + walk[:, 1], d)
    assert np.all(np.diff(walk[:, 0]) >= 0) and np.all(np.diff(walk[:, 1]) >= 0)
    assert tuple(walk[0]) == (0, 0) and tuple(walk[-1]) == (m, nnz)
    inside = walk[:, 0] < m
    i = walk[inside, 0]
    assert np.all(rowptr[i] <= walk[inside, 1]) and np.all(walk[inside, 1] <= rowptr[i + 1])
    # a step increases i exactly when the item is a row end, which happens
    # exactly m times, once per row, at j = rowptr[i+1]
    steps_i = np.nonzero(np.diff(walk[:, 0]) == 1)[0]
    assert steps_i.shape[0] == m
    assert np.array_equal(walk[steps_i, 1], rowptr[1:])
    for dd in range(m + nnz + 1):
        assert oracle.merge_search(rowptr, dd) == tuple(walk[dd])
    for W in (1, 2, 3, 7, 64, 1000):
        part = oracle.merge_partition(rowptr, W)
        P = oracle.merge_num_parts(m, nnz, W)
        assert part.shape[0] == P + 1
        dp = np.minimum(np.arange(P + 1) * W, m + nnz)
        assert np.array_equal(part, walk[dp])


def test_merge_closed_forms():
    for m in (0, 1, 5, 33):
        w = oracle.merge_walk(np.zeros(m + 1, np.int32))
        assert np.array_equal(w, np.stack([np.arange(m + 1), np.zeros(m + 1, int)], 1))
    for nnz in (0, 1, 40):
        w = oracle.merge_walk(np.array([0, nnz], np.int32))
        exp = [(0, d) for d in range(nnz + 1)] + [(1, nnz)]
        assert [tuple(x) for x in w] == exp
    m = 25
    w = oracle.merge_walk(np.arange(m + 1, dtype=np.int32))
    d = np.arange(2 * m + 1)
    assert np.array_equal(w[:, 0], d // 2) and np.array_equal(w[:, 1], d - d // 2)


# ---------------------------------------------------------------- nonzero split

@pytest.mark.parametrize("name,rowptr", list(_adversarial().items()))
def test_nz_partition_against_merge_walk(name, rowptr):
    """Piece p of the nonzero split starts at the last merge state whose
    nonzero coordinate is min(p*W, nnz): the state from which nonzero p*W is
    the next item (all row ends up to it, empty rows included, are taken
    first). The merge walk is pinned on its own above."""
    m = rowptr.shape[0] - 1
    nnz = int(rowptr[-1])
    walk = oracle.merge_walk(rowptr)
    last_at_j = {}
    for i, j in walk:
        last_at_j[int(j)] = int(i)
    for W in (1, 2, 3, 7, 64, 1000):
        part = oracle.nz_partition(rowptr, W)
        P = oracle.nz_num_parts(m, nnz, W)
        assert part.shape[0] == P + 1
        if m == 0:
            assert P == 0 and tuple(part[0]) == (0, 0)
            continue
        assert P == max(1, -(-nnz // W))
        assert tuple(part[0]) == (0, 0) and tuple(part[-1]) == (m, nnz)
        # equal nonzeros per piece, the last one takes the rest
        assert np.array_equal(part[:, 1], np.minimum(np.arange(P + 1) * W, nnz))
        for p in range(1, P):
            i, j = part[p]
            assert i == last_at_j[int(j)]
            # row i holds nonzero j (the 1-D search on the row offsets)
            assert rowptr[i] <= j < rowptr[i + 1]
        assert np.all(np.diff(part[:, 0]) >= 0)


def test_nz_partition_closed_forms():
    # constant row length L, no empty rows: piece p starts in row p*W // L
    for m, L, W in ((100, 3, 7), (64, 16, 64), (10, 1, 4), (33, 5, 5)):
        rp = np.arange(0, (m + 1) * L, L, dtype=np.int32)
        part = oracle.nz_partition(rp, W)
        P = part.shape[0] - 1
        assert P == -(-(m * L) // W)
        for p in range(P):
            assert tuple(part[p]) == ((p * W) // L, p * W)
        assert tuple(part[P]) == (m, m * L)
    # no nonzeros: one piece of m empty rows
    assert oracle.nz_partition(np.zeros(6, np.int32), 4).tolist() == [[0, 0], [5, 0]]
    # leading empty rows stay in the first piece; trailing ones in the last
    rp = np.array([0, 0, 0, 4, 4, 8, 8, 8], np.int32)
    assert oracle.nz_partition(rp, 4).tolist() == [[0, 0], [4, 4], [7, 8]]
    assert oracle.nz_partition(rp, 2).tolist() == [[0, 0], [2, 2], [4, 4], [4, 6], [7, 8]]


# ---------------------------------------------------------------- heuristic

@pytest.mark.parametrize("m,nnz,merge", [
    (20, 187, False),         # d = 9.35 exactly: not below the threshold
    (20, 186, True),          # d = 9.30
    (100, 935, False), (100, 934, True),
    (4096, 65536, False),     # d = 16
    (1_000_000, 16_000_000, False),
    (2_097_152, 55_742_968, False),
    (10, 0, True), (1, 9, True), (1, 10, False),
    (0, 0, False),
])
def test_heuristic_table(m, nnz, merge):
    assert oracle.heuristic_merge(m, nnz) == merge


# ---------------------------------------------------------------- semirings

def _dense_with(A, fill):
    D = np.full((A.m, A.k), fill, dtype=np.float64)
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    D[rows, A.colind] = A.vals
    return D


@pytest.mark.parametrize("seed", range(6))
def test_semirings_brute_force(seed):
    """Brute force over every (i, j, c) with numpy broadcasting; missing
    entries take the value that never wins (+inf for min, -inf for max)."""
    rng = np.random.default_rng(seed)
    A = wl.random_csr(seed, 30, 25, density=0.2, empty_frac=0.2, dtype=np.float64)
    B = rng.uniform(-2, 2, (25, 6))
    C = oracle.spmm_semiring(A.rowptr, A.colind, A.vals, B, oracle.PLUS_TIMES)
    assert np.allclose(C, dense_of(A) @ B, rtol=1e-13, atol=1e-13)
    C = oracle.spmm_semiring(A.rowptr, A.colind, A.vals, B, oracle.MIN_PLUS)
    assert np.array_equal(C, np.min(_dense_with(A, np.inf)[:, :, None] + B[None], axis=1))
    C = oracle.spmm_semiring(A.rowptr, A.colind, A.vals, B, oracle.MAX_PLUS)
    assert np.array_equal(C, np.max(_dense_with(A, -np.inf)[:, :, None] + B[None], axis=1))
    D = _dense_with(A, np.nan)
    prod = np.where(np.isnan(D)[:, :, None], -np.inf, np.nan_to_num(D)[:, :, None] * B[None])
    C = oracle.spmm_semiring(A.rowptr, A.colind, A.vals, B, oracle.MAX_TIMES)
    assert np.array_equal(C, np.max(prod, axis=1))


def test_min_plus_bellman_ford_matches_scipy_shortest_paths():
    """Repeated min-plus products relax distances (Bellman-Ford); after |V|
    rounds they equal scipy's shortest-path distances."""
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(3)
    N = 40
    A = wl.random_csr(3, N, N, density=0.1)
    A.vals = rng.integers(1, 10, A.nnz).astype(np.float64)
    # A^T as CSR: row v lists its in-edges (u, w), so d'[v] = min_u w(u,v) + d[u]
    at_rp, at_ci, perm = oracle.transpose(A.rowptr, A.colind, N)
    at_v = A.vals[perm]
    src = [0, 5, 17]
    d = np.full((N, len(src)), np.inf)
    d[src, np.arange(len(src))] = 0.0
    for _ in range(N):
        relax = oracle.spmm_semiring(at_rp, at_ci, at_v, d, oracle.MIN_PLUS)
        d = np.minimum(d, relax)
    ref = shortest_path(scipy_of(A), method="BF", directed=True, indices=src).T
    assert np.array_equal(d, ref)


def test_native_build_is_bitwise_the_test_build(tmp_path):
    """The CPU baseline times an -O3 -march=native build of the oracle; it
    must compute exactly what the pinned test build computes (same double
    additions in CSR order), at one thread and at all threads."""
    native = oracle.native_build(str(tmp_path / "liboracle_native.so"))
    for A, n in ((wl.power_law(seed=41, m=20_000, cap=5_000), 64),
                 (wl.stencil27(g=16), 16),
                 (wl.random_csr(42, 3000, 2000, density=0.01, empty_frac=0.2, dup_frac=0.1), 7)):
        B = wl.dense(43, A.k, n)
        ref = oracle.spmm(A.rowptr, A.colind, A.vals, B, nthreads=1)
        for th in (1, 0):
            got = oracle.spmm(A.rowptr, A.colind, A.vals, B, nthreads=th, library=native)
            assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
