"""Seeded synthetic inputs shaped like the paper's SpMM workloads.

This module only draws inputs. It contains none of the SpMM arithmetic and is
the one piece of code that both the GPU tests/benchmark and the CPU oracle
consume (the oracle never imports it; tests hand its arrays to both sides).

The paper measures on SuiteSparse matrices, which are not available here; the
matrices below stand in for its regimes: short irregular rows (power law),
long regular rows (stencil), a graph-learning adjacency, and a batch of
uneven problems. Every generator is deterministic for a given seed (numpy
PCG64). Column indices are distinct and sorted within each row; rows may be
empty where the recipe allows it.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np


@dataclasses.dataclass
class CSR:
    """A in CSR: int32 row offsets (m+1), int32 column indices, values."""
    rowptr: np.ndarray
    colind: np.ndarray
    vals: np.ndarray
    m: int
    k: int

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.rowptr, self.colind, self.vals):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


def _rng(seed, stream=0):
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


def rowptr_from_lengths(lengths) -> np.ndarray:
    lengths = np.asarray(lengths, dtype=np.int64)
    rp = np.zeros(lengths.shape[0] + 1, dtype=np.int64)
    np.cumsum(lengths, out=rp[1:])
    if rp[-1] >= 2**31:
        raise ValueError("nnz must fit int32")
    return rp.astype(np.int32)


def distinct_sorted_columns(rng, lengths, k) -> np.ndarray:
    """Column indices for rows of the given lengths: per row a uniform random
    subset of [0, k) of that size, sorted ascending."""
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.size and lengths.max() > k:
        raise ValueError("row longer than k")
    m = lengths.shape[0]
    nnz = int(lengths.sum())
    out = np.empty(nnz, dtype=np.int32)
    if nnz == 0:
        return out
    offs = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=offs[1:])
    # Dense rows (more than a quarter of k) take a random permutation prefix.
    dense = np.nonzero(lengths * 4 > k)[0]
    sparse_mask = np.ones(nnz, dtype=bool)
    for r in dense:
        a, b = offs[r], offs[r + 1]
        out[a:b] = np.sort(rng.permutation(k)[: b - a])
        sparse_mask[a:b] = False
    idx = np.nonzero(sparse_mask)[0]
    if idx.size == 0:
        return out
    row_of = np.repeat(np.arange(m, dtype=np.int64), lengths)[idx]
    cols = rng.integers(0, k, idx.size, dtype=np.int64)
    while True:
        key = row_of * k + cols
        order = np.argsort(key, kind="stable")
        key = key[order]
        dup = np.zeros(key.shape[0], dtype=bool)
        dup[1:] = key[1:] == key[:-1]
        cols = key - row_of * k  # row_of is already grouped, so sorting keeps it
        nd = int(dup.sum())
        if nd == 0:
            break
        cols[dup] = rng.integers(0, k, nd, dtype=np.int64)
    out[idx] = cols.astype(np.int32)
    return out


def uniform(rng, shape, lo=-1.0, hi=1.0, dtype=np.float32):
    return rng.uniform(lo, hi, size=shape).astype(dtype)


def int_valued(rng, shape, lim=8, dtype=np.float32):
    """Integers in [-lim, lim]: exact in fp32/bf16/fp16, so every partial sum of
    a small product is exact and results are order-independent."""
    return rng.integers(-lim, lim + 1, size=shape).astype(dtype)


# --------------------------------------------------------------------------
# Row-length laws
# --------------------------------------------------------------------------

PARETO_SHAPE = 1.1  # survival exponent; pdf exponent 2.1 (Zipf 2.1)


def power_law_lengths(rng, m, mean=16.0, cap=100_000, shape=PARETO_SHAPE):
    """l_i = min(cap, floor(s * U_i^(-1/shape))), U_i in (0, 1], with the scale
    s chosen by bisection so that the realised mean is as close to ``mean`` as
    the integer steps allow."""
    u = 1.0 - rng.random(m)
    base = u ** (-1.0 / shape)

    def lens(s):
        return np.minimum(cap, np.floor(s * base)).astype(np.int64)

    lo, hi = 1e-6, float(mean) * 4.0
    while lens(hi).mean() < mean:
        hi *= 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if lens(mid).mean() < mean:
            lo = mid
        else:
            hi = mid
    l_lo, l_hi = lens(lo), lens(hi)
    best = l_lo if abs(l_lo.mean() - mean) <= abs(l_hi.mean() - mean) else l_hi
    return best, (lo if best is l_lo else hi)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def plain(seed=1001, m=4096, k=4096, per_row=16, values="uniform") -> CSR:
    """Uniform random pattern: ``per_row`` distinct columns in every row,
    values U[-1, 1) in fp32."""
    rng = _rng(seed, 0)
    lengths = np.full(m, per_row, dtype=np.int64)
    colind = distinct_sorted_columns(rng, lengths, k)
    vals = _values(rng, colind.shape[0], values)
    return CSR(rowptr_from_lengths(lengths), colind, vals, m, k)


def power_law(seed=1002, m=1_000_000, k=None, mean=16.0, cap=100_000, values="normal") -> CSR:
    """Power-law rows (Zipf exponent 2.1, mean ``mean``, capped), uniform
    random distinct columns, values N(0, 1) in fp32."""
    k = m if k is None else k
    rng = _rng(seed, 0)
    lengths, _ = power_law_lengths(rng, m, mean=mean, cap=min(cap, k))
    colind = distinct_sorted_columns(rng, lengths, k)
    vals = _values(rng, colind.shape[0], values)
    return CSR(rowptr_from_lengths(lengths), colind, vals, m, k)


def stencil27(seed=1003, g=128, values="stencil") -> CSR:
    """27-point stencil on a g^3 grid, row index x + g*y + g^2*z, no wrap at
    the boundary (boundary rows have 8..18 neighbours). Diagonal 26.0,
    off-diagonals -1.0 plus U(-1e-3, 1e-3) noise, fp32."""
    rng = _rng(seed, 0)
    m = g ** 3
    idx = np.arange(m, dtype=np.int64)
    x, y, z = idx % g, (idx // g) % g, idx // (g * g)
    cols = np.empty((m, 27), dtype=np.int32)
    ok = np.empty((m, 27), dtype=bool)
    t = 0
    for dz in (-1, 0, 1):          # offsets in increasing column order
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok[:, t] = ((x + dx >= 0) & (x + dx < g) & (y + dy >= 0) & (y + dy < g)
                            & (z + dz >= 0) & (z + dz < g))
                cols[:, t] = (idx + dx + g * dy + g * g * dz).astype(np.int32)
                t += 1
    lengths = ok.sum(axis=1)
    colind = cols[ok]
    del cols
    diag = (np.repeat(idx, lengths) == colind)
    if values == "stencil":
        vals = (-1.0 + rng.uniform(-1e-3, 1e-3, colind.shape[0])).astype(np.float32)
        vals[diag] = 26.0
    else:
        vals = _values(rng, colind.shape[0], values)
    return CSR(rowptr_from_lengths(lengths), colind, vals, m, m)


def grid_stencil(seed, dims, points, values="uniform") -> CSR:
    """Stencil matrix on a grid of the given dimensions (row index x + g0*y +
    g0*g1*z ...), no wrap at the boundary: `points` = 3^d takes every offset
    in {-1, 0, 1}^d (the 9- and 27-point stencils), `points` = 2d + 1 the
    axis neighbours only (the 5- and 7-point stencils). Columns ascend within
    each row."""
    import itertools
    rng = _rng(seed, 0)
    d = len(dims)
    m = int(np.prod(dims))
    idx = np.arange(m, dtype=np.int64)
    coord, stride, rem = [], [], idx
    s = 1
    for g in dims:
        coord.append(rem % g)
        rem = rem // g
        stride.append(s)
        s *= g
    if points == 3 ** d:
        offs = list(itertools.product((-1, 0, 1), repeat=d))
    elif points == 2 * d + 1:
        offs = [tuple(0 for _ in range(d))]
        for a in range(d):
            for sgn in (-1, 1):
                offs.append(tuple(sgn if b == a else 0 for b in range(d)))
    else:
        raise ValueError("points must be 3^d or 2d + 1")
    offs.sort(key=lambda o: sum(o[a] * stride[a] for a in range(d)))  # ascending columns
    cols = np.empty((m, len(offs)), dtype=np.int32)
    ok = np.ones((m, len(offs)), dtype=bool)
    for t, o in enumerate(offs):
        c = idx.copy()
        for a in range(d):
            ok[:, t] &= (coord[a] + o[a] >= 0) & (coord[a] + o[a] < dims[a])
            c += o[a] * stride[a]
        cols[:, t] = c.astype(np.int32)
    lengths = ok.sum(axis=1)
    colind = cols[ok]
    return CSR(rowptr_from_lengths(lengths), colind, _values(rng, colind.shape[0], values), m, m)


def banded(seed, m, per_row=16, half_band=512, values="uniform") -> CSR:
    """Each row holds `per_row` distinct random columns in a window of
    2 * half_band + 1 columns around its diagonal (shifted inward at the
    edges), ascending."""
    rng = _rng(seed, 0)
    width = 2 * half_band + 1
    if m < width:
        raise ValueError("m must be at least 2 * half_band + 1")
    lengths = np.full(m, per_row, dtype=np.int64)
    rel = distinct_sorted_columns(rng, lengths, width).astype(np.int64)
    lo = np.clip(np.arange(m, dtype=np.int64) - half_band, 0, m - width)
    colind = (np.repeat(lo, per_row) + rel).astype(np.int32)
    return CSR(rowptr_from_lengths(lengths), colind, _values(rng, colind.shape[0], values), m, m)


def chung_lu_graph(seed=1004, N=500_000, mean_deg=32.0, cap=100_000):
    """Undirected simple graph with power-law expected degrees: node weights
    from the same Pareto law as ``power_law`` (exponent 2.1), endpoints drawn
    in proportion to weight, self-loops dropped, duplicates merged, and exactly
    round(mean_deg * N / 2) edges kept. Returns (u, v) with u < v."""
    rng = _rng(seed, 0)
    u01 = 1.0 - rng.random(N)
    w = np.minimum(float(cap), u01 ** (-1.0 / PARETO_SHAPE))
    p = w / w.sum()
    target = int(round(mean_deg * N / 2.0))
    keys = np.empty(0, dtype=np.int64)
    batch = int(target * 1.25) + 16
    while keys.shape[0] < target:
        a = rng.choice(N, size=batch, p=p)
        b = rng.choice(N, size=batch, p=p)
        keep = a != b
        lo = np.minimum(a[keep], b[keep]).astype(np.int64)
        hi = np.maximum(a[keep], b[keep]).astype(np.int64)
        keys = np.unique(np.concatenate([keys, lo * N + hi]))
        batch = max(int((target - keys.shape[0]) * 2.0), 1024)
    if keys.shape[0] > target:
        keys = np.sort(rng.choice(keys, size=target, replace=False))
    return (keys // N).astype(np.int64), (keys % N).astype(np.int64)


def gcn_adjacency(seed=1004, N=500_000, mean_deg=32.0) -> CSR:
    """Symmetric normalised adjacency D^-1/2 (A + I) D^-1/2 of a Chung-Lu
    graph, D_ii = 1 + deg(i), values in fp64 (callers round to their storage
    type)."""
    u, v = chung_lu_graph(seed, N, mean_deg)
    loops = np.arange(N, dtype=np.int64)
    rows = np.concatenate([u, v, loops])
    cols = np.concatenate([v, u, loops])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    lengths = np.bincount(rows, minlength=N)
    deg = lengths.astype(np.float64)  # = 1 + number of neighbours
    vals = 1.0 / np.sqrt(deg[rows] * deg[cols])
    return CSR(rowptr_from_lengths(lengths), cols.astype(np.int32), vals, N, N)


def random_csr(seed, m, k, density=0.1, empty_frac=0.0, values="uniform",
               dtype=np.float32, dup_frac=0.0) -> CSR:
    """Small irregular matrix for edge cases: each row keeps Binomial(k,
    density) distinct columns, a fraction of rows is emptied, and optionally
    some rows receive duplicated column indices (which the product sums)."""
    rng = _rng(seed, 7)
    lengths = rng.binomial(k, density, size=m).astype(np.int64) if k > 0 else np.zeros(m, np.int64)
    if empty_frac > 0:
        lengths[rng.random(m) < empty_frac] = 0
    colind = distinct_sorted_columns(rng, lengths, k) if k > 0 else np.empty(0, np.int32)
    rowptr = rowptr_from_lengths(lengths)
    if dup_frac > 0 and colind.size:
        lens = lengths.copy()
        newcols = []
        for r in range(m):
            a, b = rowptr[r], rowptr[r + 1]
            row = list(colind[a:b])
            if row and rng.random() < dup_frac:
                row.append(row[int(rng.integers(0, len(row)))])
                rng.shuffle(row)
            newcols.extend(row)
            lens[r] = len(row)
        colind = np.asarray(newcols, dtype=np.int32)
        rowptr = rowptr_from_lengths(lens)
    vals = _values(rng, colind.shape[0], values).astype(dtype)
    return CSR(rowptr, colind, vals, m, k)


def fixed_density_device(seed, N, density, chunk=1000):
    """Square N x N matrix with L = max(1, round(density * N)) distinct
    uniformly random columns in every row (sorted), values U[-0.5, 0.5) -
    the sparse operand of the sparse-versus-dense comparison (Fig. 7). Built
    on the current GPU with a seeded torch generator (at 10 % of 100k x 100k
    it holds 1e9 entries); the same seed gives the same matrix. Returns
    (rowptr, colind, vals) as int32 / int32 / float32 device tensors and L."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    L = max(1, int(round(density * N)))
    parts = []
    for r0 in range(0, N, chunk):  # the L smallest of N random keys per row
        keys = torch.rand(min(chunk, N - r0), N, generator=g, device="cuda")
        parts.append(torch.topk(keys, L, dim=1, largest=False).indices.sort(dim=1).values
                     .to(torch.int32))
        del keys
    colind = torch.cat(parts).reshape(-1)
    del parts
    rowptr = torch.arange(0, (N + 1) * L, L, dtype=torch.int64, device="cuda").to(torch.int32)
    vals = torch.rand(N * L, generator=g, device="cuda") - 0.5
    return rowptr, colind, vals, L


def _values(rng, size, kind):
    if kind == "uniform":
        return uniform(rng, size)
    if kind == "normal":
        return rng.standard_normal(size, dtype=np.float32)
    if kind == "int":
        return int_valued(rng, size)
    if kind == "ones":
        return np.ones(size, dtype=np.float32)
    raise ValueError(kind)


def dense(seed, rows, cols, kind="uniform", stream=1, dtype=np.float32):
    """Dense row-major operand (B, dC, ...): U[-1, 1), N(0, 1) or integers."""
    rng = _rng(seed, stream)
    if kind == "uniform":
        return uniform(rng, (rows, cols), dtype=dtype)
    if kind == "normal":
        return rng.standard_normal((rows, cols), dtype=np.float32).astype(dtype)
    if kind == "int":
        return int_valued(rng, (rows, cols), dtype=dtype)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# Batch of uneven problems
# --------------------------------------------------------------------------

@dataclasses.dataclass
class BatchProblem:
    A: CSR
    n: int
    kind: str  # "uniform" or "zipf"


def batch_specs(seed=1005, count=512, m_lo=1_000, m_hi=200_000, n_choices=(8, 32, 128)):
    """Sizes of the uneven batch: m = k log-uniform in [m_lo, m_hi]; even
    problems have U{8..64} row lengths, odd ones the power-law law capped at
    min(1e5, k); n uniform over ``n_choices``."""
    rng = _rng(seed, 0)
    ms = np.rint(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi), count))).astype(np.int64)
    ns = rng.choice(np.asarray(n_choices), size=count)
    return [(int(m), int(n), "uniform" if b % 2 == 0 else "zipf")
            for b, (m, n) in enumerate(zip(ms, ns))]


def batch_problem(seed, b, m, kind, values="uniform") -> CSR:
    rng = _rng(seed, 100 + b)
    if kind == "uniform":
        lengths = rng.integers(8, 65, size=m).astype(np.int64)
        lengths = np.minimum(lengths, m)
    else:
        lengths, _ = power_law_lengths(rng, m, mean=16.0, cap=min(100_000, m))
    colind = distinct_sorted_columns(rng, lengths, m)
    vals = _values(rng, colind.shape[0], values)
    return CSR(rowptr_from_lengths(lengths), colind, vals, m, m)


def batch(seed=1005, count=512, m_lo=1_000, m_hi=200_000, n_choices=(8, 32, 128),
          values="uniform"):
    return [BatchProblem(batch_problem(seed, b, m, kind, values), n, kind)
            for b, (m, n, kind) in enumerate(batch_specs(seed, count, m_lo, m_hi, n_choices))]


def _batch_one(args):
    seed, b, m, kind, values = args
    return b, batch_problem(seed, b, m, kind, values)


def batch_parallel(seed=1005, count=512, m_lo=1_000, m_hi=200_000, n_choices=(8, 32, 128),
                   values="uniform", workers=None):
    """Same problems as ``batch``, generated by a process pool (each problem
    has its own random stream, so the result does not depend on workers).
    Workers are fresh interpreters (spawn), never forks of a process that may
    hold a GPU context."""
    import concurrent.futures
    import multiprocessing
    import os
    specs = batch_specs(seed, count, m_lo, m_hi, n_choices)
    workers = workers or min(16, len(os.sched_getaffinity(0)))
    out = [None] * count
    jobs = [(seed, b, m, kind, values) for b, (m, n, kind) in enumerate(specs)]
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        for b, A in ex.map(_batch_one, jobs, chunksize=4):
            out[b] = BatchProblem(A, specs[b][1], specs[b][2])
    return out
