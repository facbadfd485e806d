"""Shared helpers for the GPU parity tests: device transfer and the error
measure against the FP64 oracle.

Error measure (per element, reported as the maximum): |C_gpu - C_ref| / N with
N = |A| |B| (sum of |a| |b| over the terms of each element); where N is zero
the GPU value must be exactly zero. Float32 bound: the sum of l products in
float32 is within l * 2^-24 * N of the exact value in the worst case and
about 2^-24 * N for random signs, so 1e-5 leaves a wide margin at every row
length used here. BF16/FP16 storage: rounding both inputs costs at most
(2 u + u^2) N with u = 2^-8 (bf16), i.e. below 7.9e-3 N, hence 1e-2.
"""
import numpy as np
import torch

import oracle

TOL_F32 = 1e-5
TOL_STORAGE_16 = 1e-2
DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
TAG = {"f32": oracle.F32, "bf16": oracle.BF16, "f16": oracle.F16}


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host_bits(t):
    """Host copy of a device tensor in the form the oracle takes (fp32 array
    or 16-bit patterns) plus its oracle tag."""
    t = t.detach().cpu().contiguous()
    if t.dtype == torch.float32:
        return t.numpy(), oracle.F32
    if t.dtype == torch.float64:
        return t.numpy(), oracle.F64
    tag = oracle.BF16 if t.dtype == torch.bfloat16 else oracle.F16
    return t.view(torch.int16).numpy().view(np.uint16), tag


def rel_err(C_gpu, C_ref, N):
    C_gpu = np.asarray(C_gpu, dtype=np.float64)
    diff = np.abs(C_gpu - C_ref)
    zero = N == 0
    if np.any(C_gpu[zero] != 0):
        return np.inf
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(zero, 0.0, diff / np.where(zero, 1.0, N))
    return float(r.max()) if r.size else 0.0


def oracle_product(rowptr, colind, vals_t, B_t, n, rows=None):
    """FP64 product and normaliser from the exact device inputs."""
    v, vt = host_bits(vals_t)
    b, bt = host_bits(B_t)
    if rows is None:
        C = oracle.spmm(rowptr, colind, v, b, n=n, vals_tag=vt, b_tag=bt)
        N = oracle.spmm(rowptr, colind, v, b, n=n, vals_tag=vt, b_tag=bt, absval=True)
    else:
        C = oracle.spmm_rows(rowptr, colind, v, b, rows, n=n, vals_tag=vt, b_tag=bt)
        N = oracle.spmm_rows(rowptr, colind, v, b, rows, n=n, vals_tag=vt, b_tag=bt, absval=True)
    return C, N
