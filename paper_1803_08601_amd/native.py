"""ctypes binding of ``libspmm.so`` (include/spmm.h): argument marshalling only.

Functions carry the C names. Tensors supply device pointers (``data_ptr()``)
and the current HIP stream; every computation runs in the library's kernels.
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "spmm.h")

SPMM_OK, SPMM_ERR_INVALID, SPMM_ERR_UNSUPPORTED, SPMM_ERR_HIP, SPMM_ERR_NOMEM, SPMM_ERR_STATE = \
    0, -1, -2, -3, -4, -5
SPMM_F32, SPMM_BF16, SPMM_F16 = 0, 1, 2
SPMM_MODE_PAPER, SPMM_MODE_AUTOTUNE, SPMM_MODE_ROWSPLIT, SPMM_MODE_MERGE, SPMM_MODE_RULE = 0, 1, 2, 3, 4
SPMM_MODE_NZSPLIT, SPMM_MODE_ROWBLOCK = 5, 6
SPMM_KERNEL_ROWSPLIT, SPMM_KERNEL_MERGE, SPMM_KERNEL_NZSPLIT, SPMM_KERNEL_ROWBLOCK = 0, 1, 2, 3
SPMM_PLUS_TIMES, SPMM_MIN_PLUS, SPMM_MAX_PLUS, SPMM_MAX_TIMES = 0, 1, 2, 3

MODES = {"paper": SPMM_MODE_PAPER, "autotune": SPMM_MODE_AUTOTUNE,
         "rowsplit": SPMM_MODE_ROWSPLIT, "merge": SPMM_MODE_MERGE, "rule": SPMM_MODE_RULE,
         "nzsplit": SPMM_MODE_NZSPLIT, "rowblock": SPMM_MODE_ROWBLOCK}
KERNEL_NAMES = {SPMM_KERNEL_ROWSPLIT: "rowsplit", SPMM_KERNEL_MERGE: "merge",
                SPMM_KERNEL_NZSPLIT: "nzsplit", SPMM_KERNEL_ROWBLOCK: "rowblock"}


class spmm_config(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("lanes_per_row", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("items_per_wg", ctypes.c_int32), ("tile_cols", ctypes.c_int32),
                ("rows_per_block", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("col_panels", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class spmm_plan_info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("k", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("paper_choice", ctypes.c_int32),
                ("config", spmm_config), ("lanes_per_slot", ctypes.c_int32),
                ("col_tiles", ctypes.c_int32), ("num_parts", ctypes.c_int64),
                ("max_row_len", ctypes.c_int64), ("mean_row_len", ctypes.c_double),
                ("tuned_ms", ctypes.c_double), ("has_transpose", ctypes.c_int32),
                ("long_rows", ctypes.c_int64), ("plane_rows", ctypes.c_int64),
                ("strip_rows", ctypes.c_int64)]


class spmm_problem(ctypes.Structure):
    _fields_ = [("A_rowptr", ctypes.c_void_p), ("A_colind", ctypes.c_void_p),
                ("A_vals", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("m", ctypes.c_int64), ("k", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("n", ctypes.c_int64), ("ld", ctypes.c_int64)]


class SpmmError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn}: {status_string(status)} ({status}): {msg}")
        self.status = status


_lib = None
_VP, _I64, _I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
_SIGS = {
    "spmm_csr": [_VP, _VP, _VP, _VP, _VP, _I64, _I64, _I64, _I64, _VP],
    "spmm_csr_noalloc": [_VP, _VP, _VP, _VP, _VP, _I64, _I64, _I64, _I64, _I64, _VP],
    "spmm_csr_plan_info": [_VP, _VP, _I64, _I64, _I64, _I64, _VP, _VP],
    "spmm_cache_clear": [],
    "spmm_tune_cache_save": [ctypes.c_char_p],
    "spmm_tune_cache_load": [ctypes.c_char_p],
    "spmm_plan_create": [_VP, _VP, _VP, _I64, _I64, _I64, _I64, _I64, _I32, _I32, _VP],
    "spmm_plan_create_config": [_VP, _VP, _VP, _I64, _I64, _I64, _I64, _I64, _I32, _VP, _VP],
    "spmm_execute": [_VP, _VP, _VP, _VP, _VP],
    "spmm_execute_events": [_VP, _VP, _VP, _VP, _VP, _VP, _VP],
    "spmm_execute_semiring": [_VP, _I32, _VP, _VP, _VP, _VP],
    "spmm_plan_info_get": [_VP, _VP],
    "spmm_plan_partition": [_VP, _VP, _I64],
    "spmm_plan_destroy": [_VP],
    "spmm_transpose_build": [_VP, _VP],
    "spmm_transpose_get": [_VP, _VP, _VP, _VP, _VP],
    "spmm_execute_t": [_VP, _VP, _VP, _VP, _VP],
    "spmm_execute_t_scatter": [_VP, _VP, _VP, _VP, _VP],
    "spmm_sddmm": [_VP, _VP, _VP, _VP, _VP],
    "spmm_batch_plan": [_VP, _VP, _I64, _I32, _I32, _VP],
    "spmm_batch_run": [_VP, _VP],
    "spmm_batch_run_direct": [_VP, _VP],
    "spmm_batch_problem_config": [_VP, _I64, _VP],
    "spmm_batch_destroy": [_VP],
    "spmm_csr_validate": [_VP, _VP, _I64, _I64, _I64, _VP],
    "spmm_calibrate_gather": [_VP, _I64, _I32, _I32, _VP, _I64, _VP],
    "spmm_status_string": [ctypes.c_int],
    "spmm_last_error": [],
    "spmm_version": [],
}
_STR_FUNCS = {"spmm_status_string", "spmm_last_error", "spmm_version"}


def lib():
    """Load the HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name in _STR_FUNCS else ctypes.c_int
        _lib = L
    return _lib


def header_functions():
    """Names of the functions include/spmm.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(spmm_\w+)\s*\(", text, re.M)))


def status_string(status):
    return lib().spmm_status_string(status).decode()


def spmm_last_error():
    return lib().spmm_last_error().decode()


def spmm_version():
    return lib().spmm_version().decode()


def _check(fn, status):
    if status != SPMM_OK:
        raise SpmmError(fn, status, spmm_last_error())
    return status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def dtype_code(torch_dtype):
    import torch
    return {torch.float32: SPMM_F32, torch.bfloat16: SPMM_BF16, torch.float16: SPMM_F16}[torch_dtype]


# ---------------------------------------------------------------- entry points

def spmm_csr(A_rowptr, A_colind, A_vals, B, C, m, k, n, ld, stream=None):
    return _check("spmm_csr", lib().spmm_csr(_ptr(A_rowptr), _ptr(A_colind), _ptr(A_vals),
                                             _ptr(B), _ptr(C), m, k, n, ld, _stream(stream)))


def spmm_csr_noalloc(A_rowptr, A_colind, A_vals, B, C, m, k, nnz, n, ld, stream=None):
    return _check("spmm_csr_noalloc", lib().spmm_csr_noalloc(
        _ptr(A_rowptr), _ptr(A_colind), _ptr(A_vals), _ptr(B), _ptr(C), m, k, nnz, n, ld,
        _stream(stream)))


def spmm_csr_plan_info(A_rowptr, A_colind, m, k, n, ld, stream=None):
    info = spmm_plan_info()
    _check("spmm_csr_plan_info", lib().spmm_csr_plan_info(
        _ptr(A_rowptr), _ptr(A_colind), m, k, n, ld, _stream(stream), ctypes.byref(info)))
    return info


def spmm_cache_clear():
    return _check("spmm_cache_clear", lib().spmm_cache_clear())


def spmm_tune_cache_save(path):
    return _check("spmm_tune_cache_save", lib().spmm_tune_cache_save(os.fsencode(path)))


def spmm_tune_cache_load(path):
    return _check("spmm_tune_cache_load", lib().spmm_tune_cache_load(os.fsencode(path)))


def spmm_plan_create(A_rowptr, A_colind, m, k, nnz, n, ld, dtype, mode, stream=None):
    h = ctypes.c_void_p()
    _check("spmm_plan_create",
           lib().spmm_plan_create(ctypes.byref(h), _ptr(A_rowptr), _ptr(A_colind), m, k, nnz, n,
                                  ld, dtype, mode, _stream(stream)))
    return h


def spmm_plan_create_config(A_rowptr, A_colind, m, k, nnz, n, ld, dtype, config, stream=None):
    h = ctypes.c_void_p()
    _check("spmm_plan_create_config",
           lib().spmm_plan_create_config(ctypes.byref(h), _ptr(A_rowptr), _ptr(A_colind), m, k,
                                         nnz, n, ld, dtype, ctypes.byref(config),
                                         _stream(stream)))
    return h


def spmm_execute(plan, A_vals, B, C, stream=None):
    return _check("spmm_execute", lib().spmm_execute(plan, _ptr(A_vals), _ptr(B), _ptr(C),
                                                     _stream(stream)))


def spmm_execute_events(plan, A_vals, B, C, ev_before, ev_after, stream=None):
    return _check("spmm_execute_events", lib().spmm_execute_events(
        plan, _ptr(A_vals), _ptr(B), _ptr(C), ev_before, ev_after, _stream(stream)))


def spmm_execute_semiring(plan, semiring, A_vals, B, C, stream=None):
    return _check("spmm_execute_semiring", lib().spmm_execute_semiring(
        plan, semiring, _ptr(A_vals), _ptr(B), _ptr(C), _stream(stream)))


def spmm_plan_info_get(plan):
    info = spmm_plan_info()
    _check("spmm_plan_info_get", lib().spmm_plan_info_get(plan, ctypes.byref(info)))
    return info


def spmm_plan_partition(plan, num_parts):
    import numpy as np
    out = np.empty((num_parts + 1, 2), dtype=np.int32)
    _check("spmm_plan_partition", lib().spmm_plan_partition(
        plan, out.ctypes.data_as(ctypes.c_void_p), num_parts + 1))
    return out


def spmm_plan_destroy(plan):
    return _check("spmm_plan_destroy", lib().spmm_plan_destroy(plan))


def spmm_transpose_build(plan, stream=None):
    return _check("spmm_transpose_build", lib().spmm_transpose_build(plan, _stream(stream)))


def spmm_transpose_get(plan, AT_rowptr, AT_colind, perm, stream=None):
    return _check("spmm_transpose_get", lib().spmm_transpose_get(
        plan, _ptr(AT_rowptr), _ptr(AT_colind), _ptr(perm), _stream(stream)))


def spmm_execute_t(plan, A_vals, dC, dB, stream=None):
    return _check("spmm_execute_t", lib().spmm_execute_t(plan, _ptr(A_vals), _ptr(dC), _ptr(dB),
                                                         _stream(stream)))


def spmm_execute_t_scatter(plan, A_vals, dC, dB, stream=None):
    return _check("spmm_execute_t_scatter",
                  lib().spmm_execute_t_scatter(plan, _ptr(A_vals), _ptr(dC), _ptr(dB),
                                               _stream(stream)))


def spmm_sddmm(plan, dC, B, dvals, stream=None):
    return _check("spmm_sddmm", lib().spmm_sddmm(plan, _ptr(dC), _ptr(B), _ptr(dvals),
                                                 _stream(stream)))


def spmm_batch_plan(problems, dtype, mode, stream=None):
    arr = (spmm_problem * len(problems))(*problems)
    h = ctypes.c_void_p()
    _check("spmm_batch_plan", lib().spmm_batch_plan(ctypes.byref(h), arr, len(problems), dtype,
                                                    mode, _stream(stream)))
    return h


def spmm_batch_run(batch, stream=None):
    return _check("spmm_batch_run", lib().spmm_batch_run(batch, _stream(stream)))


def spmm_batch_run_direct(batch, stream=None):
    return _check("spmm_batch_run_direct", lib().spmm_batch_run_direct(batch, _stream(stream)))


def spmm_batch_problem_config(batch, b):
    c = spmm_config()
    _check("spmm_batch_problem_config", lib().spmm_batch_problem_config(batch, b, ctypes.byref(c)))
    return c


def spmm_batch_destroy(batch):
    return _check("spmm_batch_destroy", lib().spmm_batch_destroy(batch))


def spmm_csr_validate(A_rowptr, A_colind, m, k, nnz, stream=None):
    return _check("spmm_csr_validate", lib().spmm_csr_validate(_ptr(A_rowptr), _ptr(A_colind), m,
                                                               k, nnz, _stream(stream)))


def spmm_calibrate_gather(table, table_rows, row_bytes, steps, out, threads, stream=None):
    return _check("spmm_calibrate_gather",
                  lib().spmm_calibrate_gather(_ptr(table), table_rows, row_bytes, steps, _ptr(out),
                                              threads, _stream(stream)))


# ---------------------------------------------------------------- plan wrapper

def _dtype_of(code):
    import torch
    return {SPMM_F32: torch.float32, SPMM_BF16: torch.bfloat16, SPMM_F16: torch.float16}[code]


def _require(t, name, dtype, rows, ld, n):
    """Refuse a tensor the kernels would read or write outside of, or read
    with another layout: it must be on the GPU, of the given dtype, and hold
    `rows` rows of stride `ld` of which the first `n` entries are used (a 1-D
    operand is one row). Accepted layouts: contiguous memory of at least
    (rows - 1) * ld + n elements, read as rows of stride `ld`, or a 2-D view
    with strides (ld, 1) of at least `rows` x `n`."""
    if rows <= 0 or n <= 0:
        return
    if t is None:
        raise ValueError(f"{name} is None")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, the plan needs {dtype}")
    need = (rows - 1) * ld + n
    if t.is_contiguous():
        if t.numel() < need:
            raise ValueError(f"{name} has {t.numel()} elements; {rows} rows of stride {ld} "
                             f"with {n} used need {need}")
        return
    if not (t.dim() == 2 and t.stride(1) == 1 and t.stride(0) == ld):
        raise ValueError(f"{name}: rows of stride {ld} needed, got strides {t.stride()}")
    if t.shape[0] < rows or t.shape[1] < n:
        raise ValueError(f"{name} has shape {tuple(t.shape)}; {rows} rows of {n} needed")


class Plan:
    """Owns a plan handle for one CSR structure (tensors kept alive here).
    Its methods check each tensor's device, dtype and extent against the plan
    before the call (the C entry points take raw pointers)."""

    def __init__(self, rowptr, colind, m, k, n, ld=None, dtype=SPMM_F32, mode="paper",
                 config=None, nnz=None, stream=None):
        self.rowptr, self.colind = rowptr, colind
        self.m, self.k, self.n = int(m), int(k), int(n)
        self.ld = int(n if ld is None else ld)
        self.nnz = int(colind.numel() if nnz is None else nnz)
        self.dtype = dtype
        import torch
        _require(rowptr, "rowptr", torch.int32, 1, self.m + 1, self.m + 1 if self.m > 0 else 0)
        _require(colind, "colind", torch.int32, 1, self.nnz, self.nnz)
        if config is not None:
            cfg = config if isinstance(config, spmm_config) else spmm_config(**config)
            self.handle = spmm_plan_create_config(rowptr, colind, self.m, self.k, self.nnz, self.n,
                                                  self.ld, dtype, cfg, stream)
        else:
            self.handle = spmm_plan_create(rowptr, colind, self.m, self.k, self.nnz, self.n,
                                           self.ld, dtype, MODES.get(mode, mode), stream)

    def info(self):
        return spmm_plan_info_get(self.handle)

    def _check_forward(self, vals, B, C):
        import torch
        dt = _dtype_of(self.dtype)
        if self.m > 0 and self.n > 0:
            _require(vals, "vals", dt, 1, self.nnz, self.nnz)
            _require(B, "B", dt, self.k, self.ld, self.n)
        _require(C, "C", torch.float32, self.m, self.ld, self.n)

    def execute(self, vals, B, C, stream=None):
        self._check_forward(vals, B, C)
        spmm_execute(self.handle, vals, B, C, stream)
        return C

    def execute_semiring(self, semiring, vals, B, C, stream=None):
        self._check_forward(vals, B, C)
        spmm_execute_semiring(self.handle, semiring, vals, B, C, stream)
        return C

    def partition(self):
        return spmm_plan_partition(self.handle, self.info().num_parts)

    def transpose_build(self, stream=None):
        spmm_transpose_build(self.handle, stream)

    def _check_transposed(self, vals, dC, dB):
        import torch
        if self.k > 0 and self.n > 0:
            _require(vals, "vals", _dtype_of(self.dtype), 1, self.nnz, self.nnz)
            _require(dC, "dC", torch.float32, self.m, self.ld, self.n)
        _require(dB, "dB", torch.float32, self.k, self.ld, self.n)

    def execute_t(self, vals, dC, dB, stream=None):
        self._check_transposed(vals, dC, dB)
        spmm_execute_t(self.handle, vals, dC, dB, stream)
        return dB

    def execute_t_scatter(self, vals, dC, dB, stream=None):
        self._check_transposed(vals, dC, dB)
        spmm_execute_t_scatter(self.handle, vals, dC, dB, stream)
        return dB

    def sddmm(self, dC, B, dvals, stream=None):
        import torch
        if self.m > 0 and self.nnz > 0:
            _require(dvals, "dvals", torch.float32, 1, self.nnz, self.nnz)
            _require(dC, "dC", torch.float32, self.m, self.ld, self.n)
            _require(B, "B", _dtype_of(self.dtype), self.k, self.ld, self.n)
        spmm_sddmm(self.handle, dC, B, dvals, stream)
        return dvals

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            spmm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
