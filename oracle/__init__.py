"""FP64 CPU oracle for CSR SpMM: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It never imports the GPU package and the
GPU package never imports it; the two share no code.

Thin numpy/ctypes wrappers over ``spmm_oracle.c``. Every function computes the
plain definition in double precision (see the C file for each definition and
the paper passage it follows). Storage types are passed through unchanged and
widened exactly inside the C code: float64, float32, and bfloat16/float16 given
as their 16-bit patterns (numpy ``uint16``) with an explicit ``dtype`` tag.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

F64, F32, BF16, F16 = 0, 1, 2, 3
_NP_TAG = {np.dtype(np.float64): F64, np.dtype(np.float32): F32}


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB lets the mutation test load a deliberately broken copy.
        path = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        _lib = load(path)
    return _lib


def native_build(path):
    """The same source compiled -O3 -march=native for this host (the CPU
    baseline's build; its results are bitwise those of the test build)."""
    return load(_build.build_native(path))


def load(path):
    """ctypes handle of an oracle library built from spmm_oracle.c."""
    L = ctypes.CDLL(path)
    i64, i32p, vp, dp = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
    L.oracle_spmm.argtypes = [i64, i64, i64, i32p, i32p, vp, ctypes.c_int, vp, ctypes.c_int,
                              i64, dp, i64, ctypes.c_int, ctypes.c_int]
    L.oracle_spmm_rows.argtypes = [i64, i32p, i32p, vp, ctypes.c_int, vp, ctypes.c_int, i64,
                                   vp, i64, dp, ctypes.c_int, ctypes.c_int]
    L.oracle_spmm_t.argtypes = [i64, i64, i64, i32p, i32p, vp, ctypes.c_int, vp, ctypes.c_int,
                                i64, dp, ctypes.c_int]
    L.oracle_sddmm.argtypes = [i64, i64, i32p, i32p, vp, ctypes.c_int, i64, vp, ctypes.c_int,
                               i64, dp, ctypes.c_int, ctypes.c_int]
    L.oracle_spmm_semiring.argtypes = [i64, i64, i32p, i32p, vp, ctypes.c_int, vp, ctypes.c_int,
                                       i64, dp, i64, ctypes.c_int]
    L.oracle_transpose.argtypes = [i64, i64, i32p, i32p, i32p, i32p, i32p]
    L.oracle_merge_walk.argtypes = [i64, i32p, i32p]
    L.oracle_merge_search.argtypes = [i64, i32p, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.oracle_merge_num_parts.argtypes = [i64, i64, i64]
    L.oracle_merge_num_parts.restype = i64
    L.oracle_merge_partition.argtypes = [i64, i32p, i64, i32p]
    L.oracle_nz_num_parts.argtypes = [i64, i64, i64]
    L.oracle_nz_num_parts.restype = i64
    L.oracle_nz_partition.argtypes = [i64, i32p, i64, i32p]
    L.oracle_heuristic_merge.argtypes = [i64, i64]
    L.oracle_decode.argtypes = [vp, i64, ctypes.c_int]
    L.oracle_decode.restype = ctypes.c_double
    L.oracle_max_threads.restype = ctypes.c_int
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tagged(x, tag):
    """Return (contiguous array, dtype tag). 16-bit patterns need an explicit tag."""
    x = np.ascontiguousarray(x)
    if tag is None:
        if x.dtype not in _NP_TAG:
            raise TypeError(f"oracle: give dtype tag for {x.dtype}")
        tag = _NP_TAG[x.dtype]
    elif tag in (BF16, F16) and x.dtype != np.uint16:
        raise TypeError("oracle: bf16/f16 inputs are passed as uint16 bit patterns")
    return x, tag


def _csr(rowptr, colind):
    return (np.ascontiguousarray(rowptr, dtype=np.int32),
            np.ascontiguousarray(colind, dtype=np.int32))


def max_threads():
    return lib().oracle_max_threads()


def spmm(rowptr, colind, vals, B, n=None, k=None, vals_tag=None, b_tag=None, absval=False,
         nthreads=0, library=None):
    """C = A*B in FP64 (m-by-n). ``B`` is k-by-ld row-major; only its first n columns are used.
    ``library``: another build of the same source (default: the test build)."""
    rowptr, colind = _csr(rowptr, colind)
    vals, vt = _tagged(vals, vals_tag)
    B, bt = _tagged(B, b_tag)
    m = rowptr.shape[0] - 1
    kk, ld = B.shape
    n = ld if n is None else n
    C = np.empty((m, n), dtype=np.float64)
    rc = (library or lib()).oracle_spmm(m, kk if k is None else k, n, _p(rowptr), _p(colind),
                                        _p(vals), vt, _p(B), bt, ld, _p(C), n, int(absval),
                                        nthreads)
    assert rc == 0
    return C


def spmm_rows(rowptr, colind, vals, B, rows, n=None, vals_tag=None, b_tag=None, absval=False,
              nthreads=0):
    """Rows ``rows`` of A*B in FP64, shape (len(rows), n)."""
    rowptr, colind = _csr(rowptr, colind)
    vals, vt = _tagged(vals, vals_tag)
    B, bt = _tagged(B, b_tag)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    ld = B.shape[1]
    n = ld if n is None else n
    out = np.empty((rows.shape[0], n), dtype=np.float64)
    rc = lib().oracle_spmm_rows(n, _p(rowptr), _p(colind), _p(vals), vt, _p(B), bt, ld, _p(rows),
                                rows.shape[0], _p(out), int(absval), nthreads)
    assert rc == 0
    return out


PLUS_TIMES, MIN_PLUS, MAX_PLUS, MAX_TIMES = 0, 1, 2, 3


def spmm_semiring(rowptr, colind, vals, B, semiring, n=None, vals_tag=None, b_tag=None):
    """C = A (+).(x) B over a semiring (codes above), FP64, m-by-n."""
    rowptr, colind = _csr(rowptr, colind)
    vals, vt = _tagged(vals, vals_tag)
    B, bt = _tagged(B, b_tag)
    m = rowptr.shape[0] - 1
    ld = B.shape[1]
    n = ld if n is None else n
    C = np.empty((m, n), dtype=np.float64)
    rc = lib().oracle_spmm_semiring(m, n, _p(rowptr), _p(colind), _p(vals), vt, _p(B), bt, ld,
                                    _p(C), n, semiring)
    assert rc == 0
    return C


def spmm_t(rowptr, colind, vals, dC, k, n=None, vals_tag=None, c_tag=None, absval=False):
    """dB = A^T * dC in FP64 (k-by-n)."""
    rowptr, colind = _csr(rowptr, colind)
    vals, vt = _tagged(vals, vals_tag)
    dC, ct = _tagged(dC, c_tag)
    m = rowptr.shape[0] - 1
    ld = dC.shape[1]
    n = ld if n is None else n
    dB = np.empty((k, n), dtype=np.float64)
    rc = lib().oracle_spmm_t(m, k, n, _p(rowptr), _p(colind), _p(vals), vt, _p(dC), ct, ld,
                             _p(dB), int(absval))
    assert rc == 0
    return dB


def sddmm(rowptr, colind, dC, B, n=None, c_tag=None, b_tag=None, absval=False, nthreads=0):
    """dvals[p] = <dC[row(p), :n], B[colind[p], :n]> in FP64."""
    rowptr, colind = _csr(rowptr, colind)
    dC, ct = _tagged(dC, c_tag)
    B, bt = _tagged(B, b_tag)
    m = rowptr.shape[0] - 1
    n = dC.shape[1] if n is None else n
    out = np.empty(int(rowptr[m]), dtype=np.float64)
    rc = lib().oracle_sddmm(m, n, _p(rowptr), _p(colind), _p(dC), ct, dC.shape[1], _p(B), bt,
                            B.shape[1], _p(out), int(absval), nthreads)
    assert rc == 0
    return out


def transpose(rowptr, colind, k):
    """(AT_rowptr[k+1], AT_colind[nnz], perm[nnz]) by a stable counting sort."""
    rowptr, colind = _csr(rowptr, colind)
    m = rowptr.shape[0] - 1
    nnz = int(rowptr[m])
    at_rowptr = np.empty(k + 1, dtype=np.int32)
    at_colind = np.empty(nnz, dtype=np.int32)
    perm = np.empty(nnz, dtype=np.int32)
    rc = lib().oracle_transpose(m, k, _p(rowptr), _p(colind), _p(at_rowptr), _p(at_colind),
                                _p(perm))
    assert rc == 0
    return at_rowptr, at_colind, perm


def merge_walk(rowptr):
    """Every merge-path coordinate, shape (m + nnz + 1, 2), by a sequential walk."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    m = rowptr.shape[0] - 1
    out = np.empty((m + int(rowptr[m]) + 1, 2), dtype=np.int32)
    assert lib().oracle_merge_walk(m, _p(rowptr), _p(out)) == 0
    return out


def merge_search(rowptr, d):
    """(i, j) on diagonal d by binary search."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    i, j = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().oracle_merge_search(rowptr.shape[0] - 1, _p(rowptr), d, ctypes.byref(i),
                                   ctypes.byref(j))
    assert rc == 0
    return i.value, j.value


def merge_num_parts(m, nnz, W):
    return int(lib().oracle_merge_num_parts(m, nnz, W))


def merge_partition(rowptr, W):
    """Coordinates at diagonals min(p*W, m+nnz), p = 0..P; shape (P+1, 2)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    m = rowptr.shape[0] - 1
    P = merge_num_parts(m, int(rowptr[m]), W)
    out = np.empty((P + 1, 2), dtype=np.int32)
    assert lib().oracle_merge_partition(m, _p(rowptr), W, _p(out)) == 0
    return out


def nz_num_parts(m, nnz, W):
    return int(lib().oracle_nz_num_parts(m, nnz, W))


def nz_partition(rowptr, W):
    """Nonzero split (Sec. 4): piece p starts at nonzero min(p*W, nnz) in the
    row found by a 1-D search on the row offsets; shape (P+1, 2) of (row,
    nonzero) merge states, first (0, 0), last (m, nnz)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    m = rowptr.shape[0] - 1
    P = nz_num_parts(m, int(rowptr[m]), W)
    out = np.empty((P + 1, 2), dtype=np.int32)
    assert lib().oracle_nz_partition(m, _p(rowptr), W, _p(out)) == 0
    return out


def heuristic_merge(m, nnz):
    """Sec. 5.4 rule: True selects the merge-based kernel (mean row length < 9.35)."""
    return bool(lib().oracle_heuristic_merge(m, nnz))


def decode(bits, tag):
    """Widen one stored element exactly (used by the pins on the decoders)."""
    bits = np.ascontiguousarray(bits)
    return np.array([lib().oracle_decode(_p(bits), t, tag) for t in range(bits.size)])
