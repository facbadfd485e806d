"""MI355X (gfx950) CSR sparse x dense matrix multiplication.

``native``   - ctypes binding of libspmm.so (include/spmm.h), same names as the C ABI.
``autograd`` - torch.autograd.Function with hand-written backward kernels.
``workloads``- seeded synthetic inputs shaped like the paper's workloads.
The native library is loaded on first use and must have been built
(``__graft_entry__.build()``); there is no fallback path.
"""
__version__ = "0.1.0"
