"""Binding of the sparse products on fixed patterns (include/spchol_products.h).

SparseProduct(m, p, n, A, B, transB, D) analyses C = A B (or A B^T) + D once
on the host; run() evaluates a batch of value sets on the device.  Chains
(powers, L M L^T + K) are products of products; the helpers below build
their plans.  Argument marshalling only.
"""
import ctypes
from typing import List, Optional, Tuple

import numpy as np

from . import SC_F32, SC_F64, _check, _dev_ptr, _lib, _ptr, _stream_handle

# names exported by the library for this module, in the order of the header
EXPORTS = ["sc_spprod_create", "sc_spprod_info", "sc_spprod_export", "sc_spprod_run",
           "sc_spprod_destroy"]

_P, _I32, _I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
for _name, _args in {
        "sc_spprod_create": [_I64, _I64, _I64, _P, _P, _P, _P, _I32, _P, _P, _P],
        "sc_spprod_info": [_P, _P, _P],
        "sc_spprod_export": [_P, _P, _P],
        "sc_spprod_run": [_P, ctypes.c_int, _I32, _P, _I64, _P, _I64, _P, _I64, _P, _I64, _P]
        }.items():
    getattr(_lib, _name).argtypes = _args
    getattr(_lib, _name).restype = ctypes.c_int
_lib.sc_spprod_destroy.argtypes = [_P]
_lib.sc_spprod_destroy.restype = None

Pattern = Tuple[np.ndarray, np.ndarray]   # (rowptr int64[rows+1], colind int32)


class SparseProduct:
    """Plan of C = A B (transB False) or A B^T (transB True), plus D."""

    def __init__(self, m: int, p: int, n: int, A: Pattern, B: Pattern, transB: bool = False,
                 D: Optional[Pattern] = None):
        ar, ac = (np.ascontiguousarray(A[0], np.int64), np.ascontiguousarray(A[1], np.int32))
        br, bc = (np.ascontiguousarray(B[0], np.int64), np.ascontiguousarray(B[1], np.int32))
        dr = dc = None
        if D is not None:
            dr, dc = (np.ascontiguousarray(D[0], np.int64), np.ascontiguousarray(D[1], np.int32))
        self.m, self.p, self.n = int(m), int(p), int(n)
        self.nnzA, self.nnzB = int(ar[-1]), int(br[-1])
        self.nnzD = int(dr[-1]) if dr is not None else 0
        self.has_d = D is not None
        h = ctypes.c_void_p()
        _check(_lib.sc_spprod_create(self.m, self.p, self.n, _ptr(ar), _ptr(ac), _ptr(br),
                                     _ptr(bc), 1 if transB else 0, _ptr(dr), _ptr(dc),
                                     ctypes.byref(h)), "sc_spprod_create")
        self._h = h
        nnz, nt = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.sc_spprod_info(self._h, ctypes.byref(nnz), ctypes.byref(nt)), "sc_spprod_info")
        self.nnz, self.nterms = nnz.value, nt.value
        self.rowptr = np.empty(self.m + 1, np.int64)
        self.colind = np.empty(self.nnz, np.int32)
        _check(_lib.sc_spprod_export(self._h, _ptr(self.rowptr), _ptr(self.colind)),
               "sc_spprod_export")

    @property
    def pattern(self) -> Pattern:
        return self.rowptr, self.colind

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.sc_spprod_destroy(self._h)
            self._h = None

    def run(self, A, B, C, D=None, stream=None):
        """C[batch, nnzC] <- A B (+ D); device tensors of one dtype
        (float64 or float32), [batch, nnz] each."""
        import torch
        dt = A.dtype
        if dt not in (torch.float64, torch.float32):
            raise ValueError("float64 or float32 values")
        name = "float64" if dt == torch.float64 else "float32"
        batch = int(C.shape[0])
        if A.shape[0] != batch or B.shape[0] != batch or (D is not None and D.shape[0] != batch):
            raise ValueError("all value arrays need the same batch")
        _check(_lib.sc_spprod_run(self._h, SC_F64 if dt == torch.float64 else SC_F32, batch,
                                  _dev_ptr(A, name), int(A.shape[1]), _dev_ptr(B, name),
                                  int(B.shape[1]),
                                  None if D is None else _dev_ptr(D, name),
                                  0 if D is None else int(D.shape[1]), _dev_ptr(C, name),
                                  int(C.shape[1]), _stream_handle(stream)), "sc_spprod_run")
        return C


def power_chain(n: int, A: Pattern, k: int) -> List[SparseProduct]:
    """Plans of A^2 = A A, A^3 = A^2 A, ..., A^k (each power stored once and
    read by the next product)."""
    plans = []
    cur = A
    for _ in range(2, k + 1):
        pr = SparseProduct(n, n, n, cur, A)
        plans.append(pr)
        cur = pr.pattern
    return plans


def lmlt_plus_k(n: int, L: Pattern, K: Pattern) -> Tuple[SparseProduct, SparseProduct]:
    """Plans of T = L diag(M) (M given as the values of a diagonal pattern)
    and R = T L^T + K."""
    diag = (np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32))
    t = SparseProduct(n, n, n, L, diag)
    r = SparseProduct(n, n, n, t.pattern, L, transB=True, D=K)
    return t, r
