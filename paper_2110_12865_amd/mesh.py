"""Binding of the on-device mesh assembly (include/spchol_mesh.h).

CotanAssembly(nv, colptr, rowind, tris) holds the index tables of one mesh
pattern; assemble() computes the values of A = K + c diag(m), K the clipped
cotangent stiffness, for a batch of value sets straight into a device
tensor that Numeric.factor() then reads.  Argument marshalling only: the
arithmetic runs in the library's kernels.
"""
import ctypes
from typing import Optional

import numpy as np

from . import _check, _dev_ptr, _lib, _ptr, _stream_handle

# names exported by the library for this module, in the order of the header
EXPORTS = ["sc_cotan_create", "sc_cotan_nedges", "sc_cotan_assemble", "sc_cotan_destroy"]

_P, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
for _name, _args in {
        "sc_cotan_create": [_I64, _P, _P, _I64, _P, _P],
        "sc_cotan_nedges": [_P, _P],
        "sc_cotan_assemble": [_P, _I32, _P, _I64, _P, _P, _D, _D, _D, _P, _I64, _P]}.items():
    getattr(_lib, _name).argtypes = _args
    getattr(_lib, _name).restype = ctypes.c_int
_lib.sc_cotan_destroy.argtypes = [_P]
_lib.sc_cotan_destroy.restype = None


class CotanAssembly:
    """Assembly tables of a triangle mesh on the lower CSC pattern of its
    stiffness matrix (sc_cotan_create), on the current device."""

    def __init__(self, nv, colptr, rowind, tris):
        colptr = np.ascontiguousarray(colptr, np.int64)
        rowind = np.ascontiguousarray(rowind, np.int32)
        tris = np.ascontiguousarray(tris, np.int32)
        self.nv = int(nv)
        self.nnz = int(colptr[-1])
        h = ctypes.c_void_p()
        _check(_lib.sc_cotan_create(self.nv, _ptr(colptr), _ptr(rowind), int(tris.shape[0]),
                                    _ptr(tris), ctypes.byref(h)), "sc_cotan_create")
        self._h = h
        ne = ctypes.c_int64()
        _check(_lib.sc_cotan_nedges(self._h, ctypes.byref(ne)), "sc_cotan_nedges")
        self.nedge = ne.value

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.sc_cotan_destroy(self._h)
            self._h = None

    def assemble(self, pos, mass, values, edge_scale=None, mass_coeff: float = 1e-3,
                 clip=(0.05, 2.0), stream=None):
        """values[batch, nnz] (float64 device tensor) <- the assembled
        matrices.  pos: [nv, 2] shared by every set or [batch, nv, 2];
        edge_scale: [batch, nedge] or None; mass: [nv]."""
        batch = int(values.shape[0])
        if pos.dim() == 3:
            if pos.shape[0] != batch:
                raise ValueError("pos must be [nv, 2] or [batch, nv, 2]")
            stride = int(pos.shape[1] * pos.shape[2])
        else:
            stride = 0
        if edge_scale is not None and tuple(edge_scale.shape) != (batch, self.nedge):
            raise ValueError("edge_scale must be [batch, nedge]")
        sp = None if edge_scale is None else _dev_ptr(edge_scale, "float64")
        _check(_lib.sc_cotan_assemble(self._h, batch, _dev_ptr(pos, "float64"), stride, sp,
                                      _dev_ptr(mass, "float64"), float(mass_coeff),
                                      float(clip[0]), float(clip[1]),
                                      _dev_ptr(values, "float64"), int(values.shape[1]),
                                      _stream_handle(stream)), "sc_cotan_assemble")
        return values
