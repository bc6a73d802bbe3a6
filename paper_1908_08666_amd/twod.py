"""Handle of the 2-D variant (``hhg2d_*`` in include/hhg.h): macro triangles,
the physically scaled vector operator in two dimensions.  Argument
marshalling only; every step runs in libhhg.so."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L
from .hhg import _descriptors, _dev_ptr, _prec_of, _stream_ptr


class Mesh2D:
    """``verts`` (M, 3, 2), common ``level``; operator weights and variant
    flags as for the 3-D Mesh.  Vectors are [2][n_nodes] device tensors."""

    def __init__(self, verts, level, mu0=0.0, lam0=0.0, mu1=0.0, lam1=0.0, dirichlet="outer",
                 corr="physical", khat="patch", iface="symmetric"):
        verts = np.ascontiguousarray(np.asarray(verts, dtype=np.float64))
        if verts.ndim != 3 or verts.shape[1:] != (3, 2):
            raise ValueError("verts must be (M,3,2)")
        self._verts = verts
        # the 3-D descriptor helper builds the operator descriptor
        _, od, _ = _descriptors(np.zeros((1, 4, 3)), [2], mu0, lam0, mu1, lam1, "conforming",
                                dirichlet, corr, khat, iface)
        md = L.MeshDesc2D(verts.shape[0], verts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          int(level),
                          {"outer": L.HHG_DIRICHLET_OUTER, "none": L.HHG_DIRICHLET_NONE}[dirichlet])
        self._lib = L.lib()
        h = ctypes.c_void_p()
        L.check(self._lib.hhg2d_setup(ctypes.byref(md), ctypes.byref(od), ctypes.byref(h)))
        self._h = h
        self.level = int(level)
        self.n_macro = verts.shape[0]
        nn, nu = ctypes.c_int64(), ctypes.c_int64()
        L.check(self._lib.hhg2d_layout(h, ctypes.byref(nn), ctypes.byref(nu)))
        self.n_nodes, self.n_unknown = int(nn.value), int(nu.value)

    def coords(self) -> np.ndarray:
        xy = np.zeros((2, self.n_nodes))
        L.check(self._lib.hhg2d_node_coords(self._h, xy.ctypes.data_as(ctypes.c_void_p)))
        return xy

    def flags(self) -> np.ndarray:
        f = np.zeros(self.n_nodes, dtype=np.uint8)
        L.check(self._lib.hhg2d_node_flags(self._h, f.ctypes.data_as(ctypes.c_void_p)))
        return f

    def _apply(self, method, x, k, y, stream):
        import torch
        if y is None:
            y = torch.empty_like(x)
        N = self.n_nodes
        L.check(self._lib.hhg2d_apply(self._h, _prec_of(x), method, _dev_ptr(x, (2, N), x.dtype),
                                      _dev_ptr(k, (N,), x.dtype), _dev_ptr(y, (2, N), x.dtype),
                                      _stream_ptr(stream)))
        return y

    def apply_scaled(self, x, k, y=None, stream=None):
        return self._apply(L.HHG_METHOD_SCALED, x, k, y, stream)

    def apply_onthefly(self, x, k, y=None, stream=None):
        return self._apply(L.HHG_METHOD_ONTHEFLY, x, k, y, stream)

    def close(self):
        if getattr(self, "_h", None):
            L.check(self._lib.hhg2d_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
