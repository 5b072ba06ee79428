"""Python binding of libdg.so (include/dg.h): argument marshalling only.

Device arrays are torch tensors (float64, contiguous, on the mesh's device);
their data pointers and torch's current HIP stream are handed to the C ABI.
Every numerical step runs in the library; if libdg.so is missing this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdg.so")

DG_FP64, DG_FP32, DG_SPLIT_BF16 = 0, 1, 2
PRECISIONS = {"fp64": DG_FP64, "fp32": DG_FP32, "split_bf16": DG_SPLIT_BF16}
STATUS = {0: "DG_OK", 1: "DG_ERR_ARG", 2: "DG_ERR_MESH", 3: "DG_ERR_ALLOC", 4: "DG_ERR_HIP",
          5: "DG_ERR_NOCONV", 6: "DG_ERR_NONFINITE", 7: "DG_ERR_UNSUPPORTED"}

# every symbol include/dg.h declares
EXPORTS = ("dg_reference_operators", "dg_mesh_create", "dg_mesh_info", "dg_mesh_nodes", "dg_mesh_face_map",
           "dg_mesh_destroy", "dg_rhs", "dg_rk_step", "dg_lsrk_update", "dg_last_error")


class DGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("gamma", ctypes.c_double)]


_lib_handle = None
_c_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_dbl = ctypes.c_double


def lib():
    """Load libdg.so once; raise if it has not been built."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_17101_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.dg_last_error.restype = ctypes.c_char_p
        L.dg_reference_operators.argtypes = [ctypes.c_int] + [_c_p] * 6
        L.dg_mesh_create.argtypes = [ctypes.c_int, _i64, _c_p, _c_p, ctypes.c_int, ctypes.POINTER(_c_p)]
        L.dg_mesh_info.argtypes = [_c_p, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.dg_mesh_nodes.argtypes = [_c_p, _c_p]
        L.dg_mesh_face_map.argtypes = [_c_p, _c_p, _c_p]
        L.dg_mesh_destroy.argtypes = [_c_p]
        L.dg_rhs.argtypes = [_c_p, ctypes.POINTER(_Params), ctypes.c_int, _c_p, _c_p, _c_p]
        L.dg_rk_step.argtypes = [_c_p, ctypes.POINTER(_Params), ctypes.c_int, _c_p, _c_p, _dbl, _dbl, _c_p]
        L.dg_lsrk_update.argtypes = [_i64, _dbl, _dbl, _dbl, _c_p, _c_p, _c_p, _c_p]
        for name in EXPORTS:
            if name != "dg_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _check(status: int):
    if status != 0:
        raise DGError(status, lib().dg_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype_name="float64"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA/HIP torch tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"expected dtype {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def reference_operators(order: int) -> dict:
    """The library's reference-element tables (computed on the host)."""
    from math import comb
    Np = comb(order + 3, 3)
    Nfp = comb(order + 2, 2)
    rst = np.zeros((Np, 3))
    Dr, Ds, Dt = (np.zeros((Np, Np)) for _ in range(3))
    LIFT = np.zeros((Np, 4 * Nfp))
    Fmask = np.zeros((4, Nfp), dtype=np.int32)
    _check(lib().dg_reference_operators(order, _np_ptr(rst), _np_ptr(Dr), _np_ptr(Ds), _np_ptr(Dt),
                                        _np_ptr(LIFT), _np_ptr(Fmask)))
    return dict(rst=rst, Dr=Dr, Ds=Ds, Dt=Dt, LIFT=LIFT, Fmask=Fmask, Np=Np, Nfp=Nfp)


class Mesh:
    """Owning wrapper of a dg_mesh handle."""

    def __init__(self, order: int, elem_xyz: np.ndarray, elem_vid: np.ndarray, device: int = 0):
        xyz = np.ascontiguousarray(elem_xyz, dtype=np.float64)
        vid = np.ascontiguousarray(elem_vid, dtype=np.int64)
        if xyz.ndim != 3 or xyz.shape[1:] != (4, 3) or vid.shape != (xyz.shape[0], 4):
            raise ValueError("elem_xyz must be [E,4,3] and elem_vid [E,4]")
        h = ctypes.c_void_p()
        _check(lib().dg_mesh_create(order, xyz.shape[0], _np_ptr(xyz), _np_ptr(vid), device, ctypes.byref(h)))
        self._h = h
        E, np_, nfp = _i64(), ctypes.c_int(), ctypes.c_int()
        _check(lib().dg_mesh_info(h, ctypes.byref(E), ctypes.byref(np_), ctypes.byref(nfp)))
        self.order, self.E, self.Np, self.Nfp, self.device = order, E.value, np_.value, nfp.value, device

    @property
    def handle(self):
        return self._h

    def state_shape(self, nf: int = 5):
        return (nf, self.E, self.Np)

    def nodes(self) -> np.ndarray:
        out = np.zeros((self.E, self.Np, 3))
        _check(lib().dg_mesh_nodes(self._h, _np_ptr(out)))
        return out

    def face_map(self):
        ne = np.zeros((self.E, 4 * self.Nfp), dtype=np.int64)
        nn = np.zeros((self.E, 4 * self.Nfp), dtype=np.int32)
        _check(lib().dg_mesh_face_map(self._h, _np_ptr(ne), _np_ptr(nn)))
        return ne, nn

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dg_mesh_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _params(gamma: float, model: int = 0):
    return _Params(model, gamma)


def rhs(mesh: Mesh, q, out, precision: str = "fp64", gamma: float = 1.4, stream=None):
    """out <- DG Euler RHS of q (both [5, E, Np] float64 device tensors)."""
    prm = _params(gamma)
    _check(lib().dg_rhs(mesh.handle, ctypes.byref(prm), PRECISIONS[precision], _dev_ptr(q), _dev_ptr(out),
                        _stream(stream)))
    return out


def rk_step(mesh: Mesh, q, work, t: float, dt: float, precision: str = "fp64", gamma: float = 1.4, stream=None):
    """One LSRK(5,4) step, q updated in place; work holds >= 2 state arrays."""
    if work.numel() < 2 * q.numel():
        raise ValueError("work must hold at least two state arrays")
    prm = _params(gamma)
    _check(lib().dg_rk_step(mesh.handle, ctypes.byref(prm), PRECISIONS[precision], _dev_ptr(q), _dev_ptr(work),
                            float(t), float(dt), _stream(stream)))
    return q


def lsrk_update(a: float, b: float, dt: float, rhs_t, res, q, stream=None):
    n = q.numel()
    if rhs_t.numel() != n or res.numel() != n:
        raise ValueError("rhs, res and q must have the same size")
    _check(lib().dg_lsrk_update(n, a, b, dt, _dev_ptr(rhs_t), _dev_ptr(res), _dev_ptr(q), _stream(stream)))
