"""Python binding of the hexahedron entry points of libdg.so
(include/dg_hex.h): argument marshalling only, like dg.py, whose loader,
status check and parameter record it uses."""
from __future__ import annotations

import ctypes

import numpy as np

from . import dg

# every symbol include/dg_hex.h declares
EXPORTS = ("dg_hex_reference_operators", "dg_hex_mesh_create", "dg_hex_mesh_info", "dg_hex_mesh_nodes",
           "dg_hex_mesh_destroy", "dg_hex_rhs", "dg_hex_rk_step", "dg_hex_oi_operators", "dg_hex_rhs_oi",
           "dg_hex_rk_step_oi", "dg_hex_av_viscosity", "dg_hex_av_rhs", "dg_hex_limit", "dg_hex_shock_rk_step")

AV_RHS_WORK = 15     # doubles per node of dg_hex_av_rhs scratch (plus 2 per element)
SHOCK_STEP_WORK = 25  # doubles per node of dg_hex_shock_rk_step scratch (plus 2 per element)


class AvParams(ctypes.Structure):
    _fields_ = [("s0", ctypes.c_double), ("kappa", ctypes.c_double), ("c_eps", ctypes.c_double),
                ("delta", ctypes.c_double)]


def av_params(order: int, s0=None, kappa: float = 1.0, c_eps: float = 0.5, delta: float = 1e-10) -> AvParams:
    """Shock-capturing parameters; s0 defaults to -(1 + 4 log10 p)."""
    import math
    return AvParams(-(1.0 + 4.0 * math.log10(order)) if s0 is None else float(s0), float(kappa), float(c_eps),
                    float(delta))

_c_p = ctypes.c_void_p
_dbl = ctypes.c_double
_done = False


def lib():
    """libdg.so with the hexahedron entry points' signatures set."""
    global _done
    L = dg.lib()
    if not _done:
        L.dg_hex_reference_operators.argtypes = [ctypes.c_int, _c_p, _c_p, _c_p]
        L.dg_hex_mesh_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_p, _c_p, _c_p,
                                         ctypes.c_int, ctypes.POINTER(_c_p)]
        L.dg_hex_mesh_info.argtypes = [_c_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)]
        L.dg_hex_mesh_nodes.argtypes = [_c_p, _c_p]
        L.dg_hex_mesh_destroy.argtypes = [_c_p]
        L.dg_hex_rhs.argtypes = [_c_p, ctypes.POINTER(dg._Params), _c_p, _c_p, _c_p]
        L.dg_hex_rk_step.argtypes = [_c_p, ctypes.POINTER(dg._Params), _c_p, _c_p, _dbl, _dbl, _c_p]
        L.dg_hex_oi_operators.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _c_p, _c_p, _c_p]
        L.dg_hex_rhs_oi.argtypes = [_c_p, ctypes.POINTER(dg._Params), _c_p, _c_p, _c_p]
        L.dg_hex_rk_step_oi.argtypes = [_c_p, ctypes.POINTER(dg._Params), _c_p, _c_p, _dbl, _dbl, _c_p]
        P_, A_ = ctypes.POINTER(dg._Params), ctypes.POINTER(AvParams)
        L.dg_hex_av_viscosity.argtypes = [_c_p, P_, A_, _c_p, _c_p, _c_p, _c_p, _c_p]
        L.dg_hex_av_rhs.argtypes = [_c_p, P_, A_, _c_p, _c_p, _c_p, _c_p]
        L.dg_hex_limit.argtypes = [_c_p, P_, A_, _c_p, _c_p]
        L.dg_hex_shock_rk_step.argtypes = [_c_p, P_, A_, _c_p, _c_p, _dbl, _dbl, _c_p]
        for name in EXPORTS:
            getattr(L, name).restype = ctypes.c_int
        _done = True
    return L


def reference_operators(order: int) -> dict:
    n = order + 1
    x, D1, lift = np.zeros(n), np.zeros((n, n)), np.zeros((n, 2))
    dg._check(lib().dg_hex_reference_operators(order, dg._np_ptr(x), dg._np_ptr(D1), dg._np_ptr(lift)))
    return {"x": x, "D": D1, "lift": lift}


def oi_operators(order: int) -> dict:
    """Overintegration tables: nq, Gauss points xq and weights wq, B, S, P, lift."""
    n = order + 1
    nq = ctypes.c_int()
    dg._check(lib().dg_hex_oi_operators(order, ctypes.byref(nq), None, None, None))
    k = nq.value
    xq, wq, tab = np.zeros(k), np.zeros(k), np.zeros(3 * k * n + 2 * n)
    dg._check(lib().dg_hex_oi_operators(order, ctypes.byref(nq), dg._np_ptr(xq), dg._np_ptr(wq), dg._np_ptr(tab)))
    return {"nq": k, "xq": xq, "wq": wq, "B": tab[:k * n].reshape(k, n), "S": tab[k * n:2 * k * n].reshape(n, k),
            "P": tab[2 * k * n:3 * k * n].reshape(n, k), "lift": tab[3 * k * n:].reshape(n, 2)}


class HexMesh:
    """Owning wrapper of a dg_hex_mesh handle (periodic rectilinear grid)."""

    def __init__(self, order: int, gx, gy, gz, device: int = 0):
        g = [np.ascontiguousarray(v, dtype=np.float64) for v in (gx, gy, gz)]
        if any(v.ndim != 1 or v.size < 2 for v in g):
            raise ValueError("grid lines must be 1-D arrays of at least two coordinates")
        h = ctypes.c_void_p()
        dg._check(lib().dg_hex_mesh_create(order, g[0].size - 1, g[1].size - 1, g[2].size - 1, dg._np_ptr(g[0]),
                                           dg._np_ptr(g[1]), dg._np_ptr(g[2]), device, ctypes.byref(h)))
        self._h = h
        E, np_ = ctypes.c_int64(), ctypes.c_int()
        dg._check(lib().dg_hex_mesh_info(h, ctypes.byref(E), ctypes.byref(np_)))
        self.order, self.E, self.Np, self.device = order, E.value, np_.value, device
        self.dims = tuple(v.size - 1 for v in g)

    @property
    def handle(self):
        return self._h

    def nodes(self) -> np.ndarray:
        out = np.zeros((self.E, self.Np, 3))
        dg._check(lib().dg_hex_mesh_nodes(self._h, dg._np_ptr(out)))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dg_hex_mesh_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rhs(mesh: HexMesh, q, out, gamma: float = 1.4, stream=None):
    """out <- Euler RHS of q on the hexahedra (both [5, E, Np] float64 device tensors)."""
    dg._check_state(mesh, q, 5, "q")
    dg._check_state(mesh, out, 5, "out")
    prm = dg._params(gamma)
    dg._check(lib().dg_hex_rhs(mesh.handle, ctypes.byref(prm), dg._dev_ptr(q), dg._dev_ptr(out), dg._stream(stream)))
    return out


def rhs_oi(mesh: HexMesh, q, out, gamma: float = 1.4, stream=None):
    """out <- overintegrated Euler RHS of q (Gauss-point flux evaluation)."""
    dg._check_state(mesh, q, 5, "q")
    dg._check_state(mesh, out, 5, "out")
    prm = dg._params(gamma)
    dg._check(lib().dg_hex_rhs_oi(mesh.handle, ctypes.byref(prm), dg._dev_ptr(q), dg._dev_ptr(out),
                                  dg._stream(stream)))
    return out


def rk_step(mesh: HexMesh, q, work, t: float, dt: float, gamma: float = 1.4, overintegrate: bool = False, stream=None):
    """One LSRK(5,4) step on the hexahedra, q updated in place; work holds >=
    2 state arrays; overintegrate selects the Gauss-point flux evaluation."""
    dg._check_state(mesh, q, 5, "q")
    if work.numel() < 2 * q.numel():
        raise ValueError("work must hold at least two state arrays")
    if work.is_cuda and work.device.index != mesh.device:
        raise ValueError("work lives on another device than the mesh")
    prm = dg._params(gamma)
    fn = lib().dg_hex_rk_step_oi if overintegrate else lib().dg_hex_rk_step
    dg._check(fn(mesh.handle, ctypes.byref(prm), dg._dev_ptr(q), dg._dev_ptr(work), float(t), float(dt),
                 dg._stream(stream)))
    return q


def _optr(t, dtype="float64"):
    return dg._dev_ptr(t, dtype) if t is not None else ctypes.c_void_p()


def av_viscosity(mesh: HexMesh, q, G, s_out, eps_out, av: AvParams = None, gamma: float = 1.4, stream=None):
    """Indicator s (optional) and viscosity eps per element ([E]) and the
    viscous fluxes G [3, 5, E, Np] of q (written only where eps > 0)."""
    dg._check_state(mesh, q, 5, "q")
    if G.numel() != 15 * mesh.E * mesh.Np:
        raise ValueError("G must hold 3 x 5 x E x Np doubles")
    for t in (s_out, eps_out):
        if t is not None and t.numel() != mesh.E:
            raise ValueError("s_out / eps_out must hold E doubles")
    if eps_out is None:
        raise ValueError("eps_out is required")
    av = av_params(mesh.order) if av is None else av
    prm = dg._params(gamma)
    dg._check(lib().dg_hex_av_viscosity(mesh.handle, ctypes.byref(prm), ctypes.byref(av), dg._dev_ptr(q),
                                        _optr(s_out), _optr(eps_out), dg._dev_ptr(G), dg._stream(stream)))


def av_rhs(mesh: HexMesh, q, out, work, av: AvParams = None, gamma: float = 1.4, stream=None):
    """out <- Euler RHS + artificial-viscosity term of q."""
    dg._check_state(mesh, q, 5, "q")
    dg._check_state(mesh, out, 5, "out")
    if work.numel() < AV_RHS_WORK * mesh.E * mesh.Np + 2 * mesh.E:
        raise ValueError("work must hold >= 15 E Np + 2 E doubles")
    av = av_params(mesh.order) if av is None else av
    prm = dg._params(gamma)
    dg._check(lib().dg_hex_av_rhs(mesh.handle, ctypes.byref(prm), ctypes.byref(av), dg._dev_ptr(q), dg._dev_ptr(out),
                                  dg._dev_ptr(work), dg._stream(stream)))
    return out


def limit(mesh: HexMesh, q, av: AvParams = None, gamma: float = 1.4, stream=None):
    """Positivity limiter of q in place."""
    dg._check_state(mesh, q, 5, "q")
    av = av_params(mesh.order) if av is None else av
    prm = dg._params(gamma)
    dg._check(lib().dg_hex_limit(mesh.handle, ctypes.byref(prm), ctypes.byref(av), dg._dev_ptr(q), dg._stream(stream)))
    return q


def shock_rk_step(mesh: HexMesh, q, work, t: float, dt: float, av: AvParams = None, gamma: float = 1.4, stream=None):
    """One LSRK(5,4) step with artificial viscosity and the limiter on every stage."""
    dg._check_state(mesh, q, 5, "q")
    if work.numel() < SHOCK_STEP_WORK * mesh.E * mesh.Np + 2 * mesh.E:
        raise ValueError("work must hold >= 25 E Np + 2 E doubles")
    av = av_params(mesh.order) if av is None else av
    prm = dg._params(gamma)
    dg._check(lib().dg_hex_shock_rk_step(mesh.handle, ctypes.byref(prm), ctypes.byref(av), dg._dev_ptr(q),
                                         dg._dev_ptr(work), float(t), float(dt), dg._stream(stream)))
    return q
