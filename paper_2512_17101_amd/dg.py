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
           "dg_mesh_destroy", "dg_rhs", "dg_rk_step", "dg_rk_step_noalloc", "dg_lsrk_update", "dg_thermo_create", "dg_thermo_destroy",
           "dg_mech_create", "dg_mech_destroy", "dg_temperature", "dg_sources", "dg_mlp_create", "dg_mlp_destroy",
           "dg_mlp_set_params", "dg_mlp_get_params", "dg_mlp_set_normalization", "dg_mlp_get_normalization",
           "dg_mlp_fit_normalization", "dg_mlp_loss_grad", "dg_mlp_train_step", "dg_mlp_predict",
           "dg_temperature_learned", "dg_batch_create", "dg_batch_destroy", "dg_batch_bind",
           "dg_batch_set_config", "dg_batch_get_config", "dg_batch_rk_step", "dg_batch_info", "dg_batch_autotune",
           "dg_ns_rhs", "dg_ns_rk_step", "dg_mesh_set_launch", "dg_mesh_get_launch", "dg_autotune",
           "dg_synchronize", "dg_last_error")


class DGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class LaunchConfig(ctypes.Structure):
    """dg_launch_config: one mesh's RHS / Runge-Kutta launch shape for one precision."""
    _fields_ = [("waves_per_block", ctypes.c_int), ("rk_fused", ctypes.c_int), ("lds_stage", ctypes.c_int),
                ("xcd_run", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _Params(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("gamma", ctypes.c_double), ("mu", ctypes.c_double),
                ("Pr", ctypes.c_double), ("Sc", ctypes.c_double), ("thermo", ctypes.c_void_p),
                ("mech", ctypes.c_void_p), ("work", ctypes.c_void_p), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int)]


class BatchConfig(ctypes.Structure):
    """dg_batch_config: launch shape of the batched stage kernels."""
    _fields_ = [("waves_per_block", ctypes.c_int), ("blocks_per_cu", ctypes.c_int), ("order", ctypes.c_int),
                ("xcd_chunks", ctypes.c_int), ("per_order", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


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
        L.dg_rk_step_noalloc.argtypes = [_c_p, ctypes.POINTER(_Params), ctypes.c_int, _c_p, _dbl, _dbl, _c_p]
        L.dg_lsrk_update.argtypes = [_i64, _dbl, _dbl, _dbl, _c_p, _c_p, _c_p, _c_p]
        L.dg_thermo_create.argtypes = [ctypes.c_int, _c_p, _c_p, ctypes.c_int, ctypes.POINTER(_c_p)]
        L.dg_thermo_destroy.argtypes = [_c_p]
        L.dg_mech_create.argtypes = [_c_p, ctypes.c_int, _c_p, _c_p, _c_p, _c_p, ctypes.POINTER(_c_p)]
        L.dg_mech_destroy.argtypes = [_c_p]
        L.dg_temperature.argtypes = [_i64, _c_p, _c_p, _c_p, _c_p, _c_p, _dbl, ctypes.c_int, _c_p, _c_p]
        L.dg_sources.argtypes = [_i64, _c_p, _c_p, _c_p, _c_p, _c_p]
        L.dg_synchronize.argtypes = [ctypes.c_int, _c_p]
        L.dg_mlp_create.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(_c_p)]
        L.dg_mlp_destroy.argtypes = [_c_p]
        L.dg_mlp_set_params.argtypes = [_c_p, _c_p]
        L.dg_mlp_get_params.argtypes = [_c_p, _c_p]
        L.dg_mlp_set_normalization.argtypes = [_c_p, _c_p, _c_p, _dbl, _dbl]
        L.dg_mlp_get_normalization.argtypes = [_c_p, _c_p, _c_p, _c_p, _c_p]
        L.dg_mlp_fit_normalization.argtypes = [_c_p, _i64, _i64, _c_p, _c_p, _c_p]
        L.dg_mlp_loss_grad.argtypes = [_c_p, _i64, _i64, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p]
        L.dg_mlp_train_step.argtypes = [_c_p, _i64, _i64, _c_p, _c_p, _c_p, ctypes.c_float, _c_p, _c_p]
        L.dg_mlp_predict.argtypes = [_c_p, _i64, _i64, _c_p, _c_p, _c_p]
        L.dg_temperature_learned.argtypes = [_c_p, _c_p, _i64, _c_p, _dbl, _c_p, _c_p, _dbl, ctypes.c_int,
                                             ctypes.c_int, _c_p, _c_p]
        L.dg_batch_create.argtypes = [_c_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_c_p)]
        L.dg_batch_destroy.argtypes = [_c_p]
        L.dg_batch_bind.argtypes = [_c_p, _c_p, _c_p, _c_p]
        L.dg_batch_set_config.argtypes = [_c_p, ctypes.POINTER(BatchConfig)]
        L.dg_batch_get_config.argtypes = [_c_p, ctypes.POINTER(BatchConfig)]
        L.dg_batch_rk_step.argtypes = [_c_p, ctypes.POINTER(_Params), ctypes.c_int, _c_p]
        L.dg_batch_info.argtypes = [_c_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_int)]
        L.dg_batch_autotune.argtypes = [_c_p, ctypes.POINTER(_Params), ctypes.c_char_p, ctypes.c_int,
                                        ctypes.POINTER(BatchConfig), ctypes.POINTER(_dbl), _c_p]
        L.dg_ns_rhs.argtypes = [_c_p, ctypes.POINTER(_Params), _c_p, _c_p, _c_p, _c_p, _c_p]
        L.dg_mesh_set_launch.argtypes = [_c_p, ctypes.c_int, ctypes.POINTER(LaunchConfig)]
        L.dg_mesh_get_launch.argtypes = [_c_p, ctypes.c_int, ctypes.POINTER(LaunchConfig)]
        L.dg_autotune.argtypes = [_c_p, ctypes.POINTER(_Params), ctypes.c_int, ctypes.c_char_p, ctypes.c_int,
                                  ctypes.POINTER(LaunchConfig), ctypes.POINTER(_dbl), _c_p]
        L.dg_ns_rk_step.argtypes = [_c_p, ctypes.POINTER(_Params), _c_p, _c_p, _c_p, _dbl, _dbl, ctypes.c_int, _c_p]
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

    def set_launch(self, mode: str = "fp64", waves_per_block: int = 4, rk_fused: int = 1, lds_stage: int = 1,
                   xcd_run: int = 1):
        c = LaunchConfig(waves_per_block, rk_fused, lds_stage, xcd_run)
        _check(lib().dg_mesh_set_launch(self._h, PRECISIONS[mode], ctypes.byref(c)))

    def get_launch(self, mode: str = "fp64") -> dict:
        c = LaunchConfig()
        _check(lib().dg_mesh_get_launch(self._h, PRECISIONS[mode], ctypes.byref(c)))
        return c.as_dict()

    def autotune(self, mode: str = "fp64", gamma: float = 1.4, cache_path=None, trials: int = 3, stream=None):
        """Tune this mesh's launch configuration; returns (config dict, ms per step or -1 from cache)."""
        prm = _params(gamma)
        c, ms = LaunchConfig(), _dbl()
        path = None if cache_path is None else str(cache_path).encode()
        _check(lib().dg_autotune(self._h, ctypes.byref(prm), PRECISIONS[mode], path, int(trials), ctypes.byref(c),
                                 ctypes.byref(ms), _stream(stream)))
        return c.as_dict(), ms.value

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
    return _Params(model, gamma, 0.0, 0.0, 0.0, None, None, None, 0.0, 0)


MU, PR, SC = 1.8e-5, 0.71, 0.71
NS_WORK_PER_NODE = 58  # doubles of dg_ns_rk_step scratch per node
NS_RHS_WORK = 35       # doubles per node of dg_rhs scratch with model 1 (DG_NS_RHS_WORK)
NS_STEP_WORK = 59      # doubles per node of dg_rk_step scratch with model 1 (DG_NS_STEP_WORK)


def _ns_params(thermo, mech, mu, Pr, Sc, work=None, tol=0.0, max_iter=0):
    return _Params(1, 0.0, float(mu), float(Pr), float(Sc), thermo.handle.value,
                   None if mech is None else mech.handle.value, None if work is None else _dev_ptr(work).value,
                   float(tol), int(max_iter))


def synchronize(device: int = 0, stream=None):
    """Wait for the stream and raise DGError (DG_ERR_NONFINITE / DG_ERR_NOCONV)
    if a kernel on the device flagged a failure since the last call."""
    _check(lib().dg_synchronize(int(device), _stream(stream)))


def _check_state(mesh: "Mesh", t, nf: int, name: str):
    """A device tensor of exactly nf * E * Np doubles on the mesh's device
    (the kernels index the state by the mesh's sizes)."""
    if t.numel() != nf * mesh.E * mesh.Np:
        raise ValueError(f"{name} must hold {nf} x E x Np = {nf * mesh.E * mesh.Np} doubles, got {t.numel()}")
    if t.is_cuda and t.device.index != mesh.device:
        raise ValueError(f"{name} lives on device {t.device.index}, the mesh on {mesh.device}")


def reacting_rhs(mesh: "Mesh", thermo, q, out, work, mech=None, mu: float = MU, Pr: float = PR, Sc: float = SC,
                 tol: float = 1e-10, max_iter: int = 50, stream=None):
    """dg_rhs with model 1: reacting NS right-hand side of q [12, E, Np] into
    out, the temperatures (from 1000 K) and gradients in work (>= 35 E Np)."""
    _check_state(mesh, q, 12, "q")
    _check_state(mesh, out, 12, "out")
    if work.numel() < NS_RHS_WORK * mesh.E * mesh.Np:
        raise ValueError("work must hold >= 35 E Np doubles")
    prm = _ns_params(thermo, mech, mu, Pr, Sc, work, tol, max_iter)
    _check(lib().dg_rhs(mesh.handle, ctypes.byref(prm), DG_FP64, _dev_ptr(q), _dev_ptr(out), _stream(stream)))
    return out


def reacting_rk_step(mesh: "Mesh", thermo, q, work, dt: float, mech=None, mu: float = MU, Pr: float = PR,
                     Sc: float = SC, tol: float = 1e-10, max_iter: int = 50, stream=None):
    """dg_rk_step with model 1: one LSRK(5,4) step of q [12, E, Np] in place;
    work (>= 59 E Np doubles) holds the temperatures and stage scratch."""
    _check_state(mesh, q, 12, "q")
    if work.numel() < NS_STEP_WORK * mesh.E * mesh.Np:
        raise ValueError("work must hold >= 59 E Np doubles")
    prm = _ns_params(thermo, mech, mu, Pr, Sc, work, tol, max_iter)
    _check(lib().dg_rk_step(mesh.handle, ctypes.byref(prm), DG_FP64, _dev_ptr(q), ctypes.c_void_p(), 0.0, float(dt),
                            _stream(stream)))
    return q


def ns_rhs(mesh: Mesh, thermo, q, T, sigma, out, mech=None, mu: float = MU, Pr: float = PR, Sc: float = SC,
           stream=None):
    """Reacting Navier-Stokes RHS: q [12, E, Np], T [E, Np] -> sigma [E, Np, 33]
    (lifted gradients) and out [12, E, Np]; mech=None leaves out the sources."""
    n = mesh.E * mesh.Np
    if q.numel() != 12 * n or T.numel() != n or sigma.numel() != 33 * n or out.numel() != 12 * n:
        raise ValueError("q/out must be [12, E, Np], T [E, Np], sigma [E, Np, 33]")
    prm = _ns_params(thermo, mech, mu, Pr, Sc)
    _check(lib().dg_ns_rhs(mesh.handle, ctypes.byref(prm), _dev_ptr(q), _dev_ptr(T), _dev_ptr(sigma), _dev_ptr(out),
                           _stream(stream)))
    return out


def ns_rk_step(mesh: Mesh, thermo, q, T, work, dt: float, mech=None, mu: float = MU, Pr: float = PR,
               Sc: float = SC, tol: float = 1e-10, max_iter: int = 50, stream=None):
    """One LSRK(5,4) step of the reacting NS system; q and T updated in place;
    work holds >= 58 E Np doubles."""
    n = mesh.E * mesh.Np
    if q.numel() != 12 * n or T.numel() != n or work.numel() < NS_WORK_PER_NODE * n:
        raise ValueError("q must be [12, E, Np], T [E, Np], work >= 58 E Np doubles")
    prm = _ns_params(thermo, mech, mu, Pr, Sc)
    _check(lib().dg_ns_rk_step(mesh.handle, ctypes.byref(prm), _dev_ptr(q), _dev_ptr(T), _dev_ptr(work), float(dt),
                               float(tol), int(max_iter), _stream(stream)))
    return q


def rhs(mesh: Mesh, q, out, precision: str = "fp64", gamma: float = 1.4, stream=None):
    """out <- DG Euler RHS of q (both [5, E, Np] float64 device tensors)."""
    _check_state(mesh, q, 5, "q")
    _check_state(mesh, out, 5, "out")
    prm = _params(gamma)
    _check(lib().dg_rhs(mesh.handle, ctypes.byref(prm), PRECISIONS[precision], _dev_ptr(q), _dev_ptr(out),
                        _stream(stream)))
    return out


def rk_step(mesh: Mesh, q, work, t: float, dt: float, precision: str = "fp64", gamma: float = 1.4, stream=None):
    """One LSRK(5,4) step, q updated in place; work holds >= 2 state arrays."""
    _check_state(mesh, q, 5, "q")
    if work.numel() < 2 * q.numel():
        raise ValueError("work must hold at least two state arrays")
    if work.is_cuda and work.device.index != mesh.device:
        raise ValueError("work lives on another device than the mesh")
    prm = _params(gamma)
    _check(lib().dg_rk_step(mesh.handle, ctypes.byref(prm), PRECISIONS[precision], _dev_ptr(q), _dev_ptr(work),
                            float(t), float(dt), _stream(stream)))
    return q


NOALLOC_MAX_STATE = 8 << 20  # doubles of state dg_rk_step_noalloc accepts (DG_NOALLOC_MAX_STATE)


def rk_step_noalloc(mesh: Mesh, q, t: float, dt: float, precision: str = "fp64", gamma: float = 1.4, stream=None):
    """One LSRK(5,4) step, q updated in place, with the library's fixed
    per-GPU scratch array instead of a workspace (no allocation; at most
    NOALLOC_MAX_STATE doubles of state; calls overlapping on one GPU race)."""
    _check_state(mesh, q, 5, "q")
    prm = _params(gamma)
    _check(lib().dg_rk_step_noalloc(mesh.handle, ctypes.byref(prm), PRECISIONS[precision], _dev_ptr(q), float(t),
                                    float(dt), _stream(stream)))
    return q


def lsrk_update(a: float, b: float, dt: float, rhs_t, res, q, stream=None):
    n = q.numel()
    if rhs_t.numel() != n or res.numel() != n:
        raise ValueError("rhs, res and q must have the same size")
    _check(lib().dg_lsrk_update(n, a, b, dt, _dev_ptr(rhs_t), _dev_ptr(res), _dev_ptr(q), _stream(stream)))


class Thermo:
    """Owning wrapper of a dg_thermo handle (species table)."""

    def __init__(self, W, coeffs, device: int = 0):
        W = np.ascontiguousarray(W, dtype=np.float64)
        a = np.ascontiguousarray(coeffs, dtype=np.float64)
        if a.shape != (W.shape[0], 6):
            raise ValueError("coeffs must be [n_species, 6]")
        h = ctypes.c_void_p()
        _check(lib().dg_thermo_create(W.shape[0], _np_ptr(W), _np_ptr(a), device, ctypes.byref(h)))
        self._h, self.ns, self.device = h, W.shape[0], device

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dg_thermo_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mechanism:
    """Owning wrapper of a dg_mech handle (irreversible Arrhenius reactions)."""

    def __init__(self, thermo: Thermo, A, Ea, nu_r, nu_p):
        A = np.ascontiguousarray(A, dtype=np.float64)
        Ea = np.ascontiguousarray(Ea, dtype=np.float64)
        nr = np.ascontiguousarray(nu_r, dtype=np.int32)
        npr = np.ascontiguousarray(nu_p, dtype=np.int32)
        if nr.shape != (A.shape[0], thermo.ns) or npr.shape != nr.shape or Ea.shape != A.shape:
            raise ValueError("A, Ea [nr]; nu_r, nu_p [nr, ns]")
        h = ctypes.c_void_p()
        _check(lib().dg_mech_create(thermo.handle, A.shape[0], _np_ptr(A), _np_ptr(Ea), _np_ptr(nr), _np_ptr(npr),
                                    ctypes.byref(h)))
        self._h, self.ns, self.nr = h, thermo.ns, A.shape[0]
        self._thermo = thermo

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dg_mech_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def temperature(thermo: Thermo, q, T_out, iters, T_guess=None, tol: float = 1e-10, max_iter: int = 50,
                guess=None, stream=None):
    """Newton temperature of the reacting state q ([5+ns, ...] float64 device
    tensor); T_out float64 and iters int32 device tensors of q[0]'s size.
    Starts from T_guess, or from 1000 K, or (guess = an MLP) from the
    network's prediction with the plain restart as fallback."""
    n = q[0].numel()
    if q.shape[0] != 5 + thermo.ns or T_out.numel() != n or iters.numel() != n:
        raise ValueError("q must be [5+ns, ...]; T_out and iters sized like one field")
    if T_guess is not None and T_guess.numel() != n:
        raise ValueError("T_guess must be sized like one field")
    g = _dev_ptr(T_guess) if T_guess is not None else ctypes.c_void_p()
    h = ctypes.c_void_p() if guess is None else guess.handle
    _check(lib().dg_temperature(n, _dev_ptr(q), g, _dev_ptr(T_out), _dev_ptr(iters, "int32"), thermo.handle,
                                float(tol), int(max_iter), h, _stream(stream)))


def sources(mech: Mechanism, q, T, omega, stream=None):
    """Species mass sources omega [ns, ...] from q [5+ns, ...] and T."""
    n = q[0].numel()
    if q.shape[0] != 5 + mech.ns or T.numel() != n or omega.numel() != mech.ns * n:
        raise ValueError("q [5+ns, ...], T [...], omega [ns, ...]")
    _check(lib().dg_sources(n, _dev_ptr(q), _dev_ptr(T), _dev_ptr(omega), mech.handle, _stream(stream)))


N_MLP_PARAMS = 9025


class MLP:
    """Owning wrapper of a dg_mlp handle (learned temperature guess)."""

    def __init__(self, device: int = 0, seed: int = 4002):
        h = ctypes.c_void_p()
        _check(lib().dg_mlp_create(device, seed, ctypes.byref(h)))
        self._h, self.device = h, device

    @property
    def handle(self):
        return self._h

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != N_MLP_PARAMS:
            raise ValueError("expected 9025 parameters")
        _check(lib().dg_mlp_set_params(self._h, _np_ptr(p)))

    def get_params(self) -> np.ndarray:
        p = np.zeros(N_MLP_PARAMS, dtype=np.float32)
        _check(lib().dg_mlp_get_params(self._h, _np_ptr(p)))
        return p

    def set_normalization(self, mean, std, T_mean, T_std):
        m = np.ascontiguousarray(mean, dtype=np.float64)
        s_ = np.ascontiguousarray(std, dtype=np.float64)
        _check(lib().dg_mlp_set_normalization(self._h, _np_ptr(m), _np_ptr(s_), float(T_mean), float(T_std)))

    def get_normalization(self):
        m, s_ = np.zeros(9), np.zeros(9)
        tm, ts = ctypes.c_double(), ctypes.c_double()
        _check(lib().dg_mlp_get_normalization(self._h, _np_ptr(m), _np_ptr(s_), ctypes.byref(tm), ctypes.byref(ts)))
        return m, s_, tm.value, ts.value

    def fit_normalization(self, q, idx, T):
        ld = q[0].numel()
        _check(lib().dg_mlp_fit_normalization(self._h, idx.numel(), ld, _dev_ptr(q), _dev_ptr(idx, "int64"),
                                              _dev_ptr(T)))

    def loss_grad(self, q, idx, T, grad=None, loss=None, stream=None):
        ld = q[0].numel()
        g = _dev_ptr(grad, "float32") if grad is not None else ctypes.c_void_p()
        l_ = _dev_ptr(loss, "float32") if loss is not None else ctypes.c_void_p()
        _check(lib().dg_mlp_loss_grad(self._h, idx.numel(), ld, _dev_ptr(q), _dev_ptr(idx, "int64"), _dev_ptr(T),
                                      g, l_, _stream(stream)))

    def train_step(self, q, idx, T, lr=1e-3, loss=None, stream=None):
        ld = q[0].numel()
        l_ = _dev_ptr(loss, "float32") if loss is not None else ctypes.c_void_p()
        _check(lib().dg_mlp_train_step(self._h, idx.numel(), ld, _dev_ptr(q), _dev_ptr(idx, "int64"), _dev_ptr(T),
                                       float(lr), l_, _stream(stream)))

    def predict(self, q, out, stream=None):
        n = q[0].numel()
        _check(lib().dg_mlp_predict(self._h, n, n, _dev_ptr(q), _dev_ptr(out), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dg_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def temperature_learned(thermo: Thermo, mlp: MLP, q, T_out, iters, T_default: float = 1000.0, tol: float = 1e-10,
                        max_iter: int = 50, learned_max_iter: int = 8, fallback_count=None, stream=None):
    n = q[0].numel()
    fb = _dev_ptr(fallback_count, "int32") if fallback_count is not None else ctypes.c_void_p()
    _check(lib().dg_temperature_learned(thermo.handle, mlp.handle, n, _dev_ptr(q), float(T_default),
                                        _dev_ptr(T_out), _dev_ptr(iters, "int32"), float(tol), int(max_iter),
                                        int(learned_max_iter), fb, _stream(stream)))


class Batch:
    """Owning wrapper of a dg_batch handle: many meshes stepped with one
    launch per Runge-Kutta stage.  The bound tensors are kept referenced here
    so they outlive the handle's use of them."""

    def __init__(self, meshes, precision: str = "fp32"):
        self.meshes = list(meshes)
        arr = (_c_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = ctypes.c_void_p()
        _check(lib().dg_batch_create(arr, len(self.meshes), PRECISIONS[precision], ctypes.byref(h)))
        self._h = h
        self._bound = None

    @property
    def handle(self):
        return self._h

    def bind(self, qs, works, dt):
        """qs[i]: [5, E_i, Np_i] float64 device tensors, works[i] >= 2 state
        arrays each, dt: float64 device tensor [n]."""
        n = len(self.meshes)
        if len(qs) != n or len(works) != n or dt.numel() != n:
            raise ValueError("one state, one work buffer and one dt per mesh")
        for m, q, w in zip(self.meshes, qs, works):
            if q.numel() != 5 * m.E * m.Np or w.numel() < 2 * q.numel():
                raise ValueError("state or work buffer of the wrong size")
        qa = (_c_p * n)(*[_dev_ptr(q).value for q in qs])
        wa = (_c_p * n)(*[_dev_ptr(w).value for w in works])
        _check(lib().dg_batch_bind(self._h, qa, wa, _dev_ptr(dt)))
        self._bound = (list(qs), list(works), dt)

    def set_config(self, waves_per_block=4, blocks_per_cu=2, order=0, xcd_chunks=0, per_order=1):
        c = BatchConfig(waves_per_block, blocks_per_cu, order, xcd_chunks, per_order)
        _check(lib().dg_batch_set_config(self._h, ctypes.byref(c)))

    def get_config(self) -> dict:
        c = BatchConfig()
        _check(lib().dg_batch_get_config(self._h, ctypes.byref(c)))
        return c.as_dict()

    def rk_step(self, gamma: float = 1.4, use_graph: bool = True, stream=None):
        prm = _params(gamma)
        _check(lib().dg_batch_rk_step(self._h, ctypes.byref(prm), int(bool(use_graph)), _stream(stream)))

    def info(self) -> dict:
        ni, ne, nk = _i64(), _i64(), ctypes.c_int()
        _check(lib().dg_batch_info(self._h, ctypes.byref(ni), ctypes.byref(ne), ctypes.byref(nk)))
        return dict(n_items=ni.value, n_elem=ne.value, graph_kernel_nodes=nk.value)

    def autotune(self, gamma: float = 1.4, cache_path=None, trials: int = 3, stream=None):
        """Tune the launch shape; returns (config dict, ms per step or -1 from cache)."""
        prm = _params(gamma)
        c, ms = BatchConfig(), _dbl()
        path = None if cache_path is None else str(cache_path).encode()
        _check(lib().dg_batch_autotune(self._h, ctypes.byref(prm), path, int(trials), ctypes.byref(c),
                                       ctypes.byref(ms), _stream(stream)))
        return c.as_dict(), ms.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dg_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
