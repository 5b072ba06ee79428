"""Reduced-precision element contractions, emulated on the CPU (oracle).
Test infrastructure only (see the package docstring).

Reading of the precision variants (the build's growth direction; the paper
states no floating-point precision for its runs): only the element-local
contraction rhs = [-Dr | -Ds | -Dt | LIFT] [G_r; G_s; G_t; Delta] changes;
fluxes, jumps, the state and the Runge-Kutta update stay FP64.

* FP32:  operator and operands rounded to FP32 (round to nearest, ties to
  even), products accumulated in FP32, the sum widened to FP64.
* split BF16 (Henry, Tang & Heinecke, ARITH 2019):  with x32 = fp32(x),
  x_hi = bf16(x32) and x_lo = bf16(x32 - x_hi) (the difference is exact in
  FP32), all roundings to nearest with ties to even;
  Op X ~ Op_hi X_hi + Op_hi X_lo + Op_lo X_hi, products accumulated in FP32.
  Each BF16 x BF16 product is exact in FP32.

Delta form (both reduced modes): the volume operands are the deviations
G_a - G_a(node 0) of each element's contravariant fluxes from their value at
the element's first node.  The contraction is unchanged in exact arithmetic
because every row of D_a sums to zero (D_a applied to a constant is zero),
while the rounded operands now carry the flux variation inside the element
instead of its level, so the error scales with that variation.

Error bound used by the tests (Higham, Accuracy and Stability, Sec. 3.1,
with the operand representation error added): for each output entry,
  |y_mode - y| <= (c_rep + K u32) * sum_k |Op_ik| |X_k|,
u32 = 2^-24, K = number of summed terms (in the delta form the |X| are
those of the delta operands, and the FP64 reference's own rounding
K 2^-53 sum_k |Op_ik| |X_k| on the plain operands is added), c_rep = 2 u32 for FP32 (both
operands rounded once) and 3 * 2^-16 + 2 u32 for split BF16 (dropped lo*lo
product, the two operands' residuals after the lo part, and their rounding to
FP32).
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def round_fp32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """FP64 -> FP32 -> BF16, both steps round-to-nearest-even (finite inputs)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def split_bf16(x: np.ndarray):
    x32 = round_fp32(x)
    hi = round_bf16(x32)
    lo = round_bf16(x32 - hi)
    return hi, lo


def contract(Op: np.ndarray, X: np.ndarray, mode: str) -> np.ndarray:
    """Y[..., i] = sum_k Op[i, k] X[..., k] in the given mode ('fp64', 'fp32',
    'split_bf16'), X of shape [..., K]."""
    if mode == "fp64":
        return X @ Op.T
    if mode == "fp32":
        return (X.astype(np.float32) @ Op.astype(np.float32).T).astype(np.float64)
    if mode == "split_bf16":
        Oh, Ol = split_bf16(Op)
        Xh, Xl = split_bf16(X)
        f = lambda a: a.astype(np.float32)
        acc = f(Xh) @ f(Oh).T + f(Xl) @ f(Oh).T + f(Xh) @ f(Ol).T
        return acc.astype(np.float64)
    raise ValueError(mode)


def error_bound_factor(mode: str, K: int) -> float:
    c_rep = {"fp64": 0.0, "fp32": 2 * U32, "split_bf16": 3 * 2.0 ** -16 + 2 * U32}[mode]
    acc = (2.0 ** -53) * K if mode == "fp64" else U32 * K
    return c_rep + acc


def contraction_inputs(ops: dict, geo: dict, conn: dict, q: np.ndarray, gamma: float = 1.4, elems=None,
                       delta: bool = False):
    """The operator [-Dr | -Ds | -Dt | LIFT] (Np x K) and the per-element,
    per-field operand X = [G_r; G_s; G_t; Delta] (shape [5, n, K]) of the
    Euler RHS, in FP64, so that rhs = X Op^T (up to rounding).  With
    delta=True each G_a is replaced by G_a - G_a(node 0) (delta form)."""
    from .euler import _fluxes
    E = q.shape[1]
    idx = np.arange(E) if elems is None else np.asarray(elems, dtype=np.int64)
    qe = q[:, idx, :]
    (Fx, Fy, Fz), _, _ = _fluxes(qe, gamma)
    rx = geo["rst_x"][idx]
    Gs = [rx[None, :, a, 0, None] * Fx + rx[None, :, a, 1, None] * Fy + rx[None, :, a, 2, None] * Fz for a in range(3)]
    if delta:
        Gs = [G - G[:, :, :1] for G in Gs]
    Nfp = ops["Nfp"]
    fm = ops["Fmask"].reshape(-1)
    qM = qe[:, :, fm]
    qP = q[:, conn["mapP_elem"][idx], conn["mapP_node"][idx]]
    n = np.repeat(geo["normals"][idx], Nfp, axis=1)
    Fs = np.repeat(geo["Fscale"][idx], Nfp, axis=1)
    (FxM, FyM, FzM), (uM, vM, wM), cM = _fluxes(qM, gamma)
    (FxP, FyP, FzP), (uP, vP, wP), cP = _fluxes(qP, gamma)
    nx, ny, nz = n[..., 0], n[..., 1], n[..., 2]
    lam = np.maximum(np.abs(uM * nx + vM * ny + wM * nz) + cM, np.abs(uP * nx + vP * ny + wP * nz) + cP)
    delta = Fs * (0.5 * (nx * FxM + ny * FyM + nz * FzM - nx * FxP - ny * FyP - nz * FzP) - 0.5 * lam * (qM - qP))
    X = np.concatenate(Gs + [delta], axis=2)
    Op = np.concatenate([-ops["Dr"], -ops["Ds"], -ops["Dt"], ops["LIFT"]], axis=1)
    return Op, X


def rhs(ops: dict, geo: dict, conn: dict, q: np.ndarray, mode: str, gamma: float = 1.4, elems=None):
    """Euler RHS with the contraction done in `mode` (reduced modes in the
    delta form); returns (rhs, bound) where bound is the per-entry error bound
    of that mode against FP64."""
    Op, X = contraction_inputs(ops, geo, conn, q, gamma, elems, delta=mode != "fp64")
    y = contract(Op, X, mode)
    K = Op.shape[1]
    T = np.abs(X) @ np.abs(Op).T
    bound = error_bound_factor(mode, K) * T
    if mode != "fp64":
        # the FP64 reference carries its own rounding, on the plain operands
        _, Xp = contraction_inputs(ops, geo, conn, q, gamma, elems)
        bound = bound + error_bound_factor("fp64", K) * (np.abs(Xp) @ np.abs(Op).T)
    return y, bound
