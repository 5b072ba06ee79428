"""Mixture thermodynamics, temperature Newton solve and Arrhenius sources
(oracle, FP64).  Test infrastructure only (see the package docstring).

The paper names multispecies, reacting flow and temperature-dependent
thermochemistry for MIRGE-Com (Sec. 4 compile-time example, Sec. 5) but prints
no law; the readings are:

* species k (7): R_k = R_u / W_k, cp_k / R_k = a1 + a2 T + a3 T^2 + a4 T^3
  + a5 T^4 (one range), h_k / R_k = a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4
  + a5 T^5/5 + a6, e_k = h_k - R_k T;
* mixture: e = sum Y_k e_k, cv = sum Y_k (cp_k - R_k), p = rho R_u T sum Y_k/W_k;
* temperature from (e, Y): Newton T_{n+1} = T_n - (e(T_n) - e) / cv(T_n),
  iterates clamped to [100, 6000] K, stop when |T_{n+1} - T_n| < tol and
  return T_{n+1} with iteration count n + 1; no convergence within max_iter
  gives count -1, and a step that the clamp cut short is never taken as
  convergence (a root outside the interval is a failure, not the bound);
* irreversible Arrhenius kinetics: k_j = A_j exp(-Ea_j / (R_u T)),
  r_j = k_j prod_k C_k^{nu'_kj}, C_k = rho Y_k / W_k,
  omega_k = W_k sum_j (nu''_kj - nu'_kj) r_j   [kg / (m^3 s)].
"""
from __future__ import annotations

import numpy as np

R_U = 8.314462618
T_MIN, T_MAX = 100.0, 6000.0


def species_cp_over_R(T, a):
    """[K, ...] cp_k / R_k at temperatures T (array)."""
    T = np.asarray(T, dtype=np.float64)
    return a[:, 0, None] + T.ravel()[None] * (a[:, 1, None] + T.ravel()[None] * (
        a[:, 2, None] + T.ravel()[None] * (a[:, 3, None] + T.ravel()[None] * a[:, 4, None])))


def species_h_over_R(T, a):
    T = np.asarray(T, dtype=np.float64).ravel()[None]
    return (a[:, 0, None] * T + a[:, 1, None] * T ** 2 / 2 + a[:, 2, None] * T ** 3 / 3
            + a[:, 3, None] * T ** 4 / 4 + a[:, 4, None] * T ** 5 / 5 + a[:, 5, None])


def mixture_e(T, Y, th):
    """Mixture internal energy [J/kg]; T shape S, Y shape [K] + S."""
    T = np.asarray(T, dtype=np.float64)
    Rk = R_U / th["W"]
    ek = (species_h_over_R(T, th["a"]) - T.ravel()[None]) * Rk[:, None]
    return np.sum(Y.reshape(len(Rk), -1) * ek, axis=0).reshape(T.shape)


def mixture_cv(T, Y, th):
    T = np.asarray(T, dtype=np.float64)
    Rk = R_U / th["W"]
    cvk = (species_cp_over_R(T, th["a"]) - 1.0) * Rk[:, None]
    return np.sum(Y.reshape(len(Rk), -1) * cvk, axis=0).reshape(T.shape)


def mixture_R(Y, th):
    return R_U * np.einsum("k...,k->...", Y, 1.0 / th["W"])


def primitives(q):
    """(rho, u, v, w, e, Y) from the reacting conserved state q[12][...]."""
    rho = q[0]
    u, v, w = q[1] / rho, q[2] / rho, q[3] / rho
    e = q[4] / rho - 0.5 * (u * u + v * v + w * w)
    Y = q[5:] / rho
    return rho, u, v, w, e, Y


def newton_temperature(e, Y, th, T0, tol=1e-10, max_iter=50):
    """Per-node Newton solve of e(T; Y) = e.  Returns (T, iters) with
    iters = -1 where |T_{n+1} - T_n| < tol was not reached in max_iter steps
    (T then holds the last iterate)."""
    shape = np.shape(e)
    e = np.asarray(e, dtype=np.float64).ravel()
    Y = np.asarray(Y, dtype=np.float64).reshape(Y.shape[0], -1)
    T = np.broadcast_to(np.asarray(T0, dtype=np.float64), shape).ravel().copy()
    iters = np.full(e.shape, -1, dtype=np.int64)
    active = np.ones(e.shape, dtype=bool)
    for n in range(max_iter):
        if not active.any():
            break
        Ta = T[active]
        Ya = Y[:, active]
        Tu = Ta - (mixture_e(Ta, Ya, th) - e[active]) / mixture_cv(Ta, Ya, th)
        Tn = np.clip(Tu, T_MIN, T_MAX)
        # a step cut by the clamp is not convergence (the root would lie
        # outside [T_MIN, T_MAX]); NaN compares false and never converges
        done = (np.abs(Tn - Ta) < tol) & (Tn == Tu)
        T[active] = Tn
        idx = np.flatnonzero(active)
        iters[idx[done]] = n + 1
        active[idx[done]] = False
    return T.reshape(shape), iters.reshape(shape)


def rate_constants(T, mech):
    T = np.asarray(T, dtype=np.float64)
    return mech["A"][:, None] * np.exp(-mech["Ea"][:, None] / (R_U * T.ravel()[None]))


def sources(rho, T, Y, th, mech):
    """omega_k [kg/(m^3 s)], shape [K] + shape(T)."""
    shape = np.shape(T)
    C = (rho.ravel()[None] * Y.reshape(len(th["W"]), -1)) / th["W"][:, None]  # [K, n]
    k = rate_constants(T, mech)  # [J, n]
    r = k.copy()
    for j in range(len(mech["A"])):
        for s in range(len(th["W"])):
            nu = mech["nu_r"][j, s]
            if nu != 0:
                r[j] = r[j] * C[s] ** nu
    net = (mech["nu_p"] - mech["nu_r"]).T  # [K, J]
    omega = th["W"][:, None] * (net @ r)
    return omega.reshape((len(th["W"]),) + shape)
