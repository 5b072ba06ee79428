"""Reacting compressible Navier-Stokes right-hand side with BR1 viscous terms
(oracle, FP64).  Test infrastructure only (see the package docstring).

The paper names viscous, multispecies, reacting flow for MIRGE-Com (Sec. 5)
but prints no equation; this module follows the textbook forms:

State q = (rho, rho u, rho v, rho w, E, rho Y_1 .. rho Y_K), K = 7; the
temperature T comes from the Newton solve of thermo.py; mixture pressure
p = rho R_u T sum Y_k / W_k, cp = sum Y_k cp_k, cv = sum Y_k cv_k, sound
speed c = sqrt(gamma_mix p / rho) with gamma_mix = cp / cv.

Inviscid flux (component d):
  rho u_d, rho u_i u_d + p delta_id, (E + p) u_d, rho Y_k u_d.
Viscous terms, Bassi & Rebay's first scheme (BR1):
  pass 1 (lifted gradient of the primitives v = (u, v, w, T, Y_1 .. Y_K)),
    sigma_d(v)_i = sum_a (da/dx_d) (D_a v)_i
                   + sum_(f,m) LIFT[i, (f,m)] Fscale_f n_{f,d} 1/2 (v+ - v-)
  (strong form with the central trace 1/2 (v- + v+));
  pass 2, from sigma and T at each node:
    tau = mu (grad u + grad u^T - 2/3 (div u) I)        (Stokes' hypothesis)
    heat flux       -kappa grad T,   kappa = mu cp / Pr
    species flux    J_k = -rho D grad Y_k,  rho D = mu / Sc (one D for all)
    viscous flux F^v_d: 0, tau_{i d}, u_i tau_{i d} + kappa dT/dx_d
                        - sum_k h_k J_{k,d}, -J_{k,d}
Total flux F = F^inv - F^v; volume G_a = sum_d (da/dx_d) F_d; the surface
flux is local Lax-Friedrichs on the inviscid part and the central average on
the viscous part (no penalty):
  Delta = Fscale [ 1/2 n.(F^inv- - F^inv+) - 1/2 lam (q- - q+)
                   - 1/2 n.(F^v- - F^v+) ],
  lam = max(|u-.n| + c-, |u+.n| + c+);
  rhs_i = -sum_a (D_a G_a)_i + (LIFT Delta)_i + S_i,
with the chemical sources S = (0, 0, 0, 0, 0, omega_1 .. omega_K) of
thermo.sources.
"""
from __future__ import annotations

import numpy as np

from . import thermo as th_

MU, PR, SC = 1.8e-5, 0.71, 0.71


def _mixture(T, Y, th):
    """cp, cv [J/(kg K)], R_mix [J/(kg K)] and species enthalpies h_k [J/kg]
    at temperatures T (any shape S), Y of shape [K] + S."""
    shape = np.shape(T)
    Rk = th_.R_U / th["W"]
    cpk = th_.species_cp_over_R(T, th["a"]) * Rk[:, None]  # [K, n]
    hk = th_.species_h_over_R(T, th["a"]) * Rk[:, None]
    Yf = Y.reshape(len(Rk), -1)
    cp = np.sum(Yf * cpk, axis=0)
    Rm = np.sum(Yf * Rk[:, None], axis=0)
    cv = cp - Rm
    return cp.reshape(shape), cv.reshape(shape), Rm.reshape(shape), hk.reshape((len(Rk),) + shape)


def primitive_fields(q, T):
    """v = (u, v, w, T, Y_1 .. Y_K) [3 + 1 + K] + shape of q[0]."""
    rho = q[0]
    return np.concatenate([q[1:4] / rho, T[None], q[5:] / rho], axis=0)


def inviscid_flux(q, T, th):
    """F^inv[d][nf] + S and the sound speed c (S = shape of q[0])."""
    rho = q[0]
    u = q[1:4] / rho
    Y = q[5:] / rho
    cp, cv, Rm, _ = _mixture(T, Y, th)
    p = rho * Rm * T
    F = np.empty((3,) + q.shape)
    for d in range(3):
        F[d, 0] = q[1 + d]
        for i in range(3):
            F[d, 1 + i] = q[1 + i] * u[d]
        F[d, 1 + d] += p
        F[d, 4] = (q[4] + p) * u[d]
        F[d, 5:] = q[5:] * u[d]
    c = np.sqrt(cp / cv * p / rho)
    return F, u, c


def viscous_flux(q, T, sigma, th, mu=MU, Pr=PR, Sc=SC):
    """F^v[d][nf] + S from the lifted gradients sigma[d][nv] + S of the
    primitives (u, v, w, T, Y_1 .. Y_K)."""
    rho = q[0]
    u = q[1:4] / rho
    Y = q[5:] / rho
    cp, _, _, hk = _mixture(T, Y, th)
    gu = sigma[:, 0:3]  # gu[d][i] = d u_i / d x_d
    div = gu[0, 0] + gu[1, 1] + gu[2, 2]
    tau = np.empty((3, 3) + q.shape[1:])
    for i in range(3):
        for d in range(3):
            tau[i, d] = mu * (gu[d, i] + gu[i, d])
        tau[i, i] -= mu * (2.0 / 3.0) * div
    kappa = mu * cp / Pr
    rhoD = mu / Sc
    F = np.zeros((3,) + q.shape)
    for d in range(3):
        J = -rhoD * sigma[d, 4:]  # [K] + S
        for i in range(3):
            F[d, 1 + i] = tau[i, d]
        F[d, 4] = u[0] * tau[0, d] + u[1] * tau[1, d] + u[2] * tau[2, d] + kappa * sigma[d, 3] \
            - np.sum(hk * J, axis=0)
        F[d, 5:] = -J
    return F


def gradients(ops, geo, conn, v, elems=None):
    """BR1 pass 1: sigma[d][nv][E][Np] of the nodal fields v[nv][E][Np].
    With elems (element ids), only at those elements:
    sigma[d][nv][len(elems)][Np] (the neighbour traces still come from v)."""
    ix = np.arange(v.shape[1]) if elems is None else np.asarray(elems)
    Nfp = ops["Nfp"]
    fm = ops["Fmask"].reshape(-1)
    rx = geo["rst_x"][ix]  # [E, a, d]
    vE = v[:, ix]
    Dv = [vE @ D.T for D in (ops["Dr"], ops["Ds"], ops["Dt"])]  # D_a v
    vM = vE[:, :, fm]
    vP = v[:, conn["mapP_elem"][ix], conn["mapP_node"][ix]]
    n = np.repeat(geo["normals"][ix], Nfp, axis=1)  # [E, 4Nfp, 3]
    Fs = np.repeat(geo["Fscale"][ix], Nfp, axis=1)
    out = np.empty((3,) + vE.shape)
    for d in range(3):
        vol = sum(rx[None, :, a, d, None] * Dv[a] for a in range(3))
        surf = (Fs * n[..., d] * 0.5 * (vP - vM)) @ ops["LIFT"].T
        out[d] = vol + surf
    return out


def rhs(ops, geo, conn, q, T, th, mech=None, mu=MU, Pr=PR, Sc=SC, sigma=None, split=False, elems=None):
    """Reacting NS right-hand side of q[5 + K][E][Np] at temperatures T[E][Np].
    mech=None leaves out the chemical sources.  sigma (optional) are the
    pass-1 gradients of the whole mesh; computed when not given.  elems
    (optional element ids) restricts the result to those elements (the
    gradients are then computed only where needed: at the elements and at
    their face neighbours).  split=True also returns (sigma at the result's
    elements, term magnitude) where the magnitude is
    sum_a |D_a| |G_a| + |LIFT| |Delta| (the dot-product error-bound scale)."""
    ix = np.arange(q.shape[1]) if elems is None else np.asarray(elems)
    Nfp = ops["Nfp"]
    fm = ops["Fmask"].reshape(-1)
    me, mn = conn["mapP_elem"][ix], conn["mapP_node"][ix]
    if sigma is not None:
        sE, sP = sigma[:, :, ix], sigma[:, :, me, mn]
    elif elems is None:
        sigma = gradients(ops, geo, conn, primitive_fields(q, T))
        sE, sP = sigma, sigma[:, :, me, mn]
    else:
        S = np.unique(np.concatenate([ix, me.ravel()]))
        sS = gradients(ops, geo, conn, primitive_fields(q, T), elems=S)
        sE = sS[:, :, np.searchsorted(S, ix)]
        sP = sS[:, :, np.searchsorted(S, me), mn]
    qE, TE = q[:, ix], T[ix]
    Fi, _, _ = inviscid_flux(qE, TE, th)
    Fv = viscous_flux(qE, TE, sE, th, mu, Pr, Sc)
    F = Fi - Fv
    rx = geo["rst_x"][ix]
    out = np.zeros_like(qE)
    mag = np.zeros_like(qE)
    for a, D in enumerate((ops["Dr"], ops["Ds"], ops["Dt"])):
        G = sum(rx[None, :, a, d, None] * F[d] for d in range(3))
        out -= G @ D.T
        mag += np.abs(G) @ np.abs(D).T

    qM, qP = qE[:, :, fm], q[:, me, mn]
    TM, TP = TE[:, fm], T[me, mn]
    sM = sE[:, :, :, fm]
    FiM, uM, cM = inviscid_flux(qM, TM, th)
    FiP, uP, cP = inviscid_flux(qP, TP, th)
    FvM = viscous_flux(qM, TM, sM, th, mu, Pr, Sc)
    FvP = viscous_flux(qP, TP, sP, th, mu, Pr, Sc)
    n = np.repeat(geo["normals"][ix], Nfp, axis=1)
    Fs = np.repeat(geo["Fscale"][ix], Nfp, axis=1)
    nd = [n[..., d] for d in range(3)]
    un_M = sum(uM[d] * nd[d] for d in range(3))
    un_P = sum(uP[d] * nd[d] for d in range(3))
    lam = np.maximum(np.abs(un_M) + cM, np.abs(un_P) + cP)
    FnI = sum(nd[d] * (FiM[d] - FiP[d]) for d in range(3))
    FnV = sum(nd[d] * (FvM[d] - FvP[d]) for d in range(3))
    delta = Fs * (0.5 * FnI - 0.5 * lam * (qM - qP) - 0.5 * FnV)
    out += delta @ ops["LIFT"].T
    mag += np.abs(delta) @ np.abs(ops["LIFT"]).T
    if mech is not None:
        rho = qE[0]
        out[5:] += th_.sources(rho, TE, qE[5:] / rho, th, mech)
    if split:
        return out, sE, mag
    return out


def temperature(q, th, T0=1000.0, tol=1e-10, max_iter=50):
    """Newton temperature of every node of q (thermo.newton_temperature)."""
    rho, u, v, w, e, Y = th_.primitives(q)
    return th_.newton_temperature(e, Y, th, T0, tol, max_iter)


def gradient_term_magnitude(ops, geo, conn, v, elems=None):
    """Sum of the absolute products in each lifted-gradient entry before
    cancellation (Higham's error scale of a computed sum of products, as in
    euler.rhs_term_magnitude):
      sum_a |da/dx_d| (|D_a| |v|)_i + (|LIFT| (Fscale |n_d| (|v+| + |v-|) / 2))_i,
    shaped like gradients()."""
    ix = np.arange(v.shape[1]) if elems is None else np.asarray(elems)
    Nfp = ops["Nfp"]
    fm = ops["Fmask"].reshape(-1)
    av = np.abs(v[:, ix])
    Dv = [av @ np.abs(D).T for D in (ops["Dr"], ops["Ds"], ops["Dt"])]
    tr = 0.5 * (np.abs(v[:, conn["mapP_elem"][ix], conn["mapP_node"][ix]]) + av[:, :, fm])
    n = np.repeat(geo["normals"][ix], Nfp, axis=1)
    Fs = np.repeat(geo["Fscale"][ix], Nfp, axis=1)
    out = np.empty((3,) + av.shape)
    for d in range(3):
        out[d] = sum(np.abs(geo["rst_x"][ix][None, :, a, d, None]) * Dv[a] for a in range(3))
        out[d] += (Fs * np.abs(n[..., d]) * tr) @ np.abs(ops["LIFT"]).T
    return out


def _viscous_flux_magnitude(q, T, smag, th, mu, Pr, Sc):
    """|F^v| bound with every coefficient and gradient by its magnitude:
    the viscous flux is linear in sigma, so its rounding (and the effect of
    the gradients' own rounding) scales with these absolute sums."""
    rho = q[0]
    u = np.abs(q[1:4] / rho)
    Y = q[5:] / rho
    cp, _, _, hk = _mixture(T, Y, th)
    g = smag[:, 0:3]
    div = g[0, 0] + g[1, 1] + g[2, 2]
    tau = np.empty((3, 3) + q.shape[1:])
    for i in range(3):
        for d in range(3):
            tau[i, d] = mu * (g[d, i] + g[i, d]) + (mu * (2.0 / 3.0) * div if i == d else 0.0)
    F = np.zeros((3,) + q.shape)
    for d in range(3):
        J = (mu / Sc) * smag[d, 4:]
        for i in range(3):
            F[d, 1 + i] = tau[i, d]
        F[d, 4] = u[0] * tau[0, d] + u[1] * tau[1, d] + u[2] * tau[2, d] + (mu * cp / Pr) * smag[d, 3] \
            + np.sum(np.abs(hk) * J, axis=0)
        F[d, 5:] = J
    return F


def rhs_term_magnitude(ops, geo, conn, q, T, th, mech=None, mu=MU, Pr=PR, Sc=SC, elems=None):
    """Sum of the absolute products in each right-hand-side entry before
    cancellation, the scale of its rounding error (Higham, Sec. 3.1): the
    volume and lift sums over |F^inv| + |F^v| with the viscous flux taken
    from the gradients' own magnitudes (gradient_term_magnitude), the face
    flux before its differences cancel, and for the sources
    sum_j W_k |nu''_kj - nu'_kj| |r_j| (1 + Ea_j / (R_u T)): the rate's
    exponential magnifies its argument's rounding by |Ea_j / (R_u T)|."""
    ix = np.arange(q.shape[1]) if elems is None else np.asarray(elems)
    Nfp = ops["Nfp"]
    fm = ops["Fmask"].reshape(-1)
    me, mn = conn["mapP_elem"][ix], conn["mapP_node"][ix]
    S = np.unique(np.concatenate([ix, me.ravel()]))
    sS = gradient_term_magnitude(ops, geo, conn, primitive_fields(q, T), elems=S)
    sE = sS[:, :, np.searchsorted(S, ix)]
    sP = sS[:, :, np.searchsorted(S, me), mn]
    qE, TE = q[:, ix], T[ix]
    Fi, _, _ = inviscid_flux(qE, TE, th)
    AF = np.abs(Fi) + _viscous_flux_magnitude(qE, TE, sE, th, mu, Pr, Sc)
    rx = geo["rst_x"][ix]
    mag = np.zeros_like(qE)
    for a, D in enumerate((ops["Dr"], ops["Ds"], ops["Dt"])):
        mag += sum(np.abs(rx[None, :, a, d, None]) * AF[d] for d in range(3)) @ np.abs(D).T
    qM, qP = qE[:, :, fm], q[:, me, mn]
    TM, TP = TE[:, fm], T[me, mn]
    FiM, uM, cM = inviscid_flux(qM, TM, th)
    FiP, uP, cP = inviscid_flux(qP, TP, th)
    AM = np.abs(FiM) + _viscous_flux_magnitude(qM, TM, sE[:, :, :, fm], th, mu, Pr, Sc)
    AP = np.abs(FiP) + _viscous_flux_magnitude(qP, TP, sP, th, mu, Pr, Sc)
    n = np.repeat(geo["normals"][ix], Nfp, axis=1)
    Fs = np.repeat(geo["Fscale"][ix], Nfp, axis=1)
    nd = [n[..., d] for d in range(3)]
    lam = np.maximum(np.abs(sum(uM[d] * nd[d] for d in range(3))) + cM,
                     np.abs(sum(uP[d] * nd[d] for d in range(3))) + cP)
    face = Fs * (0.5 * sum(np.abs(nd[d]) * (AM[d] + AP[d]) for d in range(3))
                 + 0.5 * lam * (np.abs(qM) + np.abs(qP)))
    mag += face @ np.abs(ops["LIFT"]).T
    if mech is not None:
        K = len(th["W"])
        rho = qE[0]
        C = (rho.ravel()[None] * (qE[5:] / rho).reshape(K, -1)) / th["W"][:, None]
        k = th_.rate_constants(TE, mech)
        r = k.copy()
        for j in range(len(mech["A"])):
            for s_ in range(K):
                if mech["nu_r"][j, s_]:
                    r[j] = r[j] * C[s_] ** mech["nu_r"][j, s_]
        cond = 1.0 + mech["Ea"][:, None] / (th_.R_U * TE.ravel()[None])
        net = np.abs(mech["nu_p"] - mech["nu_r"]).T.astype(np.float64)
        mag[5:] += (th["W"][:, None] * (net @ (np.abs(r) * cond))).reshape((K,) + TE.shape)
    return mag
