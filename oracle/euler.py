"""Strong-form nodal DG right-hand side of the compressible Euler equations
(oracle, FP64).  Test infrastructure only (see the package docstring).

The paper solves the Euler equations with nodal DG and explicit RK4 on a
periodic isentropic vortex (Sec. 5.2) and gives no formula; this is the
textbook strong form (Hesthaven & Warburton) read as follows:

  q = (rho, m_x, m_y, m_z, E),  p = (gamma - 1)(E - |m|^2 / (2 rho)),
  c = sqrt(gamma p / rho),
  F_d(q) = (m_d, m_x m_d / rho + p delta_xd, m_y m_d / rho + p delta_yd,
            m_z m_d / rho + p delta_zd, (E + p) m_d / rho)

  volume:   vol_i = sum_{a in r,s,t} sum_j D_a[i, j] G_{a,j},
            G_{a,j} = sum_d (da/dx_d) F_d(q_j)
  surface:  at face node (f, m) with own node Fmask[f][m] (q-) and matched
            neighbour node (q+), outward unit normal n, local Lax-Friedrichs
            speed lam = max(|u-.n| + c-, |u+.n| + c+),
            Delta = Fscale_f [ 1/2 n.(F(q-) - F(q+)) - 1/2 lam (q- - q+) ]
  rhs_i = -vol_i + sum_{(f, m)} LIFT[i, (f, m)] Delta_{(f, m)}.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def _fluxes(q, gamma):
    rho, mx, my, mz, E = q
    u, v, w = mx / rho, my / rho, mz / rho
    p = (gamma - 1.0) * (E - 0.5 * (mx * u + my * v + mz * w))
    Fx = np.stack([mx, mx * u + p, my * u, mz * u, (E + p) * u])
    Fy = np.stack([my, mx * v, my * v + p, mz * v, (E + p) * v])
    Fz = np.stack([mz, mx * w, my * w, mz * w + p, (E + p) * w])
    c = np.sqrt(gamma * p / rho)
    return (Fx, Fy, Fz), (u, v, w), c


def rhs(ops: dict, geo: dict, conn: dict, q: np.ndarray, gamma: float = GAMMA,
        elems=None, split: bool = False):
    """Euler RHS for q[5][E][Np].

    elems: optional index array; only those elements' RHS rows are computed
    (their neighbours' traces are read from q).  Returns rhs[5][len(elems)][Np]
    (or [5][E][Np]).  With split=True returns (rhs, volume_part, surface_part).
    """
    E = q.shape[1]
    idx = np.arange(E) if elems is None else np.asarray(elems, dtype=np.int64)
    qe = q[:, idx, :]
    (Fx, Fy, Fz), _, _ = _fluxes(qe, gamma)
    rx = geo["rst_x"][idx]  # [n, (r,s,t), x]
    vol = np.zeros_like(qe)
    for a, D in enumerate((ops["Dr"], ops["Ds"], ops["Dt"])):
        G = rx[None, :, a, 0, None] * Fx + rx[None, :, a, 1, None] * Fy + rx[None, :, a, 2, None] * Fz
        vol += G @ D.T

    Nfp = ops["Nfp"]
    fm = ops["Fmask"].reshape(-1)  # face-major own node of each face node
    qM = qe[:, :, fm]
    qP = q[:, conn["mapP_elem"][idx], conn["mapP_node"][idx]]
    n = np.repeat(geo["normals"][idx], Nfp, axis=1)  # [n, 4Nfp, 3]
    Fs = np.repeat(geo["Fscale"][idx], Nfp, axis=1)  # [n, 4Nfp]
    (FxM, FyM, FzM), (uM, vM, wM), cM = _fluxes(qM, gamma)
    (FxP, FyP, FzP), (uP, vP, wP), cP = _fluxes(qP, gamma)
    nx, ny, nz = n[..., 0], n[..., 1], n[..., 2]
    FnM = nx * FxM + ny * FyM + nz * FzM
    FnP = nx * FxP + ny * FyP + nz * FzP
    lam = np.maximum(np.abs(uM * nx + vM * ny + wM * nz) + cM, np.abs(uP * nx + vP * ny + wP * nz) + cP)
    delta = Fs * (0.5 * (FnM - FnP) - 0.5 * lam * (qM - qP))
    surf = delta @ ops["LIFT"].T
    out = -vol + surf
    if split:
        return out, vol, surf
    return out


def rhs_term_magnitude(ops: dict, geo: dict, conn: dict, q: np.ndarray, gamma: float = GAMMA, elems=None):
    """Magnitude of the products summed into each RHS entry, taken before any
    cancellation, the scale of the floating-point error bound of a computed
    sum of products (Higham, Accuracy and Stability of Numerical Algorithms,
    Sec. 3.1: |fl(sum x_k y_k) - sum x_k y_k| <= gamma_n sum |x_k y_k|):

      T_i = sum_a sum_j |D_a[i, j]| sum_d |da/dx_d| |F_d(q_j)|
            + sum_{(f,m)} |LIFT[i, (f,m)]| Fscale_f [ 1/2 sum_d |n_d| (|F_d(q-)| + |F_d(q+)|)
                                                     + 1/2 lam (|q-| + |q+|) ].

    The contravariant flux sum_d (da/dx_d) F_d and the face flux n.F(q-) -
    n.F(q+) are themselves sums whose terms may cancel; their rounding is
    relative to these absolute sums, not to the (smaller) results.  Same
    shape as rhs()."""
    E = q.shape[1]
    idx = np.arange(E) if elems is None else np.asarray(elems, dtype=np.int64)
    qe = q[:, idx, :]
    (Fx, Fy, Fz), _, _ = _fluxes(qe, gamma)
    rx = geo["rst_x"][idx]
    out = np.zeros_like(qe)
    for a, D in enumerate((ops["Dr"], ops["Ds"], ops["Dt"])):
        G = sum(np.abs(rx[None, :, a, d, None]) * np.abs(F) for d, F in enumerate((Fx, Fy, Fz)))
        out += G @ np.abs(D).T
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
    face = Fs * (0.5 * (np.abs(nx) * (np.abs(FxM) + np.abs(FxP)) + np.abs(ny) * (np.abs(FyM) + np.abs(FyP))
                        + np.abs(nz) * (np.abs(FzM) + np.abs(FzP))) + 0.5 * lam * (np.abs(qM) + np.abs(qP)))
    return out + face @ np.abs(ops["LIFT"]).T


def contraction_length(p: int) -> int:
    """K = 3 Np + 4 Nfp: products summed into one RHS entry (volume terms of
    three directions over Np nodes, lift terms over 4 Nfp face nodes)."""
    Np = (p + 1) * (p + 2) * (p + 3) // 6
    Nfp = (p + 1) * (p + 2) // 2
    return 3 * Np + 4 * Nfp


def max_wave_speed(q: np.ndarray, gamma: float = GAMMA) -> float:
    """max over nodes of |u| + c."""
    _, (u, v, w), c = _fluxes(q, gamma)
    return float(np.max(np.sqrt(u * u + v * v + w * w) + c))


def cfl_dt(ops: dict, geo: dict, q: np.ndarray, cfl: float = 0.2, gamma: float = GAMMA) -> float:
    """dt = CFL / (lambda_max (p+1)^2 max Fscale), the step-size reading used
    for all runs (computed once from the initial state)."""
    p = ops["p"]
    return cfl / (max_wave_speed(q, gamma) * (p + 1) ** 2 * float(np.max(geo["Fscale"])))
