"""Shock capturing on the tensor-product hexahedra: smoothness indicator,
artificial viscosity and a positivity-preserving limiter (oracle, FP64).

Test infrastructure only (see the package docstring).

The paper names artificial viscosity and shock limiting among what its shock
cases need (Sec. 5.3) and prints no formula.  Readings:

* Smoothness indicator (Persson & Peraire 2006), per element, of the
  density: expand rho_h in the orthonormal tensor Legendre basis
  Pt_i(r) Pt_j(s) Pt_k(t), Pt_n = sqrt((2n + 1)/2) P_n, and take
  S_e = sum_{max(i,j,k) = p} c^2 / sum_all c^2 (the energy in the modes the
  order-(p - 1) tensor space lacks), s_e = log10 S_e (-inf when S_e = 0).
* Viscosity per element: eps_e = eps0_e * ramp(s_e), with
  ramp = 0 below s0 - kappa, 1 above s0 + kappa and
  (1 + sin(pi (s - s0) / (2 kappa))) / 2 between;
  eps0_e = c_eps * h_e / p * lam_e, h_e the element's smallest edge and
  lam_e = max over its nodes of |u| + c; s0 = -(1 + 4 log10 p) (the p^-4
  decay of a smooth function's top modes), kappa = 1, c_eps = 1/2 unless
  given.
* Artificial viscosity term d q/dt += div(eps grad q) for every conserved
  field, in the BR1 form on the box elements (per direction d, only the two
  faces of direction d have n_d != 0):
    sigma_d = (2/h_d) [ D_d q + sum_side l_side x (n_d (q+ - q-) / 2) ],
    G_d = eps_e sigma_d,
    av = sum_d (2/h_d) [ D_d G_d + sum_side l_side x (n_d (G_d+ - G_d-) / 2) ]
  (central fluxes: (q- + q+)/2 for the gradient, (G- + G+)/2 for the
  viscous flux, no penalty).
* Positivity-preserving limiter (Zhang & Shu 2010), per element, applied to
  every Runge-Kutta stage state: with the cell average qbar (weights
  int l_i over the element) and delta = 1e-10: if min rho < delta, scale
  q <- qbar + theta1 (q - qbar), theta1 = (rhobar - delta) / (rhobar -
  min rho); then if some nodal pressure p_i < delta, scale again with
  theta2 = min_i (pbar - delta) / (pbar - p_i), pbar = p(qbar) (the
  pressure is concave in the conserved variables, so p stays >= delta
  along the segment).  Averages are kept; an element whose own average is
  not admissible is left as it is.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

from .euler import GAMMA, _fluxes
from . import hex as oh

DELTA = 1e-10


def default_params(p: int) -> dict:
    return dict(s0=-(1.0 + 4.0 * math.log10(p)), kappa=1.0, c_eps=0.5, delta=DELTA)


@lru_cache(maxsize=None)
def _modal_inverse(p: int) -> np.ndarray:
    """Inverse of the 1-D orthonormal Legendre Vandermonde V[i, k] = Pt_k(x_i)."""
    x = oh.gll_points(p)
    V = np.zeros((p + 1, p + 1))
    for k in range(p + 1):
        c = np.zeros(k + 1)
        c[k] = 1.0
        V[:, k] = np.polynomial.legendre.legval(x, c) * math.sqrt((2 * k + 1) / 2.0)
    return np.linalg.inv(V)


def smoothness(gr: dict, q: np.ndarray, p: int) -> np.ndarray:
    """s_e = log10 of the top-mode energy fraction of rho, per element."""
    rho = oh._split(q[:1], gr, p)[0]  # [k, j, i, c, b, a]
    Vi = _modal_inverse(p)
    c = rho
    for d in range(3):
        c = np.moveaxis(np.tensordot(c, Vi, axes=([5 - d], [1])), -1, 5 - d)
    c2 = (c * c).reshape(-1, (p + 1) ** 3)
    idx = np.arange(p + 1)
    top = (np.maximum.outer(np.maximum.outer(idx, idx), idx) == p).ravel()  # [c, b, a]
    num, den = c2[:, top].sum(axis=1), c2.sum(axis=1)
    with np.errstate(divide="ignore"):
        return np.log10(num / den)


def viscosity(gr: dict, q: np.ndarray, p: int, prm: dict = None, gamma: float = GAMMA) -> np.ndarray:
    """eps_e per element (see the module notes)."""
    prm = default_params(p) if prm is None else prm
    s = smoothness(gr, q, p)
    s0, kap = prm["s0"], prm["kappa"]
    ramp = np.where(s < s0 - kap, 0.0, np.where(s > s0 + kap, 1.0,
                                                 0.5 * (1.0 + np.sin(np.pi * (s - s0) / (2.0 * kap)))))
    _, (u, v, w), c = _fluxes(q, gamma)
    lam = (np.sqrt(u * u + v * v + w * w) + c).max(axis=1)
    hz, hy, hx = np.meshgrid(gr["h"][2], gr["h"][1], gr["h"][0], indexing="ij")
    h = np.minimum(np.minimum(hx, hy), hz).ravel()
    return prm["c_eps"] * h / p * lam * ramp


def _jump_lift(ops, gr, U, d, p):
    """sum_side l_side x (n_d (U+ - U-) / 2) along direction d, for a field
    array U [f, k, j, i, c, b, a] (the own element's faces of direction d)."""
    P1 = p + 1
    gax, nax = oh._GRID_AXIS[d], oh._NODE_AXIS[d]
    out = np.zeros_like(U)
    for side in (0, 1):
        own = np.take(U, 0 if side == 0 else P1 - 1, axis=nax)
        nbr = np.take(np.roll(U, 1 if side == 0 else -1, axis=gax), P1 - 1 if side == 0 else 0, axis=nax)
        nd = -1.0 if side == 0 else 1.0
        out += np.expand_dims(0.5 * nd * (nbr - own), nax) * ops["lift"][:, side].reshape(
            [P1 if k == nax else 1 for k in range(7)])
    return out


def av_fluxes(ops: dict, gr: dict, q: np.ndarray, eps: np.ndarray):
    """G_d = eps_e sigma_d, shaped [3][5][E][Np]."""
    p = ops["p"]
    qs = oh._split(q, gr, p)
    nx, ny, nz = gr["dims"]
    e3 = eps.reshape(nz, ny, nx)[None, :, :, :, None, None, None]
    G = []
    for d in range(3):
        sig = (oh._apply_1d(ops["D"], qs, d) + _jump_lift(ops, gr, qs, d, p)) * oh._inv_half_h(gr, d)[None]
        G.append((e3 * sig).reshape(q.shape))
    return np.stack(G)


def av_rhs(ops: dict, gr: dict, q: np.ndarray, eps: np.ndarray):
    """The artificial-viscosity term div(eps grad q) in BR1 form."""
    p = ops["p"]
    G = av_fluxes(ops, gr, q, eps)
    out = np.zeros_like(oh._split(q, gr, p))
    for d in range(3):
        Gd = oh._split(G[d], gr, p)
        out += (oh._apply_1d(ops["D"], Gd, d) + _jump_lift(ops, gr, Gd, d, p)) * oh._inv_half_h(gr, d)[None]
    return out.reshape(q.shape)


def shock_rhs(ops: dict, gr: dict, q: np.ndarray, prm: dict = None, gamma: float = GAMMA):
    """Euler RHS plus the artificial-viscosity term at this state's eps."""
    eps = viscosity(gr, q, ops["p"], prm, gamma)
    return oh.rhs(ops, gr, q, gamma) + av_rhs(ops, gr, q, eps)


def cell_weights(p: int) -> np.ndarray:
    """int l_i over the reference cube (node order of the hexahedra)."""
    w1 = oh.operators_1d(p)["M"].sum(axis=1)
    return np.kron(w1, np.kron(w1, w1))


def limit(q: np.ndarray, p: int, delta: float = DELTA, gamma: float = GAMMA) -> np.ndarray:
    """Positivity-preserving limiter, per element (see the module notes)."""
    w = cell_weights(p)
    out = q.copy()
    for e in range(q.shape[1]):
        qe = q[:, e]
        qbar = qe @ w / w.sum()
        pbar = (gamma - 1.0) * (qbar[4] - 0.5 * (qbar[1] ** 2 + qbar[2] ** 2 + qbar[3] ** 2) / qbar[0])
        if not (qbar[0] > delta and pbar > delta):
            continue
        rmin = qe[0].min()
        if rmin < delta:
            th = (qbar[0] - delta) / (qbar[0] - rmin)
            qe = qbar[:, None] + th * (qe - qbar[:, None])
        pn = (gamma - 1.0) * (qe[4] - 0.5 * (qe[1] ** 2 + qe[2] ** 2 + qe[3] ** 2) / qe[0])
        if pn.min() < delta:
            bad = pn < delta
            th = np.min((pbar - delta) / (pbar - pn[bad]))
            qe = qbar[:, None] + th * (qe - qbar[:, None])
        out[:, e] = qe
    return out

