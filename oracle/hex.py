"""Nodal DG on tensor-product hexahedra (oracle, FP64).

Test infrastructure only (see the package docstring).

The paper's own Euler benchmarks run on tensor-product elements (Sec. 5.2:
the p = 4 isentropic vortex and the p = 1 advection case, "TPEs") and prints
no formula; this module is the textbook nodal DG method on them, read as
follows:

* Mesh: a periodic rectilinear box; cell (i, j, k) is the axis-aligned box
  [gx_i, gx_{i+1}] x [gy_j, gy_{j+1}] x [gz_k, gz_{k+1}] with element id
  e = i + nx (j + ny k).  The map from the reference cube [-1, 1]^3 is affine
  with the diagonal Jacobian diag(h_x, h_y, h_z) / 2.
* Nodes: the tensor product of the p + 1 Legendre-Gauss-Lobatto (LGL) points;
  node (a, b, c) at (r_a, s_b, t_c) has index a + (p + 1)(b + (p + 1) c)
  (r fastest).  Face nodes of the x faces are the nodes with a = 0 (x-) or
  a = p (x+), ordered by (b, c); the neighbour across a face holds the
  matching node at the same (b, c), so no orientation map is needed.
* 1-D operators on the LGL points: D1[i, j] = l_j'(x_i),
  M1[i, j] = int_{-1}^{1} l_i l_j (exact, not the lumped LGL weights), and the
  lift vectors lL = M1^{-1} e_0, lR = M1^{-1} e_p.  They are the exact values
  at the FP64 points, computed in rational arithmetic and rounded once.
* 3-D operators factor: D_r = I x I x D1 (acting on a), the mass matrix is
  J M1 x M1 x M1 and the face matrix of face x- is (h_y h_z / 4)
  e_0 x M1 x M1, so M^{-1} E of face x- is (2 / h_x) lL x I x I: the lift
  acts along single lines.
* Euler right-hand side, strong form with the local Lax-Friedrichs flux and
  pointwise lam = max(|u-.n| + c-, |u+.n| + c+), as for the tetrahedra:
    rhs = - sum_d (2 / h_d) D_d F_d + sum_faces (2 / h_d) l_side x Delta,
    Delta = 1/2 n.(F(q-) - F(q+)) - 1/2 lam (q- - q+).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import numpy as np

from .euler import _fluxes, GAMMA
from .reference_element import _DEC_DIGITS, _lgl_points_dec, _solve_exact

__all__ = ["gll_points", "operators_1d", "grid", "node_coordinates", "rhs", "rhs_term_magnitude", "cfl_dt",
           "full_operators"]


@lru_cache(maxsize=None)
def _gll_cached(p: int) -> np.ndarray:
    from decimal import localcontext
    with localcontext() as ctx:
        ctx.prec = _DEC_DIGITS
        return np.array([float(x) for x in _lgl_points_dec(p)])


def gll_points(p: int) -> np.ndarray:
    """The p + 1 LGL points on [-1, 1], ascending, correctly rounded."""
    if p < 1 or p > 8:
        raise ValueError("orders 1..8")
    return _gll_cached(p).copy()


def _poly_mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


@lru_cache(maxsize=None)
def _operators_1d_cached(p: int):
    x = [Fraction(float(v)) for v in gll_points(p)]
    n = p + 1
    # Lagrange polynomials as coefficient lists (ascending powers)
    L = []
    for j in range(n):
        c = [Fraction(1)]
        for m in range(n):
            if m != j:
                c = _poly_mul(c, [-x[m] / (x[j] - x[m]), 1 / (x[j] - x[m])])
        L.append(c)

    def deriv_at(c, t):
        return sum(k * c[k] * t ** (k - 1) for k in range(1, len(c)))

    D = [[deriv_at(L[j], x[i]) for j in range(n)] for i in range(n)]

    def integral(c):  # int_{-1}^{1} sum c_k t^k
        return sum(ck * Fraction(2, k + 1) for k, ck in enumerate(c) if k % 2 == 0)

    M = [[integral(_poly_mul(L[i], L[j])) for j in range(n)] for i in range(n)]
    e = [[Fraction(int(i == 0)), Fraction(int(i == p))] for i in range(n)]
    lift = _solve_exact(M, e)
    to = lambda A: np.array([[float(v) for v in row] for row in A])
    return dict(p=p, x=gll_points(p), D=to(D), M=to(M), lift=to(lift))


def operators_1d(p: int) -> dict:
    """x (LGL points), D (D1), M (M1), lift [p + 1, 2] = [lL | lR]."""
    o = _operators_1d_cached(p)
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in o.items()}


def grid(gx, gy, gz) -> dict:
    """Cell sizes of a periodic rectilinear grid given by its lines."""
    g = [np.asarray(v, dtype=np.float64) for v in (gx, gy, gz)]
    h = [np.diff(v) for v in g]
    if any(np.any(v <= 0) for v in h):
        raise ValueError("grid lines must increase strictly")
    return dict(lines=g, h=h, dims=tuple(len(v) for v in h))


def node_coordinates(gr: dict, p: int) -> np.ndarray:
    """[E, Np, 3] physical node coordinates, element and node order as above."""
    x = gll_points(p)
    nx, ny, nz = gr["dims"]
    cx = [gr["lines"][d][:-1, None] + 0.5 * (1.0 + x)[None, :] * gr["h"][d][:, None] for d in range(3)]
    X = np.empty((nz, ny, nx, p + 1, p + 1, p + 1, 3))
    X[..., 0] = cx[0][None, None, :, None, None, :]
    X[..., 1] = cx[1][None, :, None, None, :, None]
    X[..., 2] = cx[2][:, None, None, :, None, None]
    return X.reshape(nx * ny * nz, (p + 1) ** 3, 3)


def _split(q, gr, p):
    nx, ny, nz = gr["dims"]
    P = p + 1
    return q.reshape(q.shape[0], nz, ny, nx, P, P, P)  # (f, k, j, i, c, b, a)


# axis of the element grid and of the node block, per direction d = x, y, z
_GRID_AXIS = (3, 2, 1)
_NODE_AXIS = (6, 5, 4)


def _inv_half_h(gr, d):
    """2 / h_d broadcast over (k, j, i, c, b, a)."""
    v = 2.0 / gr["h"][d]
    shape = [1] * 6
    shape[_GRID_AXIS[d] - 1] = len(v)
    return v.reshape(shape)


def _apply_1d(A, U, d):
    """A (m x n) applied along node axis of direction d of U [..., c, b, a]."""
    ax = _NODE_AXIS[d]
    return np.moveaxis(np.tensordot(U, A, axes=([ax], [1])), -1, ax)


def _faces(q, gr, p, gamma, d, side, absolute=False):
    """Delta (or its term magnitude) on the face of direction d, side 0 (-)
    or 1 (+) of every element: arrays [f, k, j, i, ...2 node axes...] with
    the node axis of direction d removed."""
    P = p + 1
    qs = _split(q, gr, p)
    gax, nax = _GRID_AXIS[d], _NODE_AXIS[d]
    own = np.take(qs, 0 if side == 0 else P - 1, axis=nax)
    nbr_all = np.roll(qs, 1 if side == 0 else -1, axis=gax)
    nbr = np.take(nbr_all, P - 1 if side == 0 else 0, axis=nax)
    sgn = -1.0 if side == 0 else 1.0
    FM, uM, cM = _fluxes(own, gamma)
    FP, uP, cP = _fluxes(nbr, gamma)
    lam = np.maximum(np.abs(uM[d]) + cM, np.abs(uP[d]) + cP)
    if absolute:
        return 0.5 * (np.abs(FM[d]) + np.abs(FP[d])) + 0.5 * lam * (np.abs(own) + np.abs(nbr))
    return 0.5 * sgn * (FM[d] - FP[d]) - 0.5 * lam * (own - nbr)


def _lift(delta, lift_vec, gr, d, P):
    """(2 / h_d) lift_vec along direction d times the face values."""
    nax = _NODE_AXIS[d]
    out = np.expand_dims(delta, nax) * lift_vec.reshape([P if k == nax else 1 for k in range(7)])
    return out * _inv_half_h(gr, d)[None]


def rhs(ops: dict, gr: dict, q: np.ndarray, gamma: float = GAMMA, split: bool = False):
    """Euler RHS of q[5][E][Np] on the rectilinear hex grid (see the module notes)."""
    p = ops["p"]
    P = p + 1
    qs = _split(q, gr, p)
    F, _, _ = _fluxes(qs, gamma)
    vol = np.zeros_like(qs)
    for d in range(3):
        vol += _apply_1d(ops["D"], F[d], d) * _inv_half_h(gr, d)[None]
    surf = np.zeros_like(qs)
    for d in range(3):
        for side in (0, 1):
            surf += _lift(_faces(q, gr, p, gamma, d, side), ops["lift"][:, side], gr, d, P)
    out = (-vol + surf).reshape(q.shape)
    if split:
        return out, vol.reshape(q.shape), surf.reshape(q.shape)
    return out


def rhs_term_magnitude(ops: dict, gr: dict, q: np.ndarray, gamma: float = GAMMA):
    """Sum of the absolute products in each RHS entry before cancellation
    (Higham's error scale of a computed sum of products, as for the
    tetrahedra): sum_d (2/h_d) |D1| |F_d| along d + sum_faces (2/h_d) |l_side|
    x [1/2 (|F_d(q-)| + |F_d(q+)|) + 1/2 lam (|q-| + |q+|)]."""
    p = ops["p"]
    P = p + 1
    qs = _split(q, gr, p)
    F, _, _ = _fluxes(qs, gamma)
    out = np.zeros_like(qs)
    for d in range(3):
        out += _apply_1d(np.abs(ops["D"]), np.abs(F[d]), d) * _inv_half_h(gr, d)[None]
        for side in (0, 1):
            out += _lift(_faces(q, gr, p, gamma, d, side, absolute=True), np.abs(ops["lift"][:, side]), gr, d, P)
    return out.reshape(q.shape)


def contraction_length(p: int) -> int:
    """Products summed into one RHS entry: 3 (p + 1) volume terms and 6 lift terms."""
    return 3 * (p + 1) + 6


def cfl_dt(gr: dict, q: np.ndarray, p: int, cfl: float = 0.2, gamma: float = GAMMA) -> float:
    """dt = CFL / (lambda_max (p + 1)^2 max_d (2 / h_d))."""
    _, (u, v, w), c = _fluxes(q, gamma)
    lam = float(np.max(np.sqrt(u * u + v * v + w * w) + c))
    hmin = min(float(np.min(h)) for h in gr["h"])
    return cfl / (lam * (p + 1) ** 2 * 2.0 / hmin)


def full_operators(p: int) -> dict:
    """Unfactored 3-D reference operators built from their definitions, for
    pins of the factored form: Dr, Ds, Dt (Np x Np), the mass matrix M3 =
    M1 x M1 x M1, the face matrices E3 [Np, 6 (p+1)^2] (face order x-, x+,
    y-, y+, z-, z+; face nodes ordered by the two remaining indices, first
    index fastest) and LIFT3 = M3^{-1} E3 (reference cube, h = 2)."""
    o = operators_1d(p)
    P = p + 1
    I = np.eye(P)
    # index a + P (b + P c): kron(C, B, A) acts on (c, b, a)
    Dr = np.kron(I, np.kron(I, o["D"]))
    Ds = np.kron(I, np.kron(o["D"], I))
    Dt = np.kron(o["D"], np.kron(I, I))
    M3 = np.kron(o["M"], np.kron(o["M"], o["M"]))
    Np = P ** 3
    E3 = np.zeros((Np, 6 * P * P))
    idx = np.arange(Np).reshape(P, P, P)  # [c, b, a]
    for d in range(3):
        for side in (0, 1):
            f = 2 * d + side
            k = 0 if side == 0 else P - 1
            nodes = np.take(idx, k, axis=2 - d)  # [slow, fast] of the remaining two indices
            Mf = np.kron(o["M"], o["M"])  # face mass on (slow, fast) = (second, first remaining index)
            for m, node_m in enumerate(nodes.ravel()):
                for n, node_n in enumerate(nodes.ravel()):
                    E3[node_n, f * P * P + m] = Mf[n, m]
    LIFT3 = np.linalg.solve(M3, E3)
    return dict(Dr=Dr, Ds=Ds, Dt=Dt, M3=M3, E3=E3, LIFT3=LIFT3)
