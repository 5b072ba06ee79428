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


# ---------------------------------------------------------------------------
# Overintegration: fluxes evaluated at Gauss-Legendre quadrature points.
#
# Reading (the paper names overintegration among what its shock cases need,
# Sec. 5.3, and prints no formula): the weak form of the same DG method,
#   (M rhs)_i = int_K grad l_i . F(q_h) - int_dK l_i Fhat,
# with the nodal interpolant q_h evaluated at nq Gauss-Legendre points per
# direction (nq = ceil(3 (p + 1) / 2), the "3/2 rule" against the aliasing
# of quadratic nonlinearities), the fluxes and the Lax-Friedrichs flux
# Fhat = 1/2 n.(F(q-) + F(q+)) + 1/2 lam (q- - q+) evaluated there, and the
# integrals taken with that tensor rule.  On the box elements this factors
# into rectangular 1-D contractions: B[k, j] = l_j(xi_k), B'[k, j] = l_j'(xi_k),
# S = M1^{-1} B'^T W, P = M1^{-1} B^T W (both (p+1) x nq), and
#   rhs = sum_d (2 / h_d) [ (S along d, P along the others) F_d(quad)
#                           - sum_side l_side x (P x P) Fhat_face(quad) ].


def oi_points(p: int) -> int:
    """Gauss points per direction of the overintegrated form."""
    return -(-3 * (p + 1) // 2)


@lru_cache(maxsize=None)
def _gauss_cached(n: int):
    """n-point Gauss-Legendre rule, nodes and weights correctly rounded:
    Newton on P_n in 60-digit decimal arithmetic from the FP64 roots,
    w = 2 / ((1 - x^2) P_n'(x)^2)."""
    from decimal import Decimal, localcontext
    xf, _ = np.polynomial.legendre.leggauss(n)
    xs, ws = [], []
    with localcontext() as ctx:
        ctx.prec = _DEC_DIGITS
        for x0 in xf:
            x = Decimal(float(x0))
            for _ in range(8):
                P0, P1 = Decimal(1), x
                d0, d1 = Decimal(0), Decimal(1)
                for k in range(1, n):
                    P2 = ((2 * k + 1) * x * P1 - k * P0) / (k + 1)
                    d2 = ((2 * k + 1) * (P1 + x * d1) - k * d0) / (k + 1)
                    P0, P1, d0, d1 = P1, P2, d1, d2
                x = x - P1 / d1
            P0, P1 = Decimal(1), x
            d0, d1 = Decimal(0), Decimal(1)
            for k in range(1, n):
                P2 = ((2 * k + 1) * x * P1 - k * P0) / (k + 1)
                d2 = ((2 * k + 1) * (P1 + x * d1) - k * d0) / (k + 1)
                P0, P1, d0, d1 = P1, P2, d1, d2
            xs.append(float(x))
            ws.append(float(2 / ((1 - x * x) * d1 * d1)))
    return np.array(xs), np.array(ws)


def gauss_rule(n: int):
    x, w = _gauss_cached(n)
    return x.copy(), w.copy()


@lru_cache(maxsize=None)
def _oi_operators_cached(p: int, nq: int):
    o = operators_1d(p)
    xg = [Fraction(float(v)) for v in o["x"]]
    xq, wq = gauss_rule(nq)
    xq = [Fraction(float(v)) for v in xq]
    wq = [Fraction(float(v)) for v in wq]
    n = p + 1
    L = []
    for j in range(n):
        c = [Fraction(1)]
        for m in range(n):
            if m != j:
                c = _poly_mul(c, [-xg[m] / (xg[j] - xg[m]), 1 / (xg[j] - xg[m])])
        L.append(c)
    val = lambda c, t: sum(ck * t ** k for k, ck in enumerate(c))
    der = lambda c, t: sum(k * c[k] * t ** (k - 1) for k in range(1, len(c)))
    B = [[val(L[j], t) for j in range(n)] for t in xq]
    Bd = [[der(L[j], t) for j in range(n)] for t in xq]

    def integral(c):
        return sum(ck * Fraction(2, k + 1) for k, ck in enumerate(c) if k % 2 == 0)

    M = [[integral(_poly_mul(L[i], L[j])) for j in range(n)] for i in range(n)]
    BtW = [[B[k][j] * wq[k] for k in range(nq)] for j in range(n)]
    BdtW = [[Bd[k][j] * wq[k] for k in range(nq)] for j in range(n)]
    P_ = _solve_exact(M, BtW)
    S_ = _solve_exact(M, BdtW)
    to = lambda A: np.array([[float(v) for v in row] for row in A])
    return dict(p=p, nq=nq, B=to(B), S=to(S_), P=to(P_), lift=o["lift"], xq=np.array([float(v) for v in xq]),
                wq=np.array([float(v) for v in wq]))


def oi_operators(p: int, nq: int = None) -> dict:
    """Overintegration tables: B [nq, p+1], S and P [p+1, nq], lift [p+1, 2],
    Gauss points xq and weights wq; exact at the FP64 points and weights,
    rounded once."""
    o = _oi_operators_cached(p, oi_points(p) if nq is None else nq)
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in o.items()}


def _apply_axes(U, mats):
    """Apply mats[d] (m x n) along the node axis of direction d of U [..., c, b, a]."""
    for d, A in enumerate(mats):
        if A is not None:
            U = _apply_1d(A, U, d)
    return U


def _face_apply(U, A, d):
    """Apply A along both remaining node axes of a face array U [..., s, f]
    (the face of direction d: its two axes are the other two directions,
    slower first)."""
    U = np.moveaxis(np.tensordot(U, A, axes=([-1], [1])), -1, -1)
    U = np.moveaxis(np.tensordot(U, A, axes=([-2], [1])), -1, -2)
    return U


def rhs_overintegrated(oi: dict, gr: dict, q: np.ndarray, gamma: float = GAMMA, split: bool = False):
    """Overintegrated Euler RHS of q[5][E][Np] (see the notes above)."""
    p = oi["p"]
    P1 = p + 1
    qs = _split(q, gr, p)
    qq = _apply_axes(qs, [oi["B"]] * 3)
    F, _, _ = _fluxes(qq, gamma)
    vol = np.zeros_like(qs)
    for d in range(3):
        mats = [oi["P"]] * 3
        mats[d] = oi["S"]
        vol += _apply_axes(F[d], mats) * _inv_half_h(gr, d)[None]
    surf = np.zeros_like(qs)
    for d in range(3):
        gax, nax = _GRID_AXIS[d], _NODE_AXIS[d]
        for side in (0, 1):
            own = np.take(qs, 0 if side == 0 else P1 - 1, axis=nax)
            nbr = np.take(np.roll(qs, 1 if side == 0 else -1, axis=gax), P1 - 1 if side == 0 else 0, axis=nax)
            qm, qp = _face_apply(own, oi["B"], d), _face_apply(nbr, oi["B"], d)
            FM, uM, cM = _fluxes(qm, gamma)
            FP, uP, cP = _fluxes(qp, gamma)
            sgn = -1.0 if side == 0 else 1.0
            lam = np.maximum(np.abs(uM[d]) + cM, np.abs(uP[d]) + cP)
            fhat = 0.5 * sgn * (FM[d] + FP[d]) + 0.5 * lam * (qm - qp)
            surf += _lift(_face_apply(fhat, oi["P"], d), oi["lift"][:, side], gr, d, P1)
    out = (vol - surf).reshape(q.shape)
    if split:
        return out, vol.reshape(q.shape), surf.reshape(q.shape)
    return out


def rhs_overintegrated_term_magnitude(oi: dict, gr: dict, q: np.ndarray, gamma: float = GAMMA):
    """Sum of the absolute products in each entry of the overintegrated RHS
    before cancellation: the interpolation to the quadrature points taken
    with |B| and |q|, the fluxes there by their absolute values, the volume
    and face contractions with |S|, |P| and |lift|, the face flux's terms
    absolutely (1/2 (|F(q-)| + |F(q+)|) + 1/2 lam (|q-| + |q+|))."""
    p = oi["p"]
    P1 = p + 1
    aB, aS, aP = np.abs(oi["B"]), np.abs(oi["S"]), np.abs(oi["P"])
    qs = _split(q, gr, p)
    qq = _apply_axes(qs, [oi["B"]] * 3)
    F, _, _ = _fluxes(qq, gamma)
    # the interpolated state's own rounding scales with |B| |q|; the fluxes
    # are products of the interpolated fields, so their magnitude is taken at
    # the absolutely interpolated state (|B| x |B| x |B|) |q| where it is larger
    Fa, _, _ = _fluxes(np.maximum(np.abs(qq), _apply_axes(np.abs(qs), [aB] * 3)) * np.sign(qq + (qq == 0)), gamma)
    out = np.zeros_like(qs)
    for d in range(3):
        mats = [aP] * 3
        mats[d] = aS
        out += _apply_axes(np.maximum(np.abs(F[d]), np.abs(Fa[d])), mats) * _inv_half_h(gr, d)[None]
    for d in range(3):
        gax, nax = _GRID_AXIS[d], _NODE_AXIS[d]
        for side in (0, 1):
            own = np.take(qs, 0 if side == 0 else P1 - 1, axis=nax)
            nbr = np.take(np.roll(qs, 1 if side == 0 else -1, axis=gax), P1 - 1 if side == 0 else 0, axis=nax)
            qm, qp = _face_apply(own, oi["B"], d), _face_apply(nbr, oi["B"], d)
            qma, qpa = _face_apply(np.abs(own), aB, d), _face_apply(np.abs(nbr), aB, d)
            FM, uM, cM = _fluxes(qm, gamma)
            FP, uP, cP = _fluxes(qp, gamma)
            lam = np.maximum(np.abs(uM[d]) + cM, np.abs(uP[d]) + cP)
            term = 0.5 * (np.abs(FM[d]) + np.abs(FP[d])) + 0.5 * lam * (qma + qpa)
            out += _lift(_face_apply(term, aP, d), np.abs(oi["lift"][:, side]), gr, d, P1)
    return out.reshape(q.shape)


def oi_contraction_length(p: int) -> int:
    """Longest chain of sums into one overintegrated entry: the three
    interpolation passes (p + 1 terms each), the three projection passes (nq
    each), the six faces' two interpolation and two projection passes."""
    nq = oi_points(p)
    return 3 * (p + 1) + 3 * nq + 6 + 2 * (p + 1) + 2 * nq
