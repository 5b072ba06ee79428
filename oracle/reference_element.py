"""Reference tetrahedron: nodes, Lagrange operators, mass and lift (oracle, FP64).

Test infrastructure only (see the package docstring).

Readings (the paper cites Hesthaven & Warburton's nodal DG for its per-element
node layout, Sec. 1 and Fig. "dg_mesh", but prints no formula):

* Reference tet with vertices v1=(-1,-1,-1), v2=(1,-1,-1), v3=(-1,1,-1),
  v4=(-1,-1,1); faces  f0 = {t=-1} (v1 v2 v3), f1 = {s=-1} (v1 v2 v4),
  f2 = {r+s+t=-1} (v2 v3 v4), f3 = {r=-1} (v1 v3 v4).
* Node index order: equidistant lattice walked with t outermost, then s, then r
  innermost; the warp & blend map (Warburton 2006) moves each lattice point and
  keeps its index.  On edges the map is exactly the Legendre-Gauss-Lobatto
  distribution; for p <= 3 the blend parameter alpha is 0.
* Operators are defined basis-free: l_j is the Lagrange polynomial of node j,
  Dr[i, j] = d l_j / dr (x_i), M[i, j] = int_T l_i l_j, and the face matrix
  E[i, (f, m)] = int_{face f} l_i l_{Fmask[f][m]} with the face parametrised by
  two reference coordinates (area 2): (r, s) on f0, (r, t) on f1, (s, t) on f2
  and f3.  LIFT = M^{-1} E.
* Nodes are formed in 60-digit decimal arithmetic and rounded to FP64 once,
  so they are the correctly rounded warp & blend points.  The operators are
  then the exact operators of the Lagrange basis at those FP64 nodes, computed
  in rational arithmetic (monomial Vandermonde, Dirichlet integrals of
  monomials over the element and its faces) and rounded to FP64 once.  An FP64
  route through a Vandermonde matrix loses accuracy with its condition number
  (at p = 4 a Legendre tensor basis gives errors of hundreds of units in the
  last place of a row's largest entry); the exact route leaves only the final
  rounding.  The FP64 route (Legendre tensor basis P_a(r) P_b(s) P_c(t) and
  collapsed Gauss quadrature) is kept as `operators_by_quadrature`, an
  independent cross-check of the definitions.
"""
from __future__ import annotations

import math
from decimal import Decimal, localcontext
from fractions import Fraction
from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg

TOL = 1e-10

# Warp & blend alpha per order (Warburton 2006 optimised values as tabulated in
# Hesthaven & Warburton, Sec. 10.1); orders 1..3 use alpha = 0.
_ALPHA = {1: 0.0, 2: 0.0, 3: 0.0, 4: 0.1002}
_ALPHA_TEXT = {1: "0", 2: "0", 3: "0", 4: "0.1002"}

# equilateral tetrahedron used by the warp & blend construction, vertex a <-> v_a
_VEQ = np.array([
    [-1.0, -1.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
    [1.0, -1.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
    [0.0, 2.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
    [0.0, 0.0, 3.0 / math.sqrt(6.0)],
])

# local vertices (0-based) of each face, in the order v_a listed above
FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))


def n_nodes(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def n_face_nodes(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def lgl_points(p: int) -> np.ndarray:
    """p+1 Legendre-Gauss-Lobatto points on [-1, 1], ascending."""
    if p == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    interior = np.sort(npleg.legroots(npleg.legder(c)).real)
    return np.concatenate([[-1.0], interior, [1.0]])


def equidistant_lattice(p: int) -> np.ndarray:
    """Lattice points (r, s, t) in the contract's index order (t outer, r inner)."""
    pts = []
    for n in range(p + 1):
        for m in range(p + 1 - n):
            for q in range(p + 1 - n - m):
                pts.append((-1.0 + 2.0 * q / p, -1.0 + 2.0 * m / p, -1.0 + 2.0 * n / p))
    return np.array(pts)


def barycentric(rst: np.ndarray) -> np.ndarray:
    """Barycentric coordinates (lambda_1..lambda_4) w.r.t. v1..v4."""
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    return np.stack([-(1.0 + r + s + t) / 2.0, (1.0 + r) / 2.0, (1.0 + s) / 2.0, (1.0 + t) / 2.0], axis=1)


_DEC_DIGITS = 60


def _lgl_points_dec(p: int):
    """p+1 LGL points as Decimals: the end points and the roots of P_p',
    refined by Newton's method from the FP64 roots."""
    x0 = lgl_points(p)
    out = [Decimal(-1)]
    for xf in x0[1:-1]:
        x = Decimal(float(xf))
        for _ in range(8):
            # P_n, P_n', P_n'' by the three-term recurrence
            P0, P1 = Decimal(1), x
            d0, d1 = Decimal(0), Decimal(1)
            e0, e1 = Decimal(0), Decimal(0)
            for n in range(1, p):
                P2 = ((2 * n + 1) * x * P1 - n * P0) / (n + 1)
                d2 = ((2 * n + 1) * (P1 + x * d1) - n * d0) / (n + 1)
                e2 = ((2 * n + 1) * (2 * d1 + x * e1) - n * e0) / (n + 1)
                P0, P1, d0, d1, e0, e1 = P1, P2, d1, d2, e1, e2
            x = x - d1 / e1
        out.append(x)
    out.append(Decimal(1))
    return out


def _warp_over_bubble_dec(p: int, x, xeq, disp):
    """w(x) / (1 - x^2) at one point, where w is the degree-p interpolant on
    equidistant points of the displacement (LGL point - equidistant point).
    The endpoint displacements are zero, so the quotient is a polynomial; it
    is formed by dropping the (x - 1)(x + 1) factor from each interior
    Lagrange polynomial ((x + 1)(x - 1) = -(1 - x^2))."""
    out = Decimal(0)
    for i in range(1, p):
        num, den = Decimal(1), Decimal(1)
        for j in range(p + 1):
            if j == i:
                continue
            den *= xeq[i] - xeq[j]
            if j not in (0, p):
                num *= x - xeq[j]
        out -= disp[i] * num / den
    return out


@lru_cache(maxsize=None)
def _nodes_cached(p: int) -> np.ndarray:
    if p < 1 or p > 4:
        raise ValueError("orders 1..4 are supported")
    return warp_blend_nodes(p, _ALPHA_TEXT[p])


def warp_blend_nodes(p: int, alpha_text: str) -> np.ndarray:
    """Warp & blend nodes of order p with blend parameter alpha (a decimal
    string), computed in 60-digit decimal arithmetic and rounded to FP64."""
    with localcontext() as ctx:
        ctx.prec = _DEC_DIGITS
        D = Decimal
        alpha = D(alpha_text)
        tol = D("1e-10")
        s3, s6 = D(3).sqrt(), D(6).sqrt()
        veq = [(D(-1), -1 / s3, -1 / s6), (D(1), -1 / s3, -1 / s6), (D(0), 2 / s3, -1 / s6), (D(0), D(0), 3 / s6)]
        xeq = [D(-1) + D(2 * i) / p for i in range(p + 1)]
        lgl = _lgl_points_dec(p)
        disp = [lgl[i] - xeq[i] for i in range(p + 1)]
        out = []
        for n in range(p + 1):
            for m in range(p + 1 - n):
                for q in range(p + 1 - n - m):
                    lam = [D(p - n - m - q) / p, D(q) / p, D(m) / p, D(n) / p]
                    X = [sum(lam[a] * veq[a][c] for a in range(4)) for c in range(3)]
                    shift = [D(0)] * 3
                    edge_shift = None
                    for opp in range(4):  # face opposite vertex `opp`
                        fv = [v for v in range(4) if v != opp]
                        La = lam[opp]
                        Lf = [lam[v] for v in fv]
                        sf = [D(0)] * 3
                        for k in range(3):
                            a, b = (k + 1) % 3, (k + 2) % 3  # edge a -> b, opposite vertex k
                            w = 4 * _warp_over_bubble_dec(p, Lf[b] - Lf[a], xeq, disp) * Lf[a] * Lf[b] \
                                * (1 + (alpha * Lf[k]) ** 2)
                            d = [veq[fv[b]][c] - veq[fv[a]][c] for c in range(3)]
                            nd = (d[0] ** 2 + d[1] ** 2 + d[2] ** 2).sqrt()
                            for c in range(3):
                                sf[c] += w * d[c] / nd
                        blend = Lf[0] * Lf[1] * Lf[2]
                        denom = (Lf[0] + La / 2) * (Lf[1] + La / 2) * (Lf[2] + La / 2)
                        if denom > tol:
                            blend = (1 + (alpha * La) ** 2) * blend / denom
                        for c in range(3):
                            shift[c] += blend * sf[c]
                        if La < tol and sum(1 for x in Lf if x > tol) < 3:
                            edge_shift = sf
                    if edge_shift is not None:
                        shift = edge_shift
                    X = [X[c] + shift[c] for c in range(3)]
                    # X - V1 = sum_d (1 + rst_d)/2 (V_{d+1} - V1): Cramer's rule
                    cols = [[(veq[d + 1][c] - veq[0][c]) / 2 for c in range(3)] for d in range(3)]
                    b = [X[c] - veq[0][c] for c in range(3)]

                    def det3(c0, c1, c2):
                        return (c0[0] * (c1[1] * c2[2] - c1[2] * c2[1]) - c1[0] * (c0[1] * c2[2] - c0[2] * c2[1])
                                + c2[0] * (c0[1] * c1[2] - c0[2] * c1[1]))
                    det = det3(*cols)
                    rst = [det3(*(b if k == d else cols[k] for k in range(3))) / det - 1 for d in range(3)]
                    out.append([float(v) for v in rst])
    return np.array(out)


def nodes(p: int) -> np.ndarray:
    """Warp & blend nodes [Np, 3] in reference coordinates (r, s, t)."""
    return _nodes_cached(p).copy()


# ---------------------------------------------------------------------------
# polynomial space: Legendre tensor basis with total degree <= p

def _multi_indices(p: int):
    return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]


def _leg(n: int, x: np.ndarray, der: int = 0) -> np.ndarray:
    c = np.zeros(n + 1)
    c[n] = 1.0
    if der:
        c = npleg.legder(c, der)
    return npleg.legval(x, c)


def basis_3d(p: int, rst: np.ndarray, der=(0, 0, 0)) -> np.ndarray:
    """[npts, Np] values (or partial derivatives) of the tensor Legendre basis."""
    cols = []
    for (a, b, c) in _multi_indices(p):
        cols.append(_leg(a, rst[:, 0], der[0]) * _leg(b, rst[:, 1], der[1]) * _leg(c, rst[:, 2], der[2]))
    return np.stack(cols, axis=1)


def lagrange_at(p: int, pts: np.ndarray, der=(0, 0, 0)) -> np.ndarray:
    """[npts, Np]: (derivatives of) the nodal Lagrange polynomials at pts."""
    V = basis_3d(p, nodes(p))
    B = basis_3d(p, pts, der)
    return np.linalg.solve(V.T, B.T).T


def tet_quadrature(nq: int):
    """Collapsed (Duffy) Gauss-Legendre rule on the reference tet."""
    x, w = npleg.leggauss(nq)
    a, b, c = np.meshgrid(x, x, x, indexing="ij")
    wa, wb, wc = np.meshgrid(w, w, w, indexing="ij")
    r = (1 + a) * (1 - b) * (1 - c) / 4 - 1
    s = (1 + b) * (1 - c) / 2 - 1
    t = c
    wt = wa * wb * wc * (1 - b) * (1 - c) ** 2 / 8
    return np.stack([r.ravel(), s.ravel(), t.ravel()], axis=1), wt.ravel()


def tri_quadrature(nq: int):
    """Collapsed Gauss-Legendre rule on the triangle {u, v >= -1, u + v <= 0}."""
    x, w = npleg.leggauss(nq)
    a, b = np.meshgrid(x, x, indexing="ij")
    wa, wb = np.meshgrid(w, w, indexing="ij")
    u = (1 + a) * (1 - b) / 2 - 1
    v = b
    wt = wa * wb * (1 - b) / 2
    return np.stack([u.ravel(), v.ravel()], axis=1), wt.ravel()


def face_point_to_rst(face: int, uv: np.ndarray) -> np.ndarray:
    """Map face parameters (two reference coordinates) to (r, s, t)."""
    u, v = uv[:, 0], uv[:, 1]
    m1 = -np.ones_like(u)
    if face == 0:
        return np.stack([u, v, m1], axis=1)
    if face == 1:
        return np.stack([u, m1, v], axis=1)
    if face == 2:
        return np.stack([-1.0 - u - v, u, v], axis=1)
    if face == 3:
        return np.stack([m1, u, v], axis=1)
    raise ValueError(face)


@lru_cache(maxsize=None)
def _operators_quadrature_cached(p: int):
    rst = nodes(p)
    Np = n_nodes(p)
    Nfp = n_face_nodes(p)
    Dr = lagrange_at(p, rst, (1, 0, 0))
    Ds = lagrange_at(p, rst, (0, 1, 0))
    Dt = lagrange_at(p, rst, (0, 0, 1))
    qx, qw = tet_quadrature(p + 3)
    Lq = lagrange_at(p, qx)
    M = Lq.T @ (qw[:, None] * Lq)
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    on_face = [np.abs(1 + t) < TOL, np.abs(1 + s) < TOL, np.abs(1 + r + s + t) < TOL, np.abs(1 + r) < TOL]
    Fmask = np.stack([np.nonzero(f)[0] for f in on_face])
    assert Fmask.shape == (4, Nfp)
    fx, fw = tri_quadrature(p + 3)
    E = np.zeros((Np, 4 * Nfp))
    for f in range(4):
        Lf = lagrange_at(p, face_point_to_rst(f, fx))
        Mf_full = Lf.T @ (fw[:, None] * Lf)  # int_face l_i l_j over all volume nodes
        E[:, f * Nfp:(f + 1) * Nfp] = Mf_full[:, Fmask[f]]
    LIFT = np.linalg.solve(M, E)
    return dict(p=p, Np=Np, Nfp=Nfp, rst=rst, Dr=Dr, Ds=Ds, Dt=Dt, M=M, E=E, LIFT=LIFT, Fmask=Fmask)


def _solve_exact(A, B):
    """X with A X = B, by Gauss-Jordan elimination over the rationals."""
    n = len(A)
    M = [list(A[i]) + list(B[i]) for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [x * inv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


def _face_monomial_integral(f: int, a: int, b: int, c: int) -> Fraction:
    """int over face f of x^a y^b z^c, with (x, y, z) = ((1+r)/2, (1+s)/2,
    (1+t)/2) and the face's parametric measure (two reference coordinates,
    area 2 = 4 x the unit triangle's 1/2).  On f0 z = 0, on f1 y = 0, on f3
    x = 0; on f2 x = 1 - y - z (Dirichlet integral with the third barycentric)."""
    F = math.factorial
    if f == 0:
        return Fraction(4 * F(a) * F(b), F(a + b + 2)) if c == 0 else Fraction(0)
    if f == 1:
        return Fraction(4 * F(a) * F(c), F(a + c + 2)) if b == 0 else Fraction(0)
    if f == 3:
        return Fraction(4 * F(b) * F(c), F(b + c + 2)) if a == 0 else Fraction(0)
    return Fraction(4 * F(a) * F(b) * F(c), F(a + b + c + 2))


@lru_cache(maxsize=None)
def _operators_cached(p: int):
    """Exact operators at the FP64 nodes, rounded once (see the module notes).
    Monomials x^a y^b z^c (a + b + c <= p) in the unit-simplex coordinates
    x = (1+r)/2, y = (1+s)/2, z = (1+t)/2 span the degree-p polynomials;
    V[i, k] = phi_k(x_i), so the Lagrange basis is l = phi V^{-1} and
      Dr = V_r V^{-1} (d/dr = d/dx / 2), M = V^{-T} Phi V^{-1},
      E[:, (f, m)] = (V^{-T} Phi_f V^{-1})[:, Fmask[f][m]], LIFT = M^{-1} E,
    with Phi, Phi_f the element and face integrals of monomial products
    (element: 8 a! b! c! / (a+b+c+3)!)."""
    rst = nodes(p)
    Np = n_nodes(p)
    Nfp = n_face_nodes(p)
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    on_face = [np.abs(1 + t) < TOL, np.abs(1 + s) < TOL, np.abs(1 + r + s + t) < TOL, np.abs(1 + r) < TOL]
    Fmask = np.stack([np.nonzero(f)[0] for f in on_face])
    assert Fmask.shape == (4, Nfp)
    mk = _multi_indices(p)
    X = [[(Fraction(float(v)) + 1) / 2 for v in row] for row in rst]
    V = [[x[0] ** a * x[1] ** b * x[2] ** c for (a, b, c) in mk] for x in X]
    I = [[Fraction(int(i == j)) for j in range(Np)] for i in range(Np)]
    Vinv = _solve_exact(V, I)

    def deriv_row(x, d):
        row = []
        for e in mk:
            if e[d] == 0:
                row.append(Fraction(0))
                continue
            e2 = list(e)
            e2[d] -= 1
            row.append(Fraction(e[d], 2) * x[0] ** e2[0] * x[1] ** e2[1] * x[2] ** e2[2])
        return row

    def matmul(A, B):
        Bt = list(zip(*B))
        return [[sum(a * b for a, b in zip(row, col)) for col in Bt] for row in A]

    def to_np(A):
        return np.array([[float(v) for v in row] for row in A])

    out = dict(p=p, Np=Np, Nfp=Nfp, rst=rst, Fmask=Fmask)
    for name, d in (("Dr", 0), ("Ds", 1), ("Dt", 2)):
        out[name] = to_np(matmul([deriv_row(x, d) for x in X], Vinv))
    F = math.factorial
    Phi = [[Fraction(8 * F(a1 + a2) * F(b1 + b2) * F(c1 + c2), F(a1 + a2 + b1 + b2 + c1 + c2 + 3))
            for (a2, b2, c2) in mk] for (a1, b1, c1) in mk]
    VinvT = [list(col) for col in zip(*Vinv)]
    M = matmul(matmul(VinvT, Phi), Vinv)
    # M^{-1} = V Phi^{-1} V^T, so LIFT[:, f] = V Phi^{-1} Phi_f V^{-1}[:, Fmask[f]]
    E = [[Fraction(0)] * (4 * Nfp) for _ in range(Np)]
    LIFT = [[Fraction(0)] * (4 * Nfp) for _ in range(Np)]
    for f in range(4):
        Phf = [[_face_monomial_integral(f, e1[0] + e2[0], e1[1] + e2[1], e1[2] + e2[2]) for e2 in mk] for e1 in mk]
        PV = matmul(Phf, [[Vinv[k][j] for j in Fmask[f]] for k in range(Np)])
        Ef = matmul(VinvT, PV)
        Lf = matmul(V, _solve_exact(Phi, PV))
        for i in range(Np):
            for m in range(Nfp):
                E[i][f * Nfp + m] = Ef[i][m]
                LIFT[i][f * Nfp + m] = Lf[i][m]
    out.update(M=to_np(M), E=to_np(E), LIFT=to_np(LIFT))
    return out


def operators(p: int) -> dict:
    """Reference operators for order p: rst, Dr, Ds, Dt, M, E, LIFT, Fmask
    (exact at the FP64 nodes, rounded once)."""
    ops = _operators_cached(p)
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ops.items()}


def operators_by_quadrature(p: int) -> dict:
    """The same operators through an FP64 Legendre tensor basis and collapsed
    Gauss quadrature: an independent route, accurate to its own rounding."""
    ops = _operators_quadrature_cached(p)
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ops.items()}
