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
* Computed here through a Legendre *tensor* basis P_a(r) P_b(s) P_c(t),
  a + b + c <= p (a basis of the degree-p polynomials), and collapsed-coordinate
  Gauss-Legendre quadrature exact for the integrands.  Any exact route gives the
  same matrices.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg

TOL = 1e-10

# Warp & blend alpha per order (Warburton 2006 optimised values as tabulated in
# Hesthaven & Warburton, Sec. 10.1); orders 1..3 use alpha = 0.
_ALPHA = {1: 0.0, 2: 0.0, 3: 0.0, 4: 0.1002}

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


def _warp_over_bubble(p: int, x: np.ndarray) -> np.ndarray:
    """w(x) / (1 - x^2), where w is the degree-p interpolant on equidistant
    points of the displacement (LGL point - equidistant point).  The endpoint
    displacements are zero, so the quotient is a polynomial; it is formed by
    dropping the (x - 1)(x + 1) factor from each interior Lagrange polynomial."""
    xeq = np.linspace(-1.0, 1.0, p + 1)
    disp = lgl_points(p) - xeq
    out = np.zeros_like(x)
    for i in range(1, p):
        num = np.ones_like(x)
        den = 1.0
        for j in range(p + 1):
            if j == i:
                continue
            den *= xeq[i] - xeq[j]
            if j not in (0, p):
                num = num * (x - xeq[j])
        # l_i(x) = num * (x + 1)(x - 1) / den  and  (x + 1)(x - 1) = -(1 - x^2)
        out = out - disp[i] * num / den
    return out


def _face_shift(p: int, alpha: float, L: np.ndarray, verts: np.ndarray) -> np.ndarray:
    """In-face displacement for points with face barycentrics L[:, 0..2] of the
    face vertices verts[0..2] (equilateral coordinates): a sum over the three
    edges of the blended 1-D edge warp along the edge direction."""
    shift = np.zeros((L.shape[0], 3))
    for k in range(3):
        a, b = (k + 1) % 3, (k + 2) % 3  # edge k joins vertices a -> b, opposite vertex k
        x = L[:, b] - L[:, a]
        warp = 4.0 * _warp_over_bubble(p, x) * L[:, a] * L[:, b] * (1.0 + (alpha * L[:, k]) ** 2)
        d = verts[b] - verts[a]
        shift += warp[:, None] * (d / np.linalg.norm(d))[None, :]
    return shift


@lru_cache(maxsize=None)
def _nodes_cached(p: int) -> np.ndarray:
    if p < 1 or p > 4:
        raise ValueError("orders 1..4 are supported")
    alpha = _ALPHA[p]
    rst_eq = equidistant_lattice(p)
    lam = barycentric(rst_eq)
    X = lam @ _VEQ
    shift = np.zeros_like(X)
    override = np.zeros(len(X), dtype=bool)
    override_val = np.zeros_like(X)
    for opp in range(4):  # face opposite vertex `opp`
        fv = [v for v in range(4) if v != opp]
        La = lam[:, opp]
        Lf = lam[:, fv]
        s_face = _face_shift(p, alpha, Lf, _VEQ[fv])
        blend = Lf[:, 0] * Lf[:, 1] * Lf[:, 2]
        denom = (Lf[:, 0] + 0.5 * La) * (Lf[:, 1] + 0.5 * La) * (Lf[:, 2] + 0.5 * La)
        ok = denom > TOL
        b = np.where(ok, (1.0 + (alpha * La) ** 2) * blend / np.where(ok, denom, 1.0), blend)
        shift += b[:, None] * s_face
        on_edge = (La < TOL) & ((Lf > TOL).sum(axis=1) < 3)
        override |= on_edge
        override_val[on_edge] = s_face[on_edge]
    shift[override] = override_val[override]
    X = X + shift
    # equilateral -> reference coordinates: X - V1 = sum_d (1 + rst_d)/2 (V_{d+1} - V1)
    A = 0.5 * np.stack([_VEQ[1] - _VEQ[0], _VEQ[2] - _VEQ[0], _VEQ[3] - _VEQ[0]], axis=1)
    rst = np.linalg.solve(A, (X - _VEQ[0]).T).T - 1.0
    return rst


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
def _operators_cached(p: int):
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


def operators(p: int) -> dict:
    """Reference operators for order p: rst, Dr, Ds, Dt, M, E, LIFT, Fmask."""
    ops = _operators_cached(p)
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ops.items()}
