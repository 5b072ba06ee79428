"""Affine geometry and face connectivity of a tetrahedral mesh (oracle, FP64).

Test infrastructure only (see the package docstring).

Readings (nodal DG on affine simplices, Hesthaven & Warburton; the paper only
names the per-element layout, Sec. 1):

* x(r,s,t) = -(1+r+s+t)/2 X1 + (1+r)/2 X2 + (1+s)/2 X3 + (1+t)/2 X4, so
  x_r = (X2-X1)/2, x_s = (X3-X1)/2, x_t = (X4-X1)/2, J = det[x_r x_s x_t] > 0
  and the metric terms (dr/dx, ...) are the inverse Jacobian matrix.
* Face normals and areas come from the physical face triangle: outward unit
  normal n_f, area A_f, surface Jacobian sJ_f = A_f / 2 (the reference face
  has parametric area 2) and Fscale_f = sJ_f / J.
* Faces match on the sorted triple of global vertex ids (periodic images share
  ids); node m of face (K, f) pairs with the node of the matching face that has
  the same barycentric coordinates with respect to the same global vertices.
"""
from __future__ import annotations

import numpy as np

from .reference_element import FACE_VERTS, barycentric, operators


def node_coordinates(elem_xyz: np.ndarray, rst: np.ndarray) -> np.ndarray:
    """Physical node coordinates [E, Np, 3] of the affine elements."""
    lam = barycentric(rst)  # [Np, 4]
    return np.einsum("na,ead->end", lam, elem_xyz)


def geometry(elem_xyz: np.ndarray) -> dict:
    """Per-element metric terms, Jacobian, face normals, areas and Fscale."""
    X1, X2, X3, X4 = (elem_xyz[:, a, :] for a in range(4))
    jac = np.stack([(X2 - X1) / 2, (X3 - X1) / 2, (X4 - X1) / 2], axis=2)  # [E, x, (r,s,t)]
    J = np.linalg.det(jac)
    if np.any(J <= 0):
        raise ValueError("non-positive element Jacobian")
    inv = np.linalg.inv(jac)  # [E, (r,s,t), x]: inv[:, 0, :] = grad r
    normals = np.zeros((elem_xyz.shape[0], 4, 3))
    area = np.zeros((elem_xyz.shape[0], 4))
    centroid = elem_xyz.mean(axis=1)
    for f, (a, b, c) in enumerate(FACE_VERTS):
        A, B, C = elem_xyz[:, a], elem_xyz[:, b], elem_xyz[:, c]
        cr = np.cross(B - A, C - A)
        nrm = np.linalg.norm(cr, axis=1)
        n = cr / nrm[:, None]
        # orient outward: away from the element centroid
        sgn = np.sign(np.einsum("ed,ed->e", n, (A + B + C) / 3.0 - centroid))
        normals[:, f] = n * sgn[:, None]
        area[:, f] = 0.5 * nrm
    sJ = area / 2.0
    return dict(J=J, rst_x=inv, normals=normals, area=area, sJ=sJ, Fscale=sJ / J[:, None])


def connectivity(elem_vid: np.ndarray, p: int) -> dict:
    """Face-node map: for each (K, f, m) the neighbour element and node index.

    Returns dict with
      nbr_elem  int64 [E, 4]          neighbour element across face f
      nbr_face  int64 [E, 4]          its local face
      mapP_elem int64 [E, 4 * Nfp]    neighbour element of each face node
      mapP_node int64 [E, 4 * Nfp]    neighbour volume-node index
    Raises ValueError if a face does not occur exactly twice.
    """
    ops = operators(p)
    Nfp = ops["Nfp"]
    Fmask = ops["Fmask"]
    lam = barycentric(ops["rst"])  # [Np, 4]
    E = elem_vid.shape[0]
    fv = np.array(FACE_VERTS)  # [4, 3]
    face_gids = elem_vid[:, fv]  # [E, 4, 3]
    keys = np.sort(face_gids, axis=2).reshape(-1, 3)
    _, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    if np.any(counts != 2):
        raise ValueError("every face of a periodic mesh must be shared by exactly two elements")
    order = np.argsort(inv, kind="stable")
    first, second = order[0::2], order[1::2]
    partner = np.empty(E * 4, dtype=np.int64)
    partner[first] = second
    partner[second] = first
    nbr_elem = (partner // 4).reshape(E, 4)
    nbr_face = (partner % 4).reshape(E, 4)

    # canonical key of every face node: barycentric weights of the face's three
    # vertices listed in ascending global-vertex-id order
    face_keys = np.zeros((E, 4, Nfp, 3))
    for f in range(4):
        lam_f = lam[Fmask[f]][:, fv[f]]  # [Nfp, 3]
        gid = face_gids[:, f, :]  # [E, 3]
        srt = np.argsort(gid, axis=1)  # [E, 3]
        face_keys[:, f] = np.take_along_axis(lam_f[None, :, :], srt[:, None, :], axis=2)
    flat = face_keys.reshape(E * 4, Nfp, 3)
    # the three weights sum to one, so the first two order the nodes; distinct
    # face nodes differ by far more than 1e-3 in one of them
    sort_idx = np.argsort(flat[:, :, 0] * 1e3 + flat[:, :, 1], axis=1, kind="stable")
    sorted_keys = np.take_along_axis(flat, sort_idx[:, :, None], axis=1)
    if np.any(np.abs(sorted_keys[partner] - sorted_keys) > 1e-10):
        raise ValueError("face nodes of matched faces do not coincide")
    # node at sorted position k of face (K,f) pairs with sorted position k of partner
    rank = np.empty_like(sort_idx)
    np.put_along_axis(rank, sort_idx, np.arange(Nfp)[None, :].repeat(E * 4, 0), axis=1)
    partner_local = np.take_along_axis(sort_idx[partner], rank, axis=1)  # [E*4, Nfp] local face-node index
    pf = (partner % 4)
    mapP_node = Fmask[pf[:, None], partner_local]  # volume node index in neighbour
    mapP_elem = np.repeat((partner // 4)[:, None], Nfp, axis=1)
    return dict(nbr_elem=nbr_elem, nbr_face=nbr_face,
                mapP_elem=mapP_elem.reshape(E, 4 * Nfp), mapP_node=mapP_node.reshape(E, 4 * Nfp))
