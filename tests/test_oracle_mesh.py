"""Pins of the oracle's geometry and connectivity: exact total volume of the
periodic box, closed surfaces, matched faces with equal area and opposite
normals, an involutive face-node map whose nodes coincide modulo the period."""
import numpy as np
import pytest

from oracle import mesh as om, reference_element as re
from paper_2512_17101_amd import workload as wl


@pytest.fixture(scope="module", params=[2, 3])
def setup(request):
    p = request.param
    xyz, vid = wl.kuhn_box_mesh(4, 10.0, 0.05, 1001)
    return p, xyz, vid, om.geometry(xyz), om.connectivity(vid, p)


def test_volume_and_closed_surface(setup):
    p, xyz, vid, geo, conn = setup
    assert abs(np.sum(4.0 / 3.0 * geo["J"]) - 1000.0) < 1e-10
    closure = np.einsum("ef,efd->ed", geo["area"], geo["normals"])
    assert np.abs(closure).max() < 1e-13
    # J equals 3/4 of the physical volume from the scalar triple product
    v = np.einsum("ed,ed->e", xyz[:, 1] - xyz[:, 0], np.cross(xyz[:, 2] - xyz[:, 0], xyz[:, 3] - xyz[:, 0])) / 6
    np.testing.assert_allclose(geo["J"], 0.75 * v, rtol=1e-13)


def test_metric_is_inverse_jacobian(setup):
    p, xyz, vid, geo, conn = setup
    ops = re.operators(p)
    X = om.node_coordinates(xyz, ops["rst"])
    # d x / d r from the nodal derivative of the coordinates, times (dr/dx) = I
    for e in (0, 17, 200):
        xr = np.stack([ops["Dr"] @ X[e, :, d] for d in range(3)])[:, 0]
        xs = np.stack([ops["Ds"] @ X[e, :, d] for d in range(3)])[:, 0]
        xt = np.stack([ops["Dt"] @ X[e, :, d] for d in range(3)])[:, 0]
        jac = np.stack([xr, xs, xt], axis=1)
        np.testing.assert_allclose(geo["rst_x"][e] @ jac, np.eye(3), atol=1e-12)


def test_matched_faces(setup):
    p, xyz, vid, geo, conn = setup
    nb, nf = conn["nbr_elem"], conn["nbr_face"]
    E = xyz.shape[0]
    e = np.arange(E)[:, None].repeat(4, 1)
    f = np.arange(4)[None, :].repeat(E, 0)
    assert np.all(nb[nb, nf] == e) and np.all(nf[nb, nf] == f)
    np.testing.assert_allclose(geo["area"][nb, nf], geo["area"], rtol=1e-12)
    np.testing.assert_allclose(geo["normals"][nb, nf], -geo["normals"], atol=1e-12)


def test_face_node_map(setup):
    p, xyz, vid, geo, conn = setup
    ops = re.operators(p)
    X = om.node_coordinates(xyz, ops["rst"])
    XM = X[:, ops["Fmask"].reshape(-1)]
    XP = X[conn["mapP_elem"], conn["mapP_node"]]
    d = XP - XM
    d -= 10.0 * np.round(d / 10.0)
    assert np.abs(d).max() < 1e-12
    # bijection: following the map twice returns to the start
    Nfp = ops["Nfp"]
    fmask = ops["Fmask"]
    back_elem = np.zeros_like(conn["mapP_elem"])
    for fm in range(4 * Nfp):
        f = fm // Nfp
        eP = conn["mapP_elem"][:, fm]
        fP = conn["nbr_face"][:, f]
        nodeP = conn["mapP_node"][:, fm]
        mP = np.array([np.nonzero(fmask[fP[i]] == nodeP[i])[0][0] for i in range(len(eP))])
        back_elem[:, fm] = conn["mapP_elem"][eP, fP * Nfp + mP]
        assert np.all(conn["mapP_node"][eP, fP * Nfp + mP] == fmask[f][fm % Nfp])
    assert np.all(back_elem == np.arange(xyz.shape[0])[:, None])


def test_inverted_element_rejected():
    xyz, vid = wl.kuhn_box_mesh(3, 10.0, 0.0, 0)
    xyz = xyz.copy()
    xyz[5, [2, 3]] = xyz[5, [3, 2]]
    with pytest.raises(ValueError):
        om.geometry(xyz)
