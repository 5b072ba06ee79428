"""Pins of the oracle's shock capturing on hexahedra (the paper's Sec. 5.3
names artificial viscosity and limiting): the modal indicator's
normalisation and limits, the viscosity ramp, the BR1 artificial-viscosity
term against its unfactored definition, its conservation and dissipation,
and the positivity limiter's invariants."""
import math

import numpy as np
import pytest

from oracle import euler as oe, hex as oh, lsrk, shock as osh
from paper_2512_17101_amd import workload as wl

U = 2.0 ** -53


def _setup(p, dims=(3, 4, 2), jitter=0.1, seed=11):
    gr = oh.grid(*wl.rectilinear_grid(dims, (10.0, 10.0 * dims[1] / dims[0], 10.0 * dims[2] / dims[0]), jitter, seed))
    return oh.operators_1d(p), gr, oh.node_coordinates(gr, p)


def _J(gr):
    hz, hy, hx = np.meshgrid(gr["h"][2], gr["h"][1], gr["h"][0], indexing="ij")
    return (hx * hy * hz / 8.0).ravel()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_modal_energy_is_the_l2_norm(p):
    """Orthonormal modes: sum c^2 = rho^T (M1 x M1 x M1) rho on the
    reference cube (Parseval), which pins the basis normalisation."""
    Vi = osh._modal_inverse(p)
    o = oh.operators_1d(p)
    rng = np.random.default_rng(p)
    rho = rng.standard_normal((p + 1) ** 3)
    c = np.kron(Vi, np.kron(Vi, Vi)) @ rho
    M3 = np.kron(o["M"], np.kron(o["M"], o["M"]))
    assert abs(c @ c - rho @ M3 @ rho) <= 1e-12 * (c @ c)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_indicator_limits(p):
    """A density of degree < p in every direction has no top-mode energy
    (s below -20); a pure top mode has all of it (s = 0)."""
    gr = oh.grid(*wl.rectilinear_box(2, 10.0, 0.0, 0))
    X = oh.node_coordinates(gr, p)
    q = wl.entropy_wave_state(X, lambda x: 2.0 + (x[..., 0] / 10) ** (p - 1) * (x[..., 1] / 10) ** (p - 1))
    assert np.all(osh.smoothness(gr, q, p) < -20)
    x = oh.gll_points(p)
    c = np.zeros(p + 1)
    c[p] = 1.0
    top = np.polynomial.legendre.legval(x, c)
    rho = np.tile(np.kron(np.ones(p + 1), np.kron(np.ones(p + 1), top)), (8, 1))  # P_p(r) in every element
    q = np.stack([rho, 0 * rho, 0 * rho, 0 * rho, rho + 10])
    np.testing.assert_allclose(osh.smoothness(gr, q, p), 0.0, atol=1e-14)


def test_viscosity_ramp():
    gr = oh.grid(*wl.rectilinear_box(2, 10.0, 0.0, 0))
    p = 2
    X = oh.node_coordinates(gr, p)
    q = wl.shock_slab_state(X, x0=2.0, x1=7.0, ripple=0.0)
    prm = osh.default_params(p)
    s = osh.smoothness(gr, q, p)
    for s0 in (s.max() + 1.5, s.max() - 1.5, s.max()):
        eps = osh.viscosity(gr, q, p, dict(prm, s0=s0))
        e_full = osh.viscosity(gr, q, p, dict(prm, s0=-1e9))
        m = np.argmax(s)
        if s0 > s.max() + 1:
            assert eps[m] == 0.0
        elif s0 < s.max() - 1:
            assert eps[m] == e_full[m]
        else:
            assert abs(eps[m] - 0.5 * e_full[m]) <= 1e-15 * e_full[m]


def _unfactored_av(p, gr, q, eps):
    F = oh.full_operators(p)
    P = p + 1
    nx, ny, nz = gr["dims"]
    idx = np.arange(P ** 3).reshape(P, P, P)
    E = q.shape[1]
    Ds = (F["Dr"], F["Ds"], F["Dt"])

    def lifted(U, e, i, j, k, d):
        """(2/h_d) (D_d U + LIFT3 over the two faces of direction d of n_d (U+ - U-)/2)."""
        h = (gr["h"][0][i], gr["h"][1][j], gr["h"][2][k])
        out = U[:, e] @ Ds[d].T
        for side in (0, 1):
            f = 2 * d + side
            ijk = [i, j, k]
            ijk[d] = (ijk[d] + (1 if side else -1)) % (nx, ny, nz)[d]
            en = ijk[0] + nx * (ijk[1] + ny * ijk[2])
            own = np.take(idx, 0 if side == 0 else P - 1, axis=2 - d).ravel()
            nbr = np.take(idx, P - 1 if side == 0 else 0, axis=2 - d).ravel()
            nd = 1.0 if side else -1.0
            jump = 0.5 * nd * (U[:, en][:, nbr] - U[:, e][:, own])
            out = out + jump @ F["LIFT3"][:, f * P * P:(f + 1) * P * P].T
        return (2.0 / h[d]) * out

    cells = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    G = np.zeros((3,) + q.shape)
    for e, (i, j, k) in enumerate(cells):
        for d in range(3):
            G[d][:, e] = eps[e] * lifted(q, e, i, j, k, d)
    out = np.zeros_like(q)
    for e, (i, j, k) in enumerate(cells):
        out[:, e] = sum(lifted(G[d], e, i, j, k, d) for d in range(3))
    return out


@pytest.mark.parametrize("p", [1, 2, 3])
def test_av_equals_unfactored_definition(p):
    ops, gr, X = _setup(p, dims=(3, 2, 2))
    q = wl.vortex_state(X, pert=wl.density_perturbation(3))
    q = q * (1.0 + 1e-2 * np.random.default_rng(1).standard_normal(q.shape))
    eps = np.random.default_rng(2).uniform(0.0, 0.1, q.shape[1])
    r = osh.av_rhs(ops, gr, q, eps)
    ref = _unfactored_av(p, gr, q, eps)
    assert np.abs(r - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_av_conservative_and_dissipative(p):
    """Central fluxes: sum J 1^T M av = 0 per field; and the BR1 form with a
    per-element viscosity is dissipative: q^T (J M) av(q) = -sum_e eps_e
    sigma_e^T (J M) sigma_e <= 0 per field."""
    ops, gr, X = _setup(p)
    q = wl.shock_slab_state(X, x0=3.1, x1=6.7)
    q = q * (1.0 + 1e-2 * np.random.default_rng(5).standard_normal(q.shape))
    eps = np.random.default_rng(6).uniform(0.0, 0.05, q.shape[1])
    r = osh.av_rhs(ops, gr, q, eps)
    M3 = np.kron(ops["M"], np.kron(ops["M"], ops["M"]))
    J = _J(gr)
    w = J[None, :, None] * (r @ M3.T)
    assert np.all(np.abs(w.sum(axis=(1, 2))) <= 1e-12 * np.abs(w).sum(axis=(1, 2)))
    energy = np.einsum("fei,fei->f", q, w)
    G = osh.av_fluxes(ops, gr, q, eps)
    sig_energy = sum(np.einsum("fei,fei->f", G[d] / np.where(eps > 0, eps, 1)[None, :, None],
                               J[None, :, None] * (G[d] @ M3.T)) for d in range(3))
    assert np.all(energy <= 0)
    np.testing.assert_allclose(energy, -sig_energy, rtol=1e-10)


def test_av_zero_for_constant_state_and_limits_to_laplacian():
    """A constant state has no viscous term; for constant eps and
    q = sin(2 pi x / L) the term approaches -eps (2 pi / L)^2 q as the grid
    is refined (order >= p)."""
    p = 3
    ops, gr, X = _setup(p)
    q = wl.constant_state(X.shape[:2])
    assert np.abs(osh.av_rhs(ops, gr, q, np.full(q.shape[1], 0.3))).max() <= 1e-13 * np.abs(q).max()
    errs = []
    for n in (4, 8):
        gr = oh.grid(*wl.rectilinear_grid((n, 2, 2), (10.0, 10.0, 10.0), 0.1, 4))
        X = oh.node_coordinates(gr, p)
        f = np.sin(2 * np.pi * X[..., 0] / 10.0)
        q = np.stack([2 + f, f, f, f, 10 + f])
        r = osh.av_rhs(ops, gr, q, np.full(q.shape[1], 0.1))
        exact = -0.1 * (2 * np.pi / 10.0) ** 2 * f
        errs.append(np.abs(r[1] - exact).max())
    assert math.log2(errs[0] / errs[1]) >= p - 0.5


def test_limiter_invariants():
    p = 2
    ops, gr, X = _setup(p, dims=(4, 3, 2))
    rng = np.random.default_rng(9)
    q = wl.shock_slab_state(X, x0=3.3, x1=6.1)
    # push some nodes below zero density / pressure, keeping averages admissible
    q[0] += rng.uniform(-3.0, 0.5, q[0].shape) * (q[0] < 2)
    q[4] += rng.uniform(-1.0, 0.1, q[4].shape)
    ql = osh.limit(q, p)
    w = osh.cell_weights(p)
    np.testing.assert_allclose(ql @ w, q @ w, rtol=1e-13, atol=1e-13)  # averages kept
    qbar = (q @ w) / w.sum()
    pbar = 0.4 * (qbar[4] - 0.5 * (qbar[1] ** 2 + qbar[2] ** 2 + qbar[3] ** 2) / qbar[0])
    ok = (qbar[0] > osh.DELTA) & (pbar > osh.DELTA)
    assert ok.sum() > 0 and (~ok).sum() >= 0
    pn = 0.4 * (ql[4] - 0.5 * (ql[1] ** 2 + ql[2] ** 2 + ql[3] ** 2) / ql[0])
    # the bound holds to the rounding of qbar + theta (q - qbar): a few u of
    # the average (delta is far below it)
    assert np.all(ql[0][ok] >= osh.DELTA - 8 * U * qbar[0][ok, None])
    assert np.all(pn[ok] >= osh.DELTA - 64 * U * np.abs(qbar[4][ok, None]))
    # admissible elements are left alone (bitwise)
    fine = ok & (q[0].min(axis=1) >= osh.DELTA) & (
        (0.4 * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0])).min(axis=1) >= osh.DELTA)
    assert np.array_equal(ql[:, fine], q[:, fine])
    assert np.array_equal(ql[:, ~ok], q[:, ~ok])


def test_limiter_hand_example():
    """One p = 1 element at rest, density 1 at seven nodes and -0.5 at one:
    the average is (7 - 0.5) / 8 = 0.8125 (equal weights at p = 1), so
    theta = (0.8125 - delta) / (0.8125 + 0.5) and the bad node becomes delta."""
    p = 1
    rho = np.ones(8)
    rho[3] = -0.5
    q = np.stack([rho, 0 * rho, 0 * rho, 0 * rho, np.full(8, 2.0)])[:, None, :]
    ql = osh.limit(q, p)
    assert abs(ql[0, 0, 3] - osh.DELTA) <= 1e-15
    th = (0.8125 - osh.DELTA) / (0.8125 + 0.5)
    np.testing.assert_allclose(ql[0, 0, 0], 0.8125 + th * (1 - 0.8125), rtol=1e-15)


def test_shock_steps_stay_admissible_and_conservative():
    """Twenty LSRK(5,4) steps of the slab at p = 2 with artificial viscosity
    and the limiter on every stage: finite, positive density and pressure,
    mass and energy conserved to 1e-12."""
    p = 2
    ops, gr, X = _setup(p, dims=(8, 2, 2))
    q = wl.shock_slab_state(X, x0=3.3, x1=6.1, ripple=0.0)
    M3 = np.kron(ops["M"], np.kron(ops["M"], ops["M"]))
    J = _J(gr)
    tot0 = (J[None, :, None] * (q @ M3.T)).sum(axis=(1, 2))
    dt = oh.cfl_dt(gr, q, p, 0.1)
    f = lambda qq, tt: osh.shock_rhs(ops, gr, qq)
    for s in range(20):
        q, _ = lsrk.lsrk_step(f, q, s * dt, dt, stage_filter=lambda qq: osh.limit(qq, p))
    assert np.all(np.isfinite(q))
    pn = 0.4 * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0])
    assert q[0].min() > 0 and pn.min() > 0
    tot = (J[None, :, None] * (q @ M3.T)).sum(axis=(1, 2))
    assert abs(tot[0] - tot0[0]) <= 1e-12 * abs(tot0[0]) and abs(tot[4] - tot0[4]) <= 1e-12 * abs(tot0[4])
