"""Pins of the oracle's thermochemistry: temperature round trips through
e(T; Y), the constant-cp closed form, residual and uniqueness conditions,
forced non-convergence, the Arrhenius law's log-linear form, mass
conservation of the sources and vanishing rates without a reactant."""
import numpy as np
import pytest

from oracle import thermo as ot
from paper_2512_17101_amd import workload as wl

TH = wl.synthetic_thermo(3003)
MECH = wl.synthetic_mechanism(3004)


def _random_Y(n, rng):
    return rng.dirichlet(np.ones(7), size=n).T


def test_round_trip_recovers_temperature():
    rng = np.random.default_rng(0)
    T_true = rng.uniform(300.0, 3000.0, 5000)
    Y = _random_Y(5000, rng)
    e = ot.mixture_e(T_true, Y, TH)
    T, it = ot.newton_temperature(e, Y, TH, 1000.0)
    assert np.all(it >= 1)
    assert np.abs(T - T_true).max() < 1e-9


def test_residual_and_cv_positive():
    rng = np.random.default_rng(1)
    Y = _random_Y(2000, rng)
    e = ot.mixture_e(rng.uniform(400, 2500, 2000), Y, TH)
    T, it = ot.newton_temperature(e, Y, TH, 1000.0, tol=1e-10)
    cv = ot.mixture_cv(T, Y, TH)
    assert np.all(np.abs(ot.mixture_e(T, Y, TH) - e) <= cv * 1e-10)
    Tg = np.linspace(100.0, 6000.0, 200)
    for k in range(7):
        Yk = np.zeros((7, 200))
        Yk[k] = 1.0
        assert np.all(ot.mixture_cv(Tg, Yk, TH) > 0)


def test_constant_cp_closed_form():
    th = {"W": TH["W"].copy(), "a": TH["a"].copy()}
    th["a"][0, 1:5] = 0.0  # species 1 with constant cp/R = a1
    Y = np.zeros((7, 3))
    Y[0] = 1.0
    Rk = ot.R_U / th["W"][0]
    a1, a6 = th["a"][0, 0], th["a"][0, 5]
    T_exact = np.array([350.0, 1200.0, 2900.0])
    e = Rk * ((a1 - 1.0) * T_exact + a6)  # e = h - R T, linear in T
    T, it = ot.newton_temperature(e, Y, th, 1000.0)
    np.testing.assert_allclose(T, T_exact, rtol=0, atol=1e-9)
    assert np.all(it <= 2)  # one exact step, one step that confirms it


def test_forced_non_convergence_and_clamp():
    rng = np.random.default_rng(2)
    Y = _random_Y(100, rng)
    e = ot.mixture_e(rng.uniform(500, 2500, 100), Y, TH)
    _, it = ot.newton_temperature(e, Y, TH, 1000.0, max_iter=1)
    assert np.all(it == -1)
    # roots beyond either end of the clamp interval: the iterate sits at the
    # bound, and that is a failure (-1), not a converged temperature
    e_hot = ot.mixture_e(np.full(100, 9000.0), Y, TH)
    T, it = ot.newton_temperature(e_hot, Y, TH, 1000.0)
    assert np.all(T == ot.T_MAX) and np.all(it == -1)
    e_cold = ot.mixture_e(np.full(100, 40.0), Y, TH)
    T, it = ot.newton_temperature(e_cold, Y, TH, 1000.0)
    assert np.all(T == ot.T_MIN) and np.all(it == -1)
    # a root just inside the bound still converges
    e_in = ot.mixture_e(np.full(100, 5990.0), Y, TH)
    T, it = ot.newton_temperature(e_in, Y, TH, 1000.0)
    assert np.all(it >= 1)
    np.testing.assert_allclose(T, 5990.0, rtol=0, atol=1e-8)


def test_non_finite_state_fails():
    Y = _random_Y(4, np.random.default_rng(5))
    e = np.array([np.nan, np.inf, 1e6, 1e6])
    Y[:, 3] = np.nan
    T, it = ot.newton_temperature(e, Y, TH, 1000.0)
    assert np.all(it[[0, 1, 3]] == -1) and it[2] >= 1
    assert np.all(~np.isfinite(T[[0, 3]]))


def test_arrhenius_log_linear():
    T = np.array([500.0, 1000.0, 2000.0])
    k = ot.rate_constants(T, MECH)
    slope = (np.log(k[:, 2]) - np.log(k[:, 0])) / (1 / T[2] - 1 / T[0])
    np.testing.assert_allclose(slope, -MECH["Ea"] / ot.R_U, rtol=1e-10)
    np.testing.assert_allclose(ot.rate_constants(np.array([1e300]), MECH)[:, 0], MECH["A"], rtol=1e-12)


def test_sources_conserve_mass_and_vanish_without_reactant():
    rng = np.random.default_rng(3)
    n = 4000
    rho = rng.uniform(0.1, 2.0, n)
    T = rng.uniform(300, 2500, n)
    Y = _random_Y(n, rng)
    w = ot.sources(rho, T, Y, TH, MECH)
    assert np.all(np.abs(w.sum(axis=0)) <= 1e-14 * np.abs(w).sum(axis=0))
    # no species 1: reaction 1 must not run
    Y0 = Y.copy()
    Y0[0] = 0.0
    m0 = {k: v.copy() for k, v in MECH.items()}
    m0["A"][0] = 0.0
    np.testing.assert_allclose(ot.sources(rho, T, Y0, TH, MECH), ot.sources(rho, T, Y0, TH, m0), rtol=0, atol=0)
    # only reaction 2 active: omega is W_k (nu'' - nu')_k k_2 C_3 C_2
    m2 = {k: v.copy() for k, v in MECH.items()}
    m2["A"][[0, 2]] = 0.0
    C = rho * Y / TH["W"][:, None]
    r2 = MECH["A"][1] * np.exp(-MECH["Ea"][1] / (ot.R_U * T)) * C[2] * C[1]
    w2 = ot.sources(rho, T, Y, TH, m2)
    np.testing.assert_allclose(w2[4], TH["W"][4] * r2, rtol=1e-13)
    np.testing.assert_allclose(w2[1], -TH["W"][1] * r2, rtol=1e-13)
    assert np.all(w2[[0, 3, 5, 6]] == 0.0)


def test_reacting_state_temperature_range():
    """The generator's blended state gives Newton temperatures in about
    300..2200 K (cold / hot endpoints) for the default tables."""
    xyz = np.random.default_rng(4).uniform(0, 0.01, (2000, 3))
    q = wl.reacting_state(xyz, n_cells=32)
    rho, u, v, w, e, Y = ot.primitives(q)
    T, it = ot.newton_temperature(e, Y, TH, 1000.0)
    assert np.all(it > 0)
    assert 250 < T.min() < 400 and 2000 < T.max() < 2300
